// Environment updates and the two-site effective Hamiltonian as grouped block GEMMs.
//
// Notation: L_w[a, a'] (bra a, ket a') is the left environment of MPO channel w at a cut,
// R_u[b, b'] the right one; W_p[w -> v] |s><s'| the MPO site tensors; theta[a, s1, s2, b]
// a two-site tensor.  The two-site local operator of the fit (Methods, Eq. (add_min)) is
//   theta_out[a s1 s2 b] = sum L_w[a a'] W_i[w v s1 s1'] W_{i+1}[v u s2 s2'] R_u[b b'] theta[a' s1' s2' b'].
// It is evaluated through the channels v of the middle cut:
//   Lop_v^{s1 s1'} = sum_w W_i[w v s1 s1'] L_w,   Rop_v^{s2 s2'} = sum_u W_{i+1}[v u s2 s2'] R_u,
//   T_v[a s1 s2' b'] = sum_{s1'} Lop_v^{s1 s1'} theta[s1' s2'],
//   theta_out[a s1 s2 b] = sum_v sum_{s2'} T_v[a s1 s2' b'] Rop_v^{s2 s2' T}[b' b].
// Single-source operators alias the environment (pass-through channels, new single
// operators); multi-source ones (complementary sums) are formed once as a real-coefficient
// GEMM over the channel index.  Consecutive middle channels with the same structure form
// "runs" whose blocks are stacked, so each block product is one batched GEMM over a run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "engine.h"

namespace tdmps {
namespace {

const cplx ONE{1.0, 0.0};

struct Run {
  int v0, n;
};

// channel-ordered W entries grouped by the "middle" channel
struct MixGroupKey {
  int pat, vcls;
  bool operator<(const MixGroupKey& o) const { return std::tie(pat, vcls) < std::tie(o.pat, o.vcls); }
};

struct MixRow {
  int v;
  std::vector<std::pair<int, double>> src;  // (source channel, coefficient)
};

// The environment-independent part of a premix: which channels of the middle cut alias an
// environment channel and which are combinations, the combination groups and their dense
// coefficient matrices (uploaded once).  It depends only on the operator's coefficients
// (its version), the site and the side, so it is cached per (stream, version, site, side).
struct SkelRef {
  int grp = 0, idx = 0;
  double coef = 0;
  bool mix = false;
};
struct SkelChan {
  std::vector<int> pat;
  std::vector<SkelRef> ref;
};
struct PremixSkel {
  struct Pend {
    int g, cw, wlo, ncol;
    size_t off;
  };
  std::vector<SkelChan> ch;
  std::vector<std::pair<Charge, int>> groups;
  std::vector<Pend> pend;
  std::shared_ptr<DevBuf> wmat;
};

std::shared_ptr<const PremixSkel> make_skeleton(Ctx* ctx, const MpoHost& W, int site, bool left) {
  const MpoCut& mc = W.cut[left ? site + 1 : site];
  const MpoCut& sc = W.cut[left ? site : site + 1];
  auto sk = std::make_shared<PremixSkel>();
  sk->ch.resize(mc.size());
  // per middle channel, per pattern: list of (source channel, coefficient)
  std::vector<std::map<int, std::vector<std::pair<int, double>>>> per(mc.size());
  for (const auto& e : W.W[site]) {
    int mid = left ? e.v : e.w;
    int src = left ? e.w : e.v;
    per[mid][e.s * 4 + e.sp].push_back({src, e.c});
  }
  std::map<MixGroupKey, std::vector<MixRow>> mix;
  for (int v = 0; v < mc.size(); ++v) {
    for (auto& kv : per[v]) {
      sk->ch[v].pat.push_back(kv.first);
      SkelRef r;
      if (kv.second.size() == 1) {
        int w = kv.second[0].first;
        r.grp = sc.cls_of[w];
        r.idx = w - sc.cls_start[r.grp];
        r.coef = kv.second[0].second;
      } else {
        r.mix = true;  // grp / idx filled below
        mix[{kv.first, mc.cls_of[v]}].push_back({v, kv.second});
      }
      sk->ch[v].ref.push_back(r);
    }
  }
  if (mix.empty()) return sk;
  // premix layout: one group per (pattern, middle class), coefficient matrices dense over the
  // used source range
  std::vector<cplx> wmat;
  int g = 0;
  for (auto& kv : mix) {
    int w0 = kv.second[0].src[0].first;
    int cw = sc.cls_of[w0];
    int lo = 1 << 30, hi = -1;
    for (auto& row : kv.second)
      for (auto& s : row.src) {
        TDMPS_REQUIRE(sc.cls_of[s.first] == cw, TDMPS_ERR_NUMERIC, "internal: premix sources differ in charge");
        lo = std::min(lo, s.first);
        hi = std::max(hi, s.first);
      }
    sk->groups.push_back({sc.cls_q[cw], (int)kv.second.size()});
    int ncol = hi - lo + 1;
    size_t off = wmat.size();
    wmat.resize(off + (size_t)kv.second.size() * ncol, cplx{0, 0});
    for (size_t r = 0; r < kv.second.size(); ++r) {
      for (auto& s : kv.second[r].src) wmat[off + r * ncol + (s.first - lo)].x += s.second;
      SkelChan& ch = sk->ch[kv.second[r].v];
      for (size_t k = 0; k < ch.pat.size(); ++k)
        if (ch.pat[k] == kv.first.pat) {
          ch.ref[k].grp = g;
          ch.ref[k].idx = (int)r;
          ch.ref[k].coef = 1.0;
        }
    }
    sk->pend.push_back({g, cw, lo - sc.cls_start[cw], ncol, off});
    ++g;
  }
  sk->wmat = std::make_shared<DevBuf>(wmat.size() * sizeof(cplx));
  dev_h2d(sk->wmat->p, wmat.data(), wmat.size() * sizeof(cplx), ctx->stream);
  return sk;
}

struct SkelKey {
  void* stream;
  uint64_t version;
  int site;
  bool left;
  bool operator<(const SkelKey& o) const {
    return std::tie(stream, version, site, left) < std::tie(o.stream, o.version, o.site, o.left);
  }
};
struct SkelEntry {
  std::shared_ptr<const PremixSkel> sk;
  size_t bytes;
  uint64_t stamp;
};
// Held through pointers that are never deleted: entries own device buffers, and a
// destructor at process exit would free them into the allocator's tables (another
// translation unit), which may already have been destroyed.
std::mutex& g_skel_mu = *new std::mutex;
std::map<SkelKey, SkelEntry>& g_skel = *new std::map<SkelKey, SkelEntry>;
uint64_t g_skel_clock = 0;
size_t g_skel_bytes = 0;
// Bounds of the cache: the dense coefficient matrices of one L = 24 operator take a few GB
// over all sites and both sides; a bound below the working set of a sweep would rebuild them
// at every site (LRU thrashing).
constexpr size_t SKEL_MAX_ENTRIES = 4096;
constexpr size_t SKEL_MAX_BYTES = (size_t)16 << 30;
uint64_t g_skel_built = 0;  // structures built so far (cache misses)

// The coefficient buffer is uploaded on, and only read on, the stream of the key, so the
// caching allocator's stream order covers its reuse after eviction.
std::shared_ptr<const PremixSkel> premix_skeleton(Ctx* ctx, const MpoHost& W, int site, bool left) {
  const SkelKey key{ctx->stream, W.version, site, left};
  std::lock_guard<std::mutex> lk(g_skel_mu);
  auto it = g_skel.find(key);
  if (it != g_skel.end()) {
    it->second.stamp = ++g_skel_clock;
    return it->second.sk;
  }
  auto sk = make_skeleton(ctx, W, site, left);
  ++g_skel_built;
  const size_t bytes = sk->wmat ? sk->wmat->bytes : 0;
  while (!g_skel.empty() && (g_skel.size() >= SKEL_MAX_ENTRIES || g_skel_bytes + bytes > SKEL_MAX_BYTES)) {
    auto oldest = g_skel.begin();
    for (auto e = g_skel.begin(); e != g_skel.end(); ++e)
      if (e->second.stamp < oldest->second.stamp) oldest = e;
    g_skel_bytes -= oldest->second.bytes;
    g_skel.erase(oldest);
  }
  g_skel.emplace(key, SkelEntry{sk, bytes, ++g_skel_clock});
  g_skel_bytes += bytes;
  return sk;
}

}  // namespace

double premix_structures_built() {
  std::lock_guard<std::mutex> lk(g_skel_mu);
  return (double)g_skel_built;
}

void premix_cache_forget(uint64_t version) {
  std::lock_guard<std::mutex> lk(g_skel_mu);
  for (auto it = g_skel.begin(); it != g_skel.end();) {
    if (it->first.version == version) {
      g_skel_bytes -= it->second.bytes;
      it = g_skel.erase(it);
    } else {
      ++it;
    }
  }
}

namespace {

// With ext != nullptr the premix products are appended to *ext (run by the caller) instead
// of being run here.
SideOps build_ops(Contractor& C, const Env& E, const MpoHost& W, int site, bool left, GemmPlan* ext = nullptr) {
  const double t0 = wall_seconds();
  struct Acc {
    Contractor& C;
    double t0;
    ~Acc() { C.t_mix += wall_seconds() - t0; }
  } acc_{C, t0};
  TDMPS_REQUIRE(E.cut == (left ? site : site + 1), TDMPS_ERR_ARG, "internal: premix environment cut");
  const auto sk = premix_skeleton(C.ctx, W, site, left);
  SideOps ops;
  ops.cut = left ? site + 1 : site;
  ops.env = &E;
  if ((int)W.plain_cls.size() > E.cut && !W.plain_cls[E.cut].empty()) ops.ref_cls = &W.plain_cls[E.cut];
  if (!sk->groups.empty()) {
    ops.mix.reset(new Blocks());
    ops.mix->layout(E.b.bra, E.b.ket, sk->groups);
    ops.mix->data = DevBuf(ops.mix->size * sizeof(cplx));
    ops.wmat = sk->wmat;
  }
  ops.ch.resize(sk->ch.size());
  for (size_t v = 0; v < sk->ch.size(); ++v) {
    const SkelChan& sc = sk->ch[v];
    ChanOps& co = ops.ch[v];
    co.pat = sc.pat;
    co.ref.resize(sc.ref.size());
    for (size_t k = 0; k < sc.ref.size(); ++k) {
      const SkelRef& r = sc.ref[k];
      co.ref[k] = OpRef{r.mix ? ops.mix.get() : &E.b, r.grp, r.idx, r.coef};
    }
  }
  if (sk->groups.empty()) return ops;
  // one real-coefficient GEMM over the source channels per group and ket sector (real-A
  // products: the coefficients are the real parts of the uploaded matrices)
  const cplx* dw = sk->wmat->c();
  GemmPlan local;
  GemmPlan& plan = ext ? *ext : local;
  TDMPS_REQUIRE(plan.real_a || plan.task_count() == 0, TDMPS_ERR_NUMERIC, "internal: premix plan with complex products");
  plan.real_a = true;
  const Blocks& eb = E.b;
  for (const auto& p : sk->pend) {
    const StackGroup& sg = ops.mix->grp[p.g];
    for (int ks = 0; ks < eb.ket.nsec(); ++ks) {
      if (sg.off[ks] < 0) continue;
      int bs = sg.bra_of[ks];
      int64_t blk = (int64_t)eb.bra.dim[bs] * eb.ket.dim[ks];
      const cplx* B = eb.stack(p.cw, ks);
      TDMPS_REQUIRE(B != nullptr, TDMPS_ERR_NUMERIC, "internal: premix source stack missing");
      plan.begin_task(ops.mix->stack(p.g, ks), 0, (int)blk, sg.n, (int)blk, 1, false);
      plan.add_seg(dw + p.off, 0, 0, p.ncol, OP_N, B + (int64_t)p.wlo * blk, 0, 0, (int)blk, OP_N, p.ncol, 1, ONE);
    }
  }
  if (!ext) {
    plan.run(C.ctx, TDMPS_FP64, C.batched);
    if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
    C.mix_flops += plan.flops;
  }
  return ops;
}

bool same_structure(const ChanOps& a, const ChanOps& b) {
  if (a.pat != b.pat) return false;
  for (size_t k = 0; k < a.pat.size(); ++k) {
    const OpRef &x = a.ref[k], &y = b.ref[k];
    if (x.src != y.src || x.grp != y.grp || x.idx + 1 != y.idx || x.coef != y.coef) return false;
  }
  return true;
}

// How pattern k continues from channel a to the next channel b: 1 = stacked (consecutive
// blocks of one stack, equal coefficient), 2 = shared (the same environment block for both,
// each with its own coefficient: a single source such as a pair on the site weighted by an
// integral), 0 = neither.
int pattern_step(const OpRef& x, const OpRef& y, const Blocks* env) {
  if (x.src != y.src || x.grp != y.grp) return 0;
  if (x.idx + 1 == y.idx && x.coef == y.coef) return 1;
  if (x.src == env && x.idx == y.idx) return 2;
  return 0;
}

// Maximal ranges of channels of one class of the middle cut whose operators, pattern by
// pattern, are either stacked over the range or one shared environment block with
// per-channel coefficients (pattern_step); shared[r][k] marks the latter for run r.
std::vector<Run> make_runs(const MpoCut& mc, const SideOps& ops, std::vector<std::vector<char>>& shared) {
  std::vector<Run> runs;
  shared.clear();
  const Blocks* env = &ops.env->b;
  const int n = mc.size();
  int v = 0;
  while (v < n) {
    const ChanOps& c0 = ops.ch[v];
    std::vector<char> kind(c0.pat.size(), 0);
    int e = v + 1;
    while (e < n && mc.cls_of[e] == mc.cls_of[v] && ops.ch[e].pat == c0.pat) {
      bool ok = true;
      for (size_t k = 0; k < c0.pat.size() && ok; ++k) {
        const int step = pattern_step(ops.ch[e - 1].ref[k], ops.ch[e].ref[k], env);
        if (step == 0 || (kind[k] != 0 && kind[k] != step)) ok = false;
      }
      if (!ok) break;
      for (size_t k = 0; k < c0.pat.size(); ++k) kind[k] = (char)pattern_step(ops.ch[e - 1].ref[k], ops.ch[e].ref[k], env);
      ++e;
    }
    for (auto& x : kind) x = x == 2;
    runs.push_back({v, e - v});
    shared.push_back(std::move(kind));
    v = e;
  }
  return runs;
}

inline cplx cmul(cplx a, cplx b) { return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

}  // namespace

SideOps premix_left(Contractor& C, const Env& L, const MpoHost& W, int site) {
  TDMPS_REQUIRE(L.cut == site, TDMPS_ERR_ARG, "internal: left environment cut");
  return build_ops(C, L, W, site, true);
}

SideOps premix_right(Contractor& C, const Env& R, const MpoHost& W, int site) {
  TDMPS_REQUIRE(R.cut == site + 1, TDMPS_ERR_ARG, "internal: right environment cut");
  return build_ops(C, R, W, site, false);
}

Env env_left_boundary(Ctx* ctx, const Bond& bra0, const Bond& ket0) {
  Env E;
  E.cut = 0;
  E.b.layout(bra0, ket0, {{Charge(0, 0), 1}});
  E.b.data = DevBuf(sizeof(cplx));
  cplx one{1.0, 0.0};
  dev_h2d(E.b.data.p, &one, sizeof(cplx), ctx->stream);
  return E;
}

Env env_right_boundary(Ctx* ctx, const Bond& braL, const Bond& ketL, int L) {
  TDMPS_REQUIRE(braL.q[0] == ketL.q[0], TDMPS_ERR_SECTOR, "bra and ket have different total charge");
  Env E;
  E.cut = L;
  E.b.layout(braL, ketL, {{Charge(0, 0), 1}});
  E.b.data = DevBuf(sizeof(cplx));
  cplx one{1.0, 0.0};
  dev_h2d(E.b.data.p, &one, sizeof(cplx), ctx->stream);
  return E;
}

static std::vector<std::pair<Charge, int>> cut_groups(const MpoCut& c) {
  std::vector<std::pair<Charge, int>> g;
  for (size_t k = 0; k < c.cls_q.size(); ++k) g.push_back({c.cls_q[k], c.cls_count[k]});
  return g;
}

// Plans a left environment update: the T stage into p1, the contraction with the bra into p2
// (run p1 before p2); T holds the intermediate and must outlive both runs.
void env_left_plan(const SideOps& ops, const cplx* bra_site, const SiteLayout& bl, const Bond& bra_l,
                   const Bond& bra_r, const cplx* ket_site, const SiteLayout& kl, const Bond& ket_l,
                   const Bond& ket_r, const MpoHost& W, Ctx* ctx, GemmPlan& p1, GemmPlan& p1b, GemmPlan& p2, DevBuf& T,
                   Env& out) {
  const MpoCut& mc = W.cut[ops.cut];
  out.cut = ops.cut;
  out.b.layout(bra_r, ket_r, cut_groups(mc));
  out.b.data = DevBuf(out.b.size * sizeof(cplx));
  if (out.b.size) dev_zero(out.b.data.p, out.b.data.bytes, ctx->stream);
  std::vector<std::vector<char>> shared;
  auto runs = make_runs(mc, ops, shared);
  // T_v[s, sig, t'] = sum_{sig'} Lop_v^{sig sig'}[s, s'] A_ket[s', sig', t']
  struct TKey {
    int r, s, sig, tk;
  };
  // the second stage below visits the (r, tk, s, sig) keys in the order they are created here
  std::vector<TKey> tkeys;
  std::vector<int64_t> toff;
  int64_t tsize = 0;
  for (int r = 0; r < (int)runs.size(); ++r) {
    int v0 = runs[r].v0;
    int g = mc.cls_of[v0];
    const StackGroup& og = out.b.grp[g];
    for (int tk = 0; tk < ket_r.nsec(); ++tk) {
      int tb = og.bra_of[tk];
      if (tb < 0) continue;
      for (int s = 0; s < bra_l.nsec(); ++s)
        for (int sig = 0; sig < 4; ++sig) {
          if (bl.rs[s][sig] != tb) continue;
          tkeys.push_back({r, s, sig, tk});
          toff.push_back(tsize);
          tsize += (int64_t)runs[r].n * bra_l.dim[s] * ket_r.dim[tk];
        }
    }
  }
  T = DevBuf(tsize * sizeof(cplx));
  std::vector<char> tnonzero(tkeys.size(), 0);
  for (size_t t = 0; t < tkeys.size(); ++t) {
    const TKey& K = tkeys[t];
    const Run& run = runs[K.r];
    const ChanOps& co = ops.ch[run.v0];
    int Ds = bra_l.dim[K.s], Dt = ket_r.dim[K.tk];
    bool started = false, any_shared = false;
    for (int pass = 0; pass < 2; ++pass)  // stacked patterns over the run, then shared ones per channel
      for (int j = 0; j < (pass == 0 ? 1 : run.n); ++j) {
        bool opened = false;
        for (size_t k = 0; k < co.pat.size(); ++k) {
          int sig = co.pat[k] >> 2, sigp = co.pat[k] & 3;
          if (sig != K.sig) continue;
          if ((run.n > 1 && shared[K.r][k]) != (pass == 1)) continue;
          const OpRef& ref = co.ref[k];
          const StackGroup& sg = ref.src->grp[ref.grp];
          int sp = sg.ket_of[K.s];
          if (sp < 0) continue;
          if (kl.rs[sp][sigp] != K.tk) continue;
          int Dsp = ket_l.dim[sp];
          const cplx* A = ref.src->stack(ref.grp, sp) + (int64_t)ref.idx * Ds * Dsp;
          const cplx* B = ket_site + kl.panel_off[sp] + kl.col[sp][sigp];
          if (pass == 0) {
            if (!started) {
              p1.begin_task(T.c() + toff[t], 0, Dt, run.n * Ds, Dt, 1, false);
              started = true;
            }
            p1.add_seg(A, 0, 0, Dsp, OP_N, B, 0, 0, kl.width[sp], OP_N, Dsp, 1, cplx{ref.coef, 0.0});
          } else {
            if (!opened) {
              p1b.begin_task(T.c() + toff[t] + (int64_t)j * Ds * Dt, 0, Dt, Ds, Dt, 1, started);
              opened = true;
              any_shared = true;
            }
            p1b.add_seg(A, 0, 0, Dsp, OP_N, B, 0, 0, kl.width[sp], OP_N, Dsp, 1,
                        cplx{ops.ch[run.v0 + j].ref[k].coef, 0.0});
          }
        }
      }
    tnonzero[t] = started || any_shared;
  }
  // L'_v[t, t'] = sum_{s, sig} conj(C[s, sig, t])^T T_v[s, sig, t']
  size_t cursor = 0;
  for (int r = 0; r < (int)runs.size(); ++r) {
    int v0 = runs[r].v0;
    int g = mc.cls_of[v0];
    int j0 = v0 - mc.cls_start[g];
    const StackGroup& og = out.b.grp[g];
    for (int tk = 0; tk < ket_r.nsec(); ++tk) {
      int tb = og.bra_of[tk];
      if (tb < 0) continue;
      int Dt = bra_r.dim[tb], Dtk = ket_r.dim[tk];
      bool started = false;
      for (int s = 0; s < bra_l.nsec(); ++s)
        for (int sig = 0; sig < 4; ++sig) {
          if (bl.rs[s][sig] != tb) continue;
          const size_t t = cursor++;
          TDMPS_REQUIRE(t < tkeys.size() && tkeys[t].r == r && tkeys[t].s == s && tkeys[t].sig == sig &&
                            tkeys[t].tk == tk,
                        TDMPS_ERR_NUMERIC, "internal: T key order");
          if (!tnonzero[t]) continue;
          int Ds = bra_l.dim[s];
          if (!started) {
            p2.begin_task(out.b.stack(g, tk) + (int64_t)j0 * Dt * Dtk, (int64_t)Dt * Dtk, Dtk, Dt, Dtk, runs[r].n,
                          true);
            started = true;
          }
          const cplx* A = bra_site + bl.panel_off[s] + bl.col[s][sig];
          p2.add_seg(A, 0, 0, bl.width[s], OP_C, T.c() + toff[t], (int64_t)Ds * Dtk, 0, Dtk, OP_N, Ds, 1, ONE);
        }
    }
  }
}

Env env_left_update(Contractor& C, const SideOps& ops, const Mps*, const cplx* bra_site, const SiteLayout& bl,
                    const Bond& bra_l, const Bond& bra_r, const cplx* ket_site, const SiteLayout& kl,
                    const Bond& ket_l, const Bond& ket_r, const MpoHost& W) {
  const double t0 = wall_seconds();
  GemmPlan p1, p1b, p2;
  DevBuf T;
  Env out;
  env_left_plan(ops, bra_site, bl, bra_l, bra_r, ket_site, kl, ket_l, ket_r, W, C.ctx, p1, p1b, p2, T, out);
  const double tb = wall_seconds();
  p1.run(C.ctx, C.precision, C.batched);
  p1b.run(C.ctx, C.precision, C.batched);
  p2.run(C.ctx, C.precision, C.batched);
  if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
  C.t_plan += (tb - t0) + p1.host_s + p1b.host_s + p2.host_s;
  C.env_flops += p1.flops + p1b.flops + p2.flops;
  C.t_env += wall_seconds() - t0;
  C.n_env += 1;
  return out;
}

Env env_right_update(Contractor& C, const SideOps& ops, const cplx* bra_site, const SiteLayout& bl, const Bond& bra_l,
                     const Bond& bra_r, const cplx* ket_site, const SiteLayout& kl, const Bond& ket_l,
                     const Bond& ket_r, const MpoHost& W) {
  const double t0 = wall_seconds();
  const MpoCut& mc = W.cut[ops.cut];
  Env out;
  out.cut = ops.cut;
  out.b.layout(bra_l, ket_l, cut_groups(mc));
  out.b.data = DevBuf(out.b.size * sizeof(cplx));
  if (out.b.size) dev_zero(out.b.data.p, out.b.data.bytes, C.ctx->stream);
  std::vector<std::vector<char>> shared;
  auto runs = make_runs(mc, ops, shared);
  // T_v[s', sig, t] = sum_{sig'} A_ket[s', sig', t'] Rop_v^{sig sig'}[t, t']^T
  struct TKey {
    int r, sk, sig, tb;
  };
  // the second stage below visits the (r, sk, sig) keys in the order they are created here
  std::vector<TKey> tkeys;
  std::vector<int64_t> toff;
  int64_t tsize = 0;
  for (int r = 0; r < (int)runs.size(); ++r) {
    int g = mc.cls_of[runs[r].v0];
    const StackGroup& og = out.b.grp[g];
    for (int sk = 0; sk < ket_l.nsec(); ++sk) {
      int sb = og.bra_of[sk];
      if (sb < 0) continue;
      for (int sig = 0; sig < 4; ++sig) {
        int tb = bl.rs[sb][sig];
        if (tb < 0) continue;
        tkeys.push_back({r, sk, sig, tb});
        toff.push_back(tsize);
        tsize += (int64_t)runs[r].n * ket_l.dim[sk] * bra_r.dim[tb];
      }
    }
  }
  DevBuf T(tsize * sizeof(cplx));
  GemmPlan p1, p1b;
  std::vector<char> tnonzero(tkeys.size(), 0);
  for (size_t t = 0; t < tkeys.size(); ++t) {
    const TKey& K = tkeys[t];
    const Run& run = runs[K.r];
    const ChanOps& co = ops.ch[run.v0];
    int Dsk = ket_l.dim[K.sk], Dt = bra_r.dim[K.tb];
    bool started = false, any_shared = false;
    for (int pass = 0; pass < 2; ++pass)  // stacked patterns batched over the run, then shared ones per channel
      for (int j = 0; j < (pass == 0 ? 1 : run.n); ++j) {
        bool opened = false;
        for (size_t k = 0; k < co.pat.size(); ++k) {
          int sig = co.pat[k] >> 2, sigp = co.pat[k] & 3;
          if (sig != K.sig) continue;
          if ((run.n > 1 && shared[K.r][k]) != (pass == 1)) continue;
          const OpRef& ref = co.ref[k];
          const StackGroup& sg = ref.src->grp[ref.grp];
          int tk = sg.ket_of[K.tb];
          if (tk < 0) continue;
          if (kl.rs[K.sk][sigp] != tk) continue;
          int Dtk = ket_r.dim[tk];
          const cplx* A = ket_site + kl.panel_off[K.sk] + kl.col[K.sk][sigp];
          const cplx* B = ref.src->stack(ref.grp, tk) + (int64_t)ref.idx * Dt * Dtk;
          if (pass == 0) {
            if (!started) {
              p1.begin_task(T.c() + toff[t], (int64_t)Dsk * Dt, Dt, Dsk, Dt, run.n, false);
              started = true;
            }
            p1.add_seg(A, 0, 0, kl.width[K.sk], OP_N, B, (int64_t)Dt * Dtk, 0, Dtk, OP_T, Dtk, 1, cplx{ref.coef, 0.0});
          } else {
            if (!opened) {
              p1b.begin_task(T.c() + toff[t] + (int64_t)j * Dsk * Dt, 0, Dt, Dsk, Dt, 1, started);
              opened = true;
              any_shared = true;
            }
            p1b.add_seg(A, 0, 0, kl.width[K.sk], OP_N, B, 0, 0, Dtk, OP_T, Dtk, 1,
                        cplx{ops.ch[run.v0 + j].ref[k].coef, 0.0});
          }
        }
      }
    tnonzero[t] = started || any_shared;
  }
  const double tb1 = wall_seconds();
  p1.run(C.ctx, C.precision, C.batched);
  p1b.run(C.ctx, C.precision, C.batched);
  const double te1 = wall_seconds();
  // R'_v[s, s'] = sum_{sig, t} conj(C[s, sig, t]) T_v[s', sig, t]^T
  GemmPlan p2;
  size_t cursor = 0;
  for (int r = 0; r < (int)runs.size(); ++r) {
    int v0 = runs[r].v0;
    int g = mc.cls_of[v0];
    int j0 = v0 - mc.cls_start[g];
    const StackGroup& og = out.b.grp[g];
    for (int sk = 0; sk < ket_l.nsec(); ++sk) {
      int sb = og.bra_of[sk];
      if (sb < 0) continue;
      int Ds = bra_l.dim[sb], Dsk = ket_l.dim[sk];
      bool started = false;
      for (int sig = 0; sig < 4; ++sig) {
        int tb = bl.rs[sb][sig];
        if (tb < 0) continue;
        const size_t t = cursor++;
        TDMPS_REQUIRE(t < tkeys.size() && tkeys[t].r == r && tkeys[t].sk == sk && tkeys[t].sig == sig &&
                          tkeys[t].tb == tb,
                      TDMPS_ERR_NUMERIC, "internal: T key order");
        if (!tnonzero[t]) continue;
        int Dt = bra_r.dim[tb];
        if (!started) {
          p2.begin_task(out.b.stack(g, sk) + (int64_t)j0 * Ds * Dsk, (int64_t)Ds * Dsk, Dsk, Ds, Dsk, runs[r].n, true);
          started = true;
        }
        const cplx* A = bra_site + bl.panel_off[sb] + bl.col[sb][sig];
        p2.add_seg(A, 0, 0, bl.width[sb], OP_J, T.c() + toff[t], (int64_t)Dsk * Dt, 0, Dt, OP_T, Dt, 1, ONE);
      }
    }
  }
  const double tb2 = wall_seconds();
  p2.run(C.ctx, C.precision, C.batched);
  if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
  C.t_plan += (tb1 - t0) + (tb2 - te1) + p1.host_s + p1b.host_s + p2.host_s;
  C.env_flops += p1.flops + p1b.flops + p2.flops;
  C.t_env += wall_seconds() - t0;
  C.n_env += 1;
  return out;
}

void HeffPlan::launch(Ctx* ctx, int precision, bool batched) {
  if (!accumulate && out_size) dev_zero(out, out_size * sizeof(cplx), ctx->stream);
  if (ops32) launch_to_f32(theta_in, theta32.p, theta_size, ctx->stream);
  p1.launch(ctx, precision, batched);
  p1b.launch(ctx, precision, batched);
  if (!share_host.empty()) {
    TDMPS_REQUIRE(p1b.dextra != nullptr, TDMPS_ERR_NUMERIC, "internal: share tasks not uploaded");
    launch_share((const ShareTask*)p1b.dextra, (const double*)(p1b.dextra + share_coef_off), (int)share_host.size(),
                 share_max_blk, ctx->stream);
  }
  p2.launch(ctx, precision, batched);
}

void heff_apply(Contractor& C, const SideOps& lops, const SideOps& rops, const cplx* theta_in, const TwoLayout& kl,
                const Bond& ket_l, const Bond& ket_r, cplx* theta_out, const TwoLayout& bl, const Bond& bra_l,
                const Bond& bra_r, cplx alpha, bool accumulate, double* alg_flops) {
  const double t0 = wall_seconds();
  auto plan = heff_plan(C, lops, rops, theta_in, kl, ket_l, ket_r, theta_out, bl, bra_l, bra_r, alpha, accumulate);
  C.t_plan += wall_seconds() - t0;
  plan->launch(C.ctx, C.precision, C.batched);
  if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
  C.heff_flops += plan->p1.flops + plan->p1b.flops + plan->p2.flops;
  if (alg_flops) *alg_flops = plan->alg_flops;
  C.t_heff += wall_seconds() - t0;
  C.n_heff += 1;
}

std::unique_ptr<HeffPlan> heff_plan(Contractor& C, const SideOps& lops, const SideOps& rops, const cplx* theta_in,
                                    const TwoLayout& kl, const Bond& ket_l, const Bond& ket_r, cplx* theta_out,
                                    const TwoLayout& bl, const Bond& bra_l, const Bond& bra_r, cplx alpha,
                                    bool accumulate, Arena* arena) {
  TDMPS_REQUIRE(lops.cut == rops.cut, TDMPS_ERR_ARG, "internal: middle cuts differ");
  auto plan = std::make_unique<HeffPlan>();
  plan->out = theta_out;
  plan->out_size = bl.size;
  plan->accumulate = accumulate;
  const int nmid = (int)lops.ch.size();
  // Mixed precisions: operands and the T intermediate in FP32 storage.  Every environment
  // operator buffer referenced by the two sides gets an FP32 copy now; theta_in is converted by
  // every launch (its contents change between launches).  Pointers into an FP32 copy keep the
  // element offsets of the FP64 buffer.
  const bool s32 = C.precision != TDMPS_FP64 && C.ctx->mixed_storage;
  plan->ops32 = s32;
  std::vector<std::pair<const Blocks*, const void*>> shadow_of;
  auto f32_at = [](const void* base, int64_t off) { return (const cplx*)((const char*)base + off * 8); };
  auto to32 = [&](const Blocks* src, const cplx* p) -> const cplx* {
    for (const auto& so : shadow_of)
      if (so.first == src) return f32_at(so.second, p - src->data.c());
    throw Error(TDMPS_ERR_NUMERIC, "internal: operand buffer without an FP32 copy");
  };
  if (s32) {
    auto add = [&](const SideOps& o) {
      for (const auto& ch : o.ch)
        for (const auto& ref : ch.ref) {
          bool seen = false;
          for (const auto& so : shadow_of) seen |= so.first == ref.src;
          if (seen || ref.src->size == 0) continue;
          plan->shadows.push_back(arena ? arena->view(ref.src->size * 8) : DevBuf(ref.src->size * 8));
          launch_to_f32(ref.src->data.c(), plan->shadows.back().p, ref.src->size, C.ctx->stream);
          shadow_of.push_back({ref.src, plan->shadows.back().p});
        }
    };
    add(lops);
    add(rops);
    plan->theta_in = theta_in;
    plan->theta_size = kl.size;
    plan->theta32 = arena ? arena->view(std::max<int64_t>(kl.size, 1) * 8) : DevBuf(std::max<int64_t>(kl.size, 1) * 8);
  }
  const int64_t esz = s32 ? 8 : (int64_t)sizeof(cplx);  // bytes per element of T
  // Runs over the middle cut: identical structure on the right; on the left every pattern
  // either stacked over the run or shared by all of its channels (shared[r][k]).  Shared
  // patterns are computed per channel in a stage of their own (p1b below), the rest as one
  // product over the whole run.
  std::vector<Run> runs;
  std::vector<std::vector<char>> shared;
  {
    const Blocks* lenv = &lops.env->b;
    int v = 0;
    while (v < nmid) {
      const ChanOps& c0 = lops.ch[v];
      std::vector<char> kind(c0.pat.size(), 0);
      int e = v + 1;
      while (e < nmid && lops.ch[e].pat == c0.pat && same_structure(rops.ch[e - 1], rops.ch[e])) {
        bool ok = true;
        for (size_t k = 0; k < c0.pat.size() && ok; ++k) {
          const int step = pattern_step(lops.ch[e - 1].ref[k], lops.ch[e].ref[k], lenv);
          if (step == 0 || (kind[k] != 0 && kind[k] != step)) ok = false;
        }
        if (!ok) break;
        for (size_t k = 0; k < c0.pat.size(); ++k) kind[k] = (char)pattern_step(lops.ch[e - 1].ref[k], lops.ch[e].ref[k], lenv);
        ++e;
      }
      for (auto& x : kind) x = x == 2;
      runs.push_back({v, e - v});
      shared.push_back(std::move(kind));
      v = e;
    }
  }
  // T is stored per row block (run r, bra sector s, s1): rows (channel of the run, a), columns
  // (s2', b') for the s2' needed by the final stage.  By charge conservation the ket sector of
  // b' depends only on (s, s1, s2') and the run's channel charge, so every left pattern
  // (s1, s1') of the run contributes to the whole row block with one product against the
  // contiguous theta columns (s1', s2' = lo..hi) of its ket sector.
  const int nbs = bra_l.nsec();
  struct Row {
    int r, s, s1, mask = 0;
    int tk[4] = {-1, -1, -1, -1};
    int lo = 4, hi = -1, width = 0;
    int coff[4] = {0, 0, 0, 0};
    int64_t off = -1;
  };
  std::vector<int> row_of(runs.size() * (size_t)nbs * 4, -1);
  std::vector<Row> rows;
  struct FSeg {
    int row, s2p;
    const OpRef* ref;
  };
  std::vector<std::vector<FSeg>> fsegs;  // per output block
  struct OBlk {
    int s, sig, tb;
  };
  std::vector<OBlk> oblk;
  for (int s = 0; s < nbs; ++s)
    for (int sig = 0; sig < 16; ++sig) {
      int tb = bl.rs[s][sig];
      if (tb < 0) continue;
      oblk.push_back({s, sig, tb});
    }
  fsegs.resize(oblk.size());
  for (size_t ob = 0; ob < oblk.size(); ++ob) {
    int s = oblk[ob].s, s1 = oblk[ob].sig >> 2, s2 = oblk[ob].sig & 3, tb = oblk[ob].tb;
    for (int r = 0; r < (int)runs.size(); ++r) {
      const ChanOps& ro = rops.ch[runs[r].v0];
      for (size_t k = 0; k < ro.pat.size(); ++k) {
        if ((ro.pat[k] >> 2) != s2) continue;
        int s2p = ro.pat[k] & 3;
        const OpRef& ref = ro.ref[k];
        int tk = ref.src->grp[ref.grp].ket_of[tb];
        if (tk < 0) continue;
        int& id = row_of[((size_t)r * nbs + s) * 4 + s1];
        if (id < 0) {
          id = (int)rows.size();
          Row nr;
          nr.r = r;
          nr.s = s;
          nr.s1 = s1;
          rows.push_back(nr);
        }
        Row& row = rows[id];
        TDMPS_REQUIRE(row.tk[s2p] < 0 || row.tk[s2p] == tk, TDMPS_ERR_NUMERIC, "internal: T column sector");
        row.tk[s2p] = tk;
        row.mask |= 1 << s2p;
        fsegs[ob].push_back({id, s2p, &ref});
      }
    }
  }
  // T stage
  int64_t tsize = 0, xsize = 0;
  GemmPlan& p1 = plan->p1;
  GemmPlan& p1b = plan->p1b;
  std::vector<size_t> row_task(rows.size(), (size_t)-1);
  struct SharedRow {
    size_t row, share;
    int64_t xoff;
    std::vector<size_t> xtask;
  };
  std::vector<SharedRow> shared_rows;
  for (size_t ri = 0; ri < rows.size(); ++ri) {
    Row& R = rows[ri];
    const Run& run = runs[R.r];
    const ChanOps& lo = lops.ch[run.v0];
    const int Ds = bra_l.dim[R.s];
    // contributing patterns of this row block and its columns: every s2' between the lowest
    // and highest needed one whose ket sector exists, taken from the first pattern
    std::vector<int> pats;
    for (size_t k = 0; k < lo.pat.size(); ++k) {
      if ((lo.pat[k] >> 2) != R.s1) continue;
      const OpRef& ref = lo.ref[k];
      if (ref.src->grp[ref.grp].ket_of[R.s] < 0) continue;
      pats.push_back((int)k);
    }
    if (pats.empty()) continue;
    {
      const OpRef& ref = lo.ref[pats[0]];
      const int sk = ref.src->grp[ref.grp].ket_of[R.s];
      const int s1p = lo.pat[pats[0]] & 3;
      for (int q = 0; q < 4; ++q)
        if (R.mask >> q & 1) {
          R.lo = std::min(R.lo, q);
          R.hi = std::max(R.hi, q);
        }
      for (int q = R.lo; q <= R.hi; ++q) {
        const int tk = kl.rs[sk][s1p * 4 + q];
        TDMPS_REQUIRE(R.tk[q] < 0 || R.tk[q] == tk, TDMPS_ERR_NUMERIC, "internal: theta column sector");
        R.tk[q] = tk;
        R.coff[q] = R.width;
        if (tk >= 0) R.width += ket_r.dim[tk];
      }
    }
    if (R.width == 0) continue;
    R.off = tsize;
    tsize += (int64_t)run.n * Ds * R.width;
    // operands of pattern k: the ket-sector block of the left operator and the theta columns
    auto operands = [&](int k, const cplx*& A, const cplx*& B, int& Dsk) {
      const OpRef& ref = lo.ref[k];
      const int sk = ref.src->grp[ref.grp].ket_of[R.s];
      const int s1p = lo.pat[k] & 3;
      int first = -1;
      for (int q = R.lo; q <= R.hi; ++q) {
        const int tk = kl.rs[sk][s1p * 4 + q];
        TDMPS_REQUIRE(tk == R.tk[q], TDMPS_ERR_NUMERIC, "internal: theta column sector");
        if (tk >= 0 && first < 0) first = q;
      }
      Dsk = ket_l.dim[sk];
      A = ref.src->stack(ref.grp, sk) + (int64_t)ref.idx * Ds * Dsk;
      const int64_t boff = kl.panel_off[sk] + kl.col[sk][s1p * 4 + first];
      B = theta_in + boff;
      if (s32) {
        A = to32(ref.src, A);
        B = f32_at(plan->theta32.p, boff);
      }
      return sk;
    };
    // stacked patterns: one product over all channels of the run
    bool main_task = false;
    for (int k : pats) {
      if (run.n > 1 && shared[R.r][k]) continue;
      const cplx *A, *B;
      int Dsk;
      const int sk = operands(k, A, B, Dsk);
      if (!main_task) {
        row_task[ri] = p1.tasks.size();
        p1.begin_task(nullptr, 0, R.width, run.n * Ds, R.width, 1, false);
        if (s32) p1.tasks.back().flags |= GEMM_OUT32;
        main_task = true;
      }
      p1.add_seg(A, 0, 0, Dsk, OP_N, B, 0, 0, kl.width[sk], OP_N, Dsk, 1, cplx{lo.ref[k].coef, 0.0});
    }
    // Shared patterns: the same block for every channel of the run, each channel with its own
    // coefficient.  Their products X_q = A_q B_q are formed once per row block (p1b), then
    // added into every channel's rows, T_j += sum_q c_jq X_q, by one elementwise pass (after
    // the stacked products of p1, which write the row block first).
    if (run.n > 1) {
      std::vector<int> sh;
      for (int k : pats)
        if (shared[R.r][k]) sh.push_back(k);
      TDMPS_REQUIRE((int)sh.size() <= SHARE_MAXQ, TDMPS_ERR_NUMERIC, "internal: too many shared patterns");
      if (!sh.empty()) {
        const int nq = (int)sh.size();
        const int64_t blk = (int64_t)Ds * R.width;
        SharedRow sr;
        sr.row = ri;
        sr.xoff = xsize;
        xsize += nq * blk;
        for (int q = 0; q < nq; ++q) {
          const cplx *A, *B;
          int Dsk;
          const int sk = operands(sh[q], A, B, Dsk);
          sr.xtask.push_back(p1b.tasks.size());
          p1b.begin_task(nullptr, 0, R.width, Ds, R.width, 1, false);
          p1b.add_seg(A, 0, 0, Dsk, OP_N, B, 0, 0, kl.width[sk], OP_N, Dsk, 1, cplx{1.0, 0.0});
        }
        const size_t coff = plan->coef_host.size();
        for (int j = 0; j < run.n; ++j)
          for (int q = 0; q < nq; ++q) plan->coef_host.push_back(lops.ch[run.v0 + j].ref[sh[q]].coef);
        ShareTask st{};
        st.coff = (int64_t)coff;
        st.blk = blk;
        st.nrun = run.n;
        st.nq = nq;
        st.accum = main_task ? 1 : 0;
        st.out32 = s32 ? 1 : 0;
        sr.share = plan->share_host.size();
        plan->share_host.push_back(st);
        plan->share_max_blk = std::max(plan->share_max_blk, blk);
        shared_rows.push_back(sr);
      }
    }
  }
  plan->T = arena ? arena->view(tsize * esz) : DevBuf(tsize * esz);
  // element off of T (FP64 or FP32 complex)
  auto t_at = [&](int64_t off) { return (cplx*)((char*)plan->T.p + off * esz); };
  for (size_t ri = 0; ri < rows.size(); ++ri)
    if (row_task[ri] != (size_t)-1) p1.tasks[row_task[ri]].C = t_at(rows[ri].off);
  if (!shared_rows.empty()) {
    // the shared products get a buffer of their own: keeping T at the size of its rows keeps
    // the caching allocator's reuse of the large T buffers from bond to bond
    plan->X = arena ? arena->view(xsize * sizeof(cplx)) : DevBuf(xsize * sizeof(cplx));
    cplx* Xb = plan->X.c();
    for (const auto& sr : shared_rows) {
      const Row& R = rows[sr.row];
      const int64_t blk = (int64_t)bra_l.dim[R.s] * R.width;
      for (size_t q = 0; q < sr.xtask.size(); ++q) p1b.tasks[sr.xtask[q]].C = Xb + sr.xoff + (int64_t)q * blk;
      ShareTask& st = plan->share_host[sr.share];
      st.T = t_at(R.off);
      st.X = Xb + sr.xoff;
    }
    // the share tasks and their coefficients travel with p1b's task tables
    const size_t tb = plan->share_host.size() * sizeof(ShareTask);
    plan->share_coef_off = (tb + 255) & ~(size_t)255;
    p1b.extra.assign(plan->share_coef_off + plan->coef_host.size() * sizeof(double), 0);
    std::memcpy(p1b.extra.data(), plan->share_host.data(), tb);
    std::memcpy(p1b.extra.data() + plan->share_coef_off, plan->coef_host.data(), plan->coef_host.size() * sizeof(double));
  }
  // final stage
  GemmPlan& p2 = plan->p2;
  for (size_t ob = 0; ob < oblk.size(); ++ob) {
    int s = oblk[ob].s, sig = oblk[ob].sig, tb = oblk[ob].tb;
    int Ds = bra_l.dim[s], Dt = bra_r.dim[tb];
    bool started = false;
    for (auto& fs : fsegs[ob]) {
      const Row& R = rows[fs.row];
      if (R.off < 0) continue;
      const Run& run = runs[R.r];
      const int tk = R.tk[fs.s2p];
      const int Dtk = ket_r.dim[tk];
      if (!started) {
        p2.begin_task(theta_out + bl.panel_off[s] + bl.col[s][sig], 0, bl.width[s], Ds, Dt, 1, true);
        started = true;
      }
      const OpRef& ref = *fs.ref;
      const cplx* A = t_at(R.off + R.coff[fs.s2p]);
      const cplx* B = ref.src->stack(ref.grp, tk) + (int64_t)ref.idx * Dt * Dtk;
      if (s32) B = to32(ref.src, B);
      p2.add_seg(A, 0, (int64_t)Ds * R.width, R.width, OP_N, B, 0, (int64_t)Dt * Dtk, Dtk, OP_T, Dtk, run.n,
                 cmul(cplx{ref.coef, 0.0}, alpha));
    }
  }
  double alg = 0;
  // algorithmic count in the plain order (L theta) -> W -> (. R): every channel of the outer
  // cuts against every compatible block, with the channels of the plain operator rule (the
  // smallest operator; the routing of pair channels changes the executed work, not this count)
  {
    auto classes = [](const SideOps& o) {
      if (o.ref_cls) return *o.ref_cls;
      std::vector<std::pair<Charge, int>> c;
      for (const auto& g : o.env->b.grp) c.push_back({g.q, g.n});
      return c;
    };
    for (const auto& g : classes(lops))
      for (int sk = 0; sk < ket_l.nsec(); ++sk) {
        const int sb = bra_l.find(ket_l.q[sk] + g.first);
        if (sb < 0) continue;
        for (int sig = 0; sig < 16; ++sig) {
          int tk = kl.rs[sk][sig];
          if (tk < 0) continue;
          alg += 8.0 * g.second * bra_l.dim[sb] * (double)ket_l.dim[sk] * ket_r.dim[tk];
        }
      }
    for (const auto& g : classes(rops))
      for (int s = 0; s < bra_l.nsec(); ++s)
        for (int sig = 0; sig < 16; ++sig) {
          int tb = bl.rs[s][sig];
          if (tb < 0) continue;
          const int tk = ket_r.find(bra_r.q[tb] - g.first);
          if (tk < 0) continue;
          alg += 8.0 * g.second * bra_l.dim[s] * (double)bra_r.dim[tb] * ket_r.dim[tk];
        }
    plan->alg_flops = alg;
  }
  p1.arena = p1b.arena = p2.arena = arena;
  p1.ops32 = p1b.ops32 = p2.ops32 = s32;
  p1.finalize(C.ctx, C.precision);
  p1b.finalize(C.ctx, C.precision);
  p2.finalize(C.ctx, C.precision);
  return plan;
}

void form_theta(Contractor& C, const Mps* m, int i, cplx* theta, const TwoLayout& tl) {
  const SiteLayout& a = m->lay[i];
  const SiteLayout& b = m->lay[i + 1];
  const Bond& l = m->bond[i];
  if (tl.size) dev_zero(theta, tl.size * sizeof(cplx), C.ctx->stream);
  GemmPlan p;
  for (int s = 0; s < l.nsec(); ++s)
    for (int s1 = 0; s1 < 4; ++s1) {
      int mid = a.rs[s][s1];
      if (mid < 0) continue;
      for (int s2 = 0; s2 < 4; ++s2) {
        int t = b.rs[mid][s2];
        if (t < 0) continue;
        int sig = s1 * 4 + s2;
        TDMPS_REQUIRE(tl.rs[s][sig] == t, TDMPS_ERR_NUMERIC, "internal: two-site layout mismatch");
        p.begin_task(theta + tl.panel_off[s] + tl.col[s][sig], 0, tl.width[s], l.dim[s], m->bond[i + 2].dim[t], 1,
                     false);
        p.add_seg(m->site[i].c() + a.panel_off[s] + a.col[s][s1], 0, 0, a.width[s], OP_N,
                  m->site[i + 1].c() + b.panel_off[mid] + b.col[mid][s2], 0, 0, b.width[mid], OP_N,
                  m->bond[i + 1].dim[mid], 1, ONE);
      }
    }
  p.run(C.ctx, TDMPS_FP64, C.batched);
}

cplx sandwich(Contractor& C, const MpoHost& O, const Mps* bra, const Mps* ket) {
  const double t0 = wall_seconds();
  struct Acc {
    Contractor& C;
    double t0;
    ~Acc() { C.t_sandwich += wall_seconds() - t0; }
  } acc_{C, t0};
  C.n_sandwich += 1;
  TDMPS_REQUIRE(bra->L == ket->L && bra->L == O.L, TDMPS_ERR_ARG, "length mismatch");
  TDMPS_REQUIRE(bra->total == ket->total, TDMPS_ERR_SECTOR, "bra and ket have different total charge");
  Env E = env_left_boundary(C.ctx, bra->bond[0], ket->bond[0]);
  for (int i = 0; i < bra->L; ++i) {
    SideOps ops = premix_left(C, E, O, i);
    Env N = env_left_update(C, ops, bra, bra->site[i].c(), bra->lay[i], bra->bond[i], bra->bond[i + 1],
                            ket->site[i].c(), ket->lay[i], ket->bond[i], ket->bond[i + 1], O);
    E = std::move(N);
  }
  cplx out{0, 0};
  if (E.b.size) dev_d2h(&out, E.b.data.p, sizeof(cplx), C.ctx->stream);
  return out;
}

cplx overlap(Contractor& C, const Mps* a, const Mps* b) {
  MpoHost I = identity_mpo(a->L);
  return sandwich(C, I, a, b);
}

std::vector<cplx> sandwich_many(Contractor& C, const MpoHost& O, const std::vector<const Mps*>& bras,
                                const Mps* ket) {
  const double t0 = wall_seconds();
  struct Acc {
    Contractor& C;
    double t0;
    ~Acc() { C.t_sandwich += wall_seconds() - t0; }
  } acc_{C, t0};
  const size_t nb = bras.size();
  C.n_sandwich += (double)nb;
  std::vector<cplx> out(nb, cplx{0, 0});
  if (nb == 0) return out;
  for (const Mps* b : bras) {
    TDMPS_REQUIRE(b->L == ket->L && b->L == O.L, TDMPS_ERR_ARG, "length mismatch");
    TDMPS_REQUIRE(b->total == ket->total, TDMPS_ERR_SECTOR, "bra and ket have different total charge");
  }
  std::vector<Env> E;
  E.reserve(nb);
  for (const Mps* b : bras) E.push_back(env_left_boundary(C.ctx, b->bond[0], ket->bond[0]));
  // Bras advance site by site together.  At each site the bras are taken in chunks: every
  // chunk's premix products run as one grouped launch, then its two environment stages as one
  // grouped launch each.  A chunk closes when its intermediates exceed the byte budget
  // (TDMPS_SANDWICH_BUDGET_GB, default 1): small environments (chain ends, small D) share
  // launches, large ones (D ~ 1000, several GB of intermediates each) go one bra at a time.
  double budget_gb = 1;
  if (const char* e = std::getenv("TDMPS_SANDWICH_BUDGET_GB")) budget_gb = std::atof(e);
  const double budget = budget_gb * (double)(1ull << 30);
  for (int i = 0; i < ket->L; ++i) {
    std::vector<Env> N(nb);
    size_t j0 = 0;
    while (j0 < nb) {
      const double tp = wall_seconds();
      GemmPlan P0, P1, P1b, P2;
      std::vector<SideOps> ops;
      std::vector<DevBuf> T;
      ops.reserve(nb - j0);
      T.reserve(nb - j0);
      double bytes = 0;
      size_t j1 = j0;
      while (j1 < nb && (j1 == j0 || bytes < budget)) {
        const Mps* b = bras[j1];
        ops.push_back(build_ops(C, E[j1], O, i, true, &P0));
        T.emplace_back();
        env_left_plan(ops.back(), b->site[i].c(), b->lay[i], b->bond[i], b->bond[i + 1], ket->site[i].c(),
                      ket->lay[i], ket->bond[i], ket->bond[i + 1], O, C.ctx, P1, P1b, P2, T.back(), N[j1]);
        bytes += (double)T.back().bytes + (ops.back().mix ? (double)ops.back().mix->data.bytes : 0.0);
        ++j1;
      }
      const double tr = wall_seconds();
      P0.run(C.ctx, TDMPS_FP64, C.batched);
      if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
      C.mix_flops += P0.flops;
      const double te = wall_seconds();
      C.t_mix += te - tr;
      P1.run(C.ctx, C.precision, C.batched);
      P1b.run(C.ctx, C.precision, C.batched);
      P2.run(C.ctx, C.precision, C.batched);
      if (C.ctx->phase_sync) dev_sync(C.ctx->stream);
      C.t_plan += (tr - tp) + P0.host_s + P1.host_s + P1b.host_s + P2.host_s;
      C.env_flops += P1.flops + P1b.flops + P2.flops;
      C.t_env += wall_seconds() - te;
      C.n_env += (double)(j1 - j0);
      j0 = j1;
    }
    E = std::move(N);
  }
  for (size_t j = 0; j < nb; ++j)
    if (E[j].b.size) dev_d2h(&out[j], E[j].b.data.p, sizeof(cplx), C.ctx->stream);
  return out;
}

}  // namespace tdmps
