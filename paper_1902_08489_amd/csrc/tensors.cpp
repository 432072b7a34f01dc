// Block-sparse layouts, device buffers, task plans and basic state constructors.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "engine.h"

namespace tdmps {

double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- device buffers
DevBuf::DevBuf(size_t b) : bytes(b) {
  if (b == 0) return;
  p = dev_alloc(b);
  TDMPS_REQUIRE(p != nullptr, TDMPS_ERR_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
}
DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
  if (p && own) dev_free(p);
  p = nullptr;
  bytes = 0;
  own = true;
}

void* Arena::take(size_t b) {
  const size_t start = (used + 255) & ~(size_t)255;
  TDMPS_REQUIRE(start <= cap && b <= cap - start, TDMPS_ERR_ARG,
                "the operation needs more than the " + std::to_string(cap >> 20) +
                    " MiB of the no-allocation scratch (intermediates and task tables)");
  used = start + b;
  return base + start;
}

DevBuf Arena::view(size_t b) {
  DevBuf d;
  if (b == 0) return d;
  d.p = take(b);
  d.bytes = b;
  d.own = false;
  return d;
}

// ---------------------------------------------------------------- bonds and layouts
int Bond::find(Charge c) const {
  auto it = std::lower_bound(q.begin(), q.end(), c);
  if (it == q.end() || *it != c) return -1;
  return (int)(it - q.begin());
}

void SiteLayout::build(const Bond& l, const Bond& r) {
  int n = l.nsec();
  panel_off.assign(n, 0);
  width.assign(n, 0);
  rs.assign(n, {-1, -1, -1, -1});
  col.assign(n, {0, 0, 0, 0});
  size = 0;
  for (int a = 0; a < n; ++a) {
    int w = 0;
    for (int s = 0; s < 4; ++s) {
      int b = r.find(l.q[a] + local_charge(s));
      rs[a][s] = b;
      if (b >= 0) {
        col[a][s] = w;
        w += r.dim[b];
      }
    }
    width[a] = w;
    panel_off[a] = size;
    size += (int64_t)l.dim[a] * w;
  }
}

void TwoLayout::build(const Bond& l, const Bond& r) {
  int n = l.nsec();
  panel_off.assign(n, 0);
  width.assign(n, 0);
  rs.assign(n, {});
  col.assign(n, {});
  size = 0;
  for (int a = 0; a < n; ++a) {
    int w = 0;
    for (int s = 0; s < 16; ++s) {
      int b = r.find(l.q[a] + pair_charge(s));
      rs[a][s] = b;
      col[a][s] = 0;
      if (b >= 0) {
        col[a][s] = w;
        w += r.dim[b];
      }
    }
    width[a] = w;
    panel_off[a] = size;
    size += (int64_t)l.dim[a] * w;
  }
}

void Blocks::layout(const Bond& b, const Bond& k, const std::vector<std::pair<Charge, int>>& groups) {
  bra = b;
  ket = k;
  grp.clear();
  size = 0;
  for (auto& g : groups) {
    StackGroup sg;
    sg.q = g.first;
    sg.n = g.second;
    sg.bra_of.assign(k.nsec(), -1);
    sg.ket_of.assign(b.nsec(), -1);
    sg.off.assign(k.nsec(), -1);
    for (int ks = 0; ks < k.nsec(); ++ks) {
      int bs = b.find(k.q[ks] + g.first);
      if (bs < 0) continue;
      sg.bra_of[ks] = bs;
      sg.ket_of[bs] = ks;
      sg.off[ks] = size;
      size += (int64_t)g.second * b.dim[bs] * k.dim[ks];
    }
    grp.push_back(std::move(sg));
  }
}

// ---------------------------------------------------------------- plans
// Per-thread pools of host vectors for plan building: the large lists of a plan (hundreds of
// thousands of segments at the L = 24, D = 1024 centre) are reused with their capacity, which
// saves the growth copies and the page faults of fresh allocations on every plan.
namespace {
template <class T>
struct VecPool {
  std::vector<std::vector<T>> free;
  std::vector<T> take() {
    if (free.empty()) return {};
    std::vector<T> v = std::move(free.back());
    free.pop_back();
    v.clear();
    return v;
  }
  void give(std::vector<T>& v) {
    constexpr size_t MAX_BYTES = (size_t)256 << 20;
    if (v.capacity() == 0 || v.capacity() * sizeof(T) > MAX_BYTES || free.size() >= 8) return;
    v.clear();
    free.push_back(std::move(v));
    v = std::vector<T>();
  }
};
thread_local VecPool<GemmTask> t_task_pool;
thread_local VecPool<GemmSeg> t_seg_pool;
thread_local VecPool<char> t_img_pool;
}  // namespace

int GemmPlan::begin_task(cplx* C, int64_t bsC, int ldc, int m, int n, int nbatch, bool accum) {
  if (tasks.capacity() == 0) tasks = t_task_pool.take();
  GemmTask t;
  t.C = C;
  t.bsC = bsC;
  t.ldc = ldc;
  t.m = m;
  t.n = n;
  t.nbatch = nbatch;
  t.seg0 = (int32_t)segs.size();
  t.nseg = 0;
  t.tiles_m = t.tiles_n = 0;
  t.flags = accum ? GEMM_ACCUM : 0;
  t.tile_base = 0;
  tasks.push_back(t);
  return (int)tasks.size() - 1;
}

void GemmPlan::add_seg(const cplx* A, int64_t bsA, int64_t rsA, int lda, int opA, const cplx* B, int64_t bsB,
                       int64_t rsB, int ldb, int opB, int k, int nred, cplx alpha) {
  if (segs.capacity() == 0) segs = t_seg_pool.take();
  GemmSeg s;
  s.A = A;
  s.B = B;
  s.bsA = bsA;
  s.bsB = bsB;
  s.rsA = rsA;
  s.rsB = rsB;
  s.nred = nred;
  s.k = k;
  s.lda = lda;
  s.ldb = ldb;
  s.opA = opA;
  s.opB = opB;
  s.alpha = alpha;
  segs.push_back(s);
  GemmTask& t = tasks.back();
  t.nseg++;
  flops += (real_a ? 4.0 : 8.0) * t.m * (double)t.n * k * nred * t.nbatch;
}

void GemmPlan::finalize(Ctx* ctx, int precision) {
  if (final_) return;
  final_ = true;
  ntasks_built = tasks.size();
  nsegs_built = segs.size();
  struct Release {
    GemmPlan& p;
    ~Release() {
      t_task_pool.give(p.tasks);
      t_seg_pool.give(p.segs);
    }
  } release_{*this};
  // Split-K: a task whose reduction is long (many channels) is cut into parts of about
  // KSPLIT complex k; parts write private partial outputs that a reduction kernel adds in
  // a fixed order (deterministic, no atomics).
  const int64_t KSPLIT = 1024;
  const int64_t esz = ops32 ? 8 : (int64_t)sizeof(cplx);  // bytes per operand element
  std::vector<GemmTask> out = t_task_pool.take();
  std::vector<GemmSeg> nsegs = t_seg_pool.take();
  struct Scratch {
    std::vector<GemmTask>& out;
    std::vector<GemmSeg>& nsegs;
    ~Scratch() {
      t_task_pool.give(out);
      t_seg_pool.give(nsegs);
    }
  } scratch_{out, nsegs};
  out.reserve(tasks.size());
  nsegs.reserve(segs.size());
  std::vector<ReduceTask> red;
  std::vector<std::pair<size_t, int64_t>> part_of;  // (task index in out, offset in workspace)
  int64_t ws = 0;
  for (auto& t : tasks) {
    // drop tasks without work that do not need to overwrite their output
    if (!(t.m > 0 && t.n > 0 && t.nbatch > 0 && (t.nseg > 0 || !(t.flags & GEMM_ACCUM)))) continue;
    int64_t work = 0;
    for (int s = t.seg0; s < t.seg0 + t.nseg; ++s) work += (int64_t)segs[s].nred * segs[s].k;
    int nparts = (t.nbatch == 1 && work > 2 * KSPLIT) ? (int)std::min<int64_t>(64, (work + KSPLIT - 1) / KSPLIT) : 1;
    if (nparts <= 1) {
      GemmTask c = t;
      c.seg0 = (int32_t)nsegs.size();
      for (int s = t.seg0; s < t.seg0 + t.nseg; ++s) nsegs.push_back(segs[s]);
      out.push_back(c);
      continue;
    }
    const int64_t target = (work + nparts - 1) / nparts;
    ReduceTask rt;
    rt.C = t.C;
    rt.parts = nullptr;
    rt.m = t.m;
    rt.n = t.n;
    rt.ldc = t.ldc;
    rt.accum = (t.flags & GEMM_ACCUM) ? 1 : 0;
    rt.out32 = (t.flags & GEMM_OUT32) ? 1 : 0;
    int64_t base = ws;
    int made = 0;
    GemmTask cur = t;
    cur.flags = 0;
    cur.ldc = t.n;
    cur.bsC = 0;
    cur.nseg = 0;
    cur.seg0 = (int32_t)nsegs.size();
    int64_t acc = 0;
    auto close = [&]() {
      if (cur.nseg == 0) return;
      part_of.push_back({out.size(), base + (int64_t)made * t.m * t.n});
      out.push_back(cur);
      ++made;
      cur.nseg = 0;
      cur.seg0 = (int32_t)nsegs.size();
      acc = 0;
    };
    for (int s = t.seg0; s < t.seg0 + t.nseg; ++s) {
      const GemmSeg& g = segs[s];
      int r = 0;
      while (r < g.nred) {
        int64_t room = target - acc;
        int take = (int)std::max<int64_t>(1, std::min<int64_t>(g.nred - r, room / std::max(1, g.k)));
        GemmSeg v = g;
        v.A = (const cplx*)((const char*)g.A + (int64_t)r * g.rsA * esz);
        v.B = (const cplx*)((const char*)g.B + (int64_t)r * g.rsB * esz);
        v.nred = take;
        nsegs.push_back(v);
        cur.nseg++;
        acc += (int64_t)take * g.k;
        r += take;
        if (acc >= target) close();
      }
    }
    close();
    rt.nparts = made;
    ws += (int64_t)made * t.m * t.n;
    red.push_back(rt);
    red_base.push_back(base);
  }
  if (out.empty()) return;
  if (ws > 0) {
    wspace = arena ? arena->view(ws * sizeof(cplx)) : DevBuf(ws * sizeof(cplx));
    for (auto& po : part_of) out[po.first].C = wspace.c() + po.second;
    for (size_t k = 0; k < red.size(); ++k) red[k].parts = wspace.c() + red_base[k];
    nred_tasks = (int)red.size();
  }
  // Tile shape per task: a forced shape (tdmps_ctx_set_tile_config), else the measured best
  // shape of the task's bucket (tdmps_ctx_autotune), else the least padded MFMA work divided
  // by the shape's relative throughput (measured on aligned shapes with enough tiles to fill
  // the chip, FP64; the 64 x 32 entry set on the real task mix instead: 0.97 -> 1.05 took the
  // FP64 H_eff apply at L = 24, D = 1024 from 39.7 to 37.9 ms and left the other precisions as
  // they were).  TDMPS_TILE_EFF (comma-separated, one value per shape in tile-configuration
  // order) overrides the table, for measuring other choices.
  static const std::vector<double> eff = [] {
    std::vector<double> e = {1.0, 0.92, 0.9, 0.96, 0.82, 0.8, 0.94, 0.85, 0.8, 1.05};
    if (const char* env = std::getenv("TDMPS_TILE_EFF")) {
      std::vector<double> v;
      for (const char* q = env; *q;) {
        char* end = nullptr;
        const double x = std::strtod(q, &end);
        if (end == q || !(x > 0.0)) break;
        v.push_back(x);
        q = *end == ',' ? end + 1 : end;
        if (*end != ',') break;
      }
      if (v.size() == e.size()) e = v;
    }
    return e;
  }();
  const TileTable* tt_tab = (precision >= 0 && precision < 4 && ctx->tune[precision].valid) ? &ctx->tune[precision]
                                                                                           : nullptr;
  // real-A products (premix) and the three-term BF16 split take the cost model over the shapes
  // whose kernels keep every value in registers (128 x 48 and 96 x 64 spill there)
  auto usable = [&](int c) {
    return !(real_a || precision == TDMPS_BF16X6) || (gemm_tile_m(c) * gemm_tile_n(c) < 6144);
  };
  // Operand traffic: a tile reads (BM + BN) k operand elements.  The reduced precisions are
  // bound by staging and operand traffic rather than by the matrix units, so their cost is
  // the larger of the padded work and lam x the tile's operand reads (lam in padded
  // multiply-adds per operand element; TDMPS_TILE_LAMBDA overrides); FP64 products hide
  // the reads behind the matrix work (lam = 0: larger tiles only lose occupancy there).
  static const char* lam_env = std::getenv("TDMPS_TILE_LAMBDA");
  const double lam = lam_env ? std::atof(lam_env) : precision == TDMPS_FP64 ? 0.0 : precision == TDMPS_FP32 ? 70.0 : 45.0;
  auto pick = [&](const GemmTask& t) {
    if (ctx->tile_cfg >= 0 && usable(ctx->tile_cfg)) return ctx->tile_cfg;
    if (tt_tab && !real_a && precision != TDMPS_BF16X6) {
      int64_t k = 0;
      for (int s = t.seg0; s < t.seg0 + t.nseg; ++s) k += (int64_t)nsegs[s].nred * nsegs[s].k;
      return (int)tt_tab->cfg[tile_bucket(t.m)][tile_bucket(t.n)][tile_kbucket(k)];
    }
    int best = 0;
    double bc = 1e300;
    for (int c = 0; c < NCFG; ++c) {
      if (!usable(c)) continue;
      const int bm = gemm_tile_m(c), bn = gemm_tile_n(c);
      const double tiles = (double)((t.m + bm - 1) / bm) * ((t.n + bn - 1) / bn);
      const double cost = std::max(tiles * bm * bn / eff[c], lam * tiles * (bm + bn));
      if (cost < bc) {
        bc = cost;
        best = c;
      }
    }
    return best;
  };
  std::vector<int> choice(out.size());
  for (size_t i = 0; i < out.size(); ++i) choice[i] = pick(out[i]);
  // Host image of the device tables: segments, reduction tasks, then per tile shape the task
  // list and the tile -> task map, each 256-byte aligned; one upload.
  std::vector<std::vector<GemmTask>> sel(NCFG);
  std::vector<std::vector<int32_t>> tmap(NCFG);
  for (int cfg = 0; cfg < NCFG; ++cfg) {
    int64_t base = 0;
    const int tm = gemm_tile_m(cfg), tn = gemm_tile_n(cfg);
    for (size_t i = 0; i < out.size(); ++i) {
      if (choice[i] != cfg) continue;
      GemmTask t = out[i];
      t.tiles_m = (t.m + tm - 1) / tm;
      t.tiles_n = (t.n + tn - 1) / tn;
      t.tile_base = base;
      base += (int64_t)t.nbatch * t.tiles_m * t.tiles_n;
      sel[cfg].push_back(t);
    }
    ntask[cfg] = (int)sel[cfg].size();
    ntiles[cfg] = base;
    htile_base[cfg].clear();
    for (auto& t : sel[cfg]) htile_base[cfg].push_back(t.tile_base);
    tmap[cfg].resize((size_t)base);
    for (size_t k = 0; k < sel[cfg].size(); ++k) {
      const int64_t nt = (int64_t)sel[cfg][k].nbatch * sel[cfg][k].tiles_m * sel[cfg][k].tiles_n;
      std::fill(tmap[cfg].begin() + sel[cfg][k].tile_base, tmap[cfg].begin() + sel[cfg][k].tile_base + nt,
                (int32_t)k);
    }
  }
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t bytes = 0;
  const size_t o_segs = bytes;
  bytes = align(bytes + nsegs.size() * sizeof(GemmSeg));
  const size_t o_red = bytes;
  bytes = align(bytes + red.size() * sizeof(ReduceTask));
  size_t o_task[NCFG], o_tile[NCFG];
  for (int cfg = 0; cfg < NCFG; ++cfg) {
    o_task[cfg] = bytes;
    bytes = align(bytes + sel[cfg].size() * sizeof(GemmTask));
    o_tile[cfg] = bytes;
    bytes = align(bytes + tmap[cfg].size() * sizeof(int32_t));
  }
  const size_t o_extra = bytes;
  bytes = align(bytes + extra.size());
  std::vector<char> img = t_img_pool.take();
  struct ImgBack {
    std::vector<char>& v;
    ~ImgBack() { t_img_pool.give(v); }
  } img_back_{img};
  img.resize(bytes);
  if (!nsegs.empty()) std::memcpy(img.data() + o_segs, nsegs.data(), nsegs.size() * sizeof(GemmSeg));
  if (!red.empty()) std::memcpy(img.data() + o_red, red.data(), red.size() * sizeof(ReduceTask));
  for (int cfg = 0; cfg < NCFG; ++cfg) {
    if (!sel[cfg].empty()) std::memcpy(img.data() + o_task[cfg], sel[cfg].data(), sel[cfg].size() * sizeof(GemmTask));
    if (!tmap[cfg].empty()) std::memcpy(img.data() + o_tile[cfg], tmap[cfg].data(), tmap[cfg].size() * sizeof(int32_t));
  }
  if (!extra.empty()) std::memcpy(img.data() + o_extra, extra.data(), extra.size());
  if (arena) {
    // the image goes back to a reuse pool on return: copy from it and wait
    dtab = arena->view(bytes);
    dev_h2d_wait(dtab.p, img.data(), bytes, ctx->stream);
  } else {
    dtab = DevBuf(bytes);
    dev_h2d(dtab.p, img.data(), bytes, ctx->stream);
  }
  char* b = (char*)dtab.p;
  dextra = extra.empty() ? nullptr : b + o_extra;
  dsegs = (const GemmSeg*)(b + o_segs);
  dred = red.empty() ? nullptr : (const ReduceTask*)(b + o_red);
  for (int cfg = 0; cfg < NCFG; ++cfg) {
    dtasks[cfg] = (const GemmTask*)(b + o_task[cfg]);
    dtile[cfg] = (const int32_t*)(b + o_tile[cfg]);
  }
}

void GemmPlan::launch(Ctx* ctx, int precision, bool batched) {
  for (int cfg = 0; cfg < NCFG; ++cfg) {
    if (ntask[cfg] <= 0) continue;
    if (batched) {
      launch_gemm(dtasks[cfg], dsegs, dtile[cfg], ntiles[cfg],
                  cfg, precision, ctx->stream, 0, ops32, real_a);
    } else {
      // one launch per task: the grid covers the task's own tiles only
      for (size_t t = 0; t < htile_base[cfg].size(); ++t) {
        const int64_t b0 = htile_base[cfg][t];
        const int64_t b1 = t + 1 < htile_base[cfg].size() ? htile_base[cfg][t + 1] : ntiles[cfg];
        launch_gemm(dtasks[cfg], dsegs, dtile[cfg], b1 - b0,
                    cfg, precision, ctx->stream, b0, ops32, real_a);
      }
    }
  }
  if (nred_tasks > 0) launch_reduce(dred, nred_tasks, ctx->stream);
}

void GemmPlan::run(Ctx* ctx, int precision, bool batched) {
  const double t0 = wall_seconds();
  finalize(ctx, precision);
  host_s += wall_seconds() - t0;
  launch(ctx, precision, batched);
  if (ctx->phase_sync) dev_sync(ctx->stream);
}

void CopyPlan::add(const cplx* src, int64_t src_rs, int64_t src_cs, cplx* dst, int dst_ld, int rows, int cols, int flags,
                   const int32_t* ridx, const int32_t* cidx, const double* rs, const double* cs) {
  if (rows <= 0 || cols <= 0) return;
  CopyTask t;
  t.src = src;
  t.dst = dst;
  t.src_rs = src_rs;
  t.src_cs = src_cs;
  t.ridx = ridx;
  t.cidx = cidx;
  t.rscale = rs;
  t.cscale = cs;
  t.rows = rows;
  t.cols = cols;
  t.dst_ld = dst_ld;
  t.flags = flags;
  tasks.push_back(t);
}

void CopyPlan::run(Ctx* ctx) {
  if (tasks.empty()) return;
  Staging st;
  const CopyTask* d = st.put(ctx, tasks);
  launch_copy(d, (int)tasks.size(), ctx->stream);
  if (ctx->phase_sync) dev_sync(ctx->stream);
}

// ---------------------------------------------------------------- states
Mps* mps_new(Ctx* ctx, int L, const std::vector<Bond>& bonds) {
  TDMPS_REQUIRE((int)bonds.size() == L + 1, TDMPS_ERR_ARG, "need L+1 bonds");
  dev_bind(ctx->device, ctx->stream);
  auto* m = new Mps();
  try {
    m->ctx = ctx;
    m->L = L;
    m->bond = bonds;
    TDMPS_REQUIRE(bonds[0].nsec() == 1 && bonds[0].q[0] == Charge(0, 0) && bonds[0].dim[0] == 1, TDMPS_ERR_ARG,
                  "bond 0 must be the single sector (0,0) of dimension 1");
    TDMPS_REQUIRE(bonds[L].nsec() == 1 && bonds[L].dim[0] == 1, TDMPS_ERR_ARG,
                  "bond L must be a single sector of dimension 1");
    m->total = bonds[L].q[0];
    m->lay.resize(L);
    m->site.resize(L);
    for (int i = 0; i < L; ++i) {
      m->lay[i].build(bonds[i], bonds[i + 1]);
      m->site[i] = DevBuf(m->lay[i].size * sizeof(cplx));
      if (m->lay[i].size) dev_zero(m->site[i].p, m->site[i].bytes, ctx->stream);
    }
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

Mps* mps_clone(const Mps* src) {
  dev_bind(src->ctx->device, src->ctx->stream);
  auto* m = new Mps();
  try {
    m->ctx = src->ctx;
    m->L = src->L;
    m->total = src->total;
    m->bond = src->bond;
    m->lay = src->lay;
    m->site.resize(src->L);
    for (int i = 0; i < src->L; ++i) {
      m->site[i] = DevBuf(src->site[i].bytes);
      if (src->site[i].bytes) dev_d2d(m->site[i].p, src->site[i].p, src->site[i].bytes, src->ctx->stream);
    }
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

void mps_from_det(Mps* m, const uint8_t* occ) {
  std::vector<cplx> one(1, cplx{1.0, 0.0});
  for (int i = 0; i < m->L; ++i) {
    TDMPS_REQUIRE(m->lay[i].size == 1, TDMPS_ERR_ARG, "determinant layout");
    dev_h2d(m->site[i].p, one.data(), sizeof(cplx), m->ctx->stream);
  }
}

Mps* mps_annihilate(Ctx* ctx, const Mps* psi, int j, int sigma) {
  const int L = psi->L;
  TDMPS_REQUIRE(j >= 0 && j < L && (sigma == 0 || sigma == 1), TDMPS_ERR_ARG, "site or spin out of range");
  const Charge e = sigma == 0 ? Charge(1, 0) : Charge(0, 1);
  auto has = [&](Charge q) { return sigma == 0 ? q.nu >= 1 : q.nd >= 1; };
  TDMPS_REQUIRE(has(psi->total), TDMPS_ERR_SECTOR, "the state has no electron of that spin");
  // bonds left of site j (cuts <= j) are kept; right of it every charge loses e, and sectors
  // without an electron of spin sigma left of the cut cannot survive the annihilation
  std::vector<Bond> nb(L + 1);
  std::vector<std::vector<int>> map(L + 1);
  for (int c = 0; c <= L; ++c) {
    const Bond& b = psi->bond[c];
    map[c].assign(b.nsec(), -1);
    for (int s = 0; s < b.nsec(); ++s) {
      if (c <= j) {
        map[c][s] = nb[c].nsec();
        nb[c].q.push_back(b.q[s]);
        nb[c].dim.push_back(b.dim[s]);
      } else if (has(b.q[s])) {
        map[c][s] = nb[c].nsec();
        nb[c].q.push_back(b.q[s] - e);
        nb[c].dim.push_back(b.dim[s]);
      }
    }
  }
  Mps* m = mps_new(ctx, L, nb);
  try {
    int maxd = 1;
    for (auto& b : psi->bond)
      for (int d : b.dim) maxd = std::max(maxd, d);
    Staging st;
    const double* minus = st.put(ctx, std::vector<double>((size_t)maxd, -1.0));
    CopyPlan cp;
    for (int k = 0; k < L; ++k) {
      const SiteLayout& ol = psi->lay[k];
      const SiteLayout& nl = m->lay[k];
      const Bond& bl = psi->bond[k];
      const Bond& br = psi->bond[k + 1];
      for (int a = 0; a < bl.nsec(); ++a) {
        const int na = map[k][a];
        if (na < 0) continue;
        for (int n = 0; n < 4; ++n) {
          const int b = ol.rs[a][n];
          if (b < 0) continue;
          int n2 = n;
          bool neg = false;
          if (k < j) {
            neg = local_parity(n) == 1;  // Jordan-Wigner string
          } else if (k == j) {
            if (!((n >> sigma) & 1)) continue;
            n2 = n ^ (1 << sigma);
            neg = sigma == 1 && (n & 1);  // the down operator passes the up electron of the site
          }
          const int b2 = map[k + 1][b];
          if (b2 < 0) continue;
          TDMPS_REQUIRE(nl.rs[na][n2] == b2, TDMPS_ERR_NUMERIC, "internal: annihilated block sector");
          cp.add(psi->site[k].c() + ol.panel_off[a] + ol.col[a][n], ol.width[a], 1,
                 m->site[k].c() + nl.panel_off[na] + nl.col[na][n2], nl.width[na], bl.dim[a], br.dim[b], 0, nullptr,
                 nullptr, neg ? minus : nullptr, nullptr);
        }
      }
    }
    cp.run(ctx);
    dev_sync(ctx->stream);
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

static MpoHost build_identity_mpo(int L) {
  MpoHost M;
  M.L = L;
  M.cut.resize(L + 1);
  for (auto& c : M.cut) {
    c.key = {0};
    c.q = {Charge(0, 0)};
    c.parity = {0};
    c.cls_q = {Charge(0, 0)};
    c.cls_start = {0};
    c.cls_count = {1};
    c.cls_of = {0};
  }
  M.W.resize(L);
  M.c_fixed.resize(L);
  for (int p = 0; p < L; ++p)
    for (int s = 0; s < 4; ++s) {
      M.W[p].push_back({0, 0, (int8_t)s, (int8_t)s, 1.0});
      M.c_fixed[p].push_back(1.0);
    }
  M.h.assign((size_t)L * L, 0.0);
  return M;
}

// One operator per length, so that its version (and the premix structures cached under it)
// stays the same from call to call.
MpoHost identity_mpo(int L) {
  static std::mutex& mu = *new std::mutex;
  static std::map<int, MpoHost>& made = *new std::map<int, MpoHost>;
  std::lock_guard<std::mutex> lk(mu);
  auto it = made.find(L);
  if (it == made.end()) it = made.emplace(L, build_identity_mpo(L)).first;
  return it->second;
}

void scale_mps(Ctx* ctx, Mps* m, cplx alpha) {
  if (m->lay[0].size) launch_scale(m->site[0].c(), m->lay[0].size, alpha, ctx->stream);
}

}  // namespace tdmps
