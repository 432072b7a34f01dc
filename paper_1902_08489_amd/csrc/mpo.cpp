// Exact MPO of the ab-initio Hamiltonian (Methods, Eq. (hamil)).
//
// The paper gives the Hamiltonian but no MPO construction; this one is built as a
// finite-state automaton over spin-orbital operator strings.  Every normal-ordered term
// (a+ a, a+ a+ a a) is sorted into spin-orbital order (sign from the anticommutations)
// and follows a path of "channels" across the cuts of the chain.  At a cut the channel
// of a term is fixed by how many of its fermion operators lie left of the cut:
//   0 -> I (identity so far),  all -> H (term complete),
//   1 -> L1(left operator)          -- left part unique, right part still to come,
//   3 -> R1(right operator)         -- right part unique, left part a coefficient sum,
//   2 -> L2(left pair)  left of the chain centre, R2(right pair) right of it.
// Channels I, L1, L2 carry a unique left operator and H, R1, R2 a unique right
// operator, so each term crosses from the first group to the second exactly once; its
// coefficient sits on that transition and every other transition is a pure operator
// with coefficient one.  Summing coefficients of terms that share a crossing realises
// the complementary-operator sums (the O(L^4 D^2) part of the cost statement in the
// "Operations on MPS" section).  Jordan-Wigner strings: the local factor on a spin
// orbital is (its operators) x P^(number of the term's operators to its right), P =
// (-1)^n, which makes the channel's fermion parity the exponent of P on pass-through.
// Spin orbitals 2p (up) and 2p+1 (down) are merged into the 4-dimensional site p.
#include "mpo.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <tuple>
#include <unordered_map>
#include <unordered_set>

namespace tdmps {
namespace {

enum KeyType { K_I = 0, K_H = 1, K_L1 = 2, K_L2 = 3, K_R2 = 4, K_R1 = 5 };
enum OpType { OP_C = 0, OP_A = 1, OP_N = 2 };

struct SOp {
  int so;  // spin orbital
  int t;   // OP_C / OP_A / OP_N
  int f;   // number of fermion operators (1, or 2 for N)
};

inline uint32_t opcode(const SOp& o) { return (uint32_t)(o.so << 2 | o.t) + 1; }  // 0 = none
inline uint64_t mk_key(int type, uint32_t a, uint32_t b) {
  return (uint64_t)type << 48 | (uint64_t)a << 24 | (uint64_t)b;
}
inline int key_type(uint64_t k) { return (int)(k >> 48); }
inline uint32_t key_a(uint64_t k) { return (uint32_t)(k >> 24) & 0xffffff; }
inline uint32_t key_b(uint64_t k) { return (uint32_t)k & 0xffffff; }
inline bool left_unique(int t) { return t == K_I || t == K_L1 || t == K_L2; }

Charge op_charge(uint32_t code) {
  if (!code) return Charge(0, 0);
  code -= 1;
  int so = code >> 2, t = code & 3;
  int sgn = t == OP_C ? 1 : (t == OP_A ? -1 : 0);
  return (so & 1) ? Charge(0, sgn) : Charge(sgn, 0);
}

Charge key_charge(uint64_t k) {
  Charge c = op_charge(key_a(k)) + op_charge(key_b(k));
  int t = key_type(k);
  if (t == K_R1 || t == K_R2) return Charge(0, 0) - c;
  return c;
}

int key_parity(uint64_t k) {
  int t = key_type(k);
  return (t == K_L1 || t == K_R1) ? 1 : 0;
}

// Order of channels inside a class: by type, then so that channels which pass
// through a site unchanged keep their relative order on both sides of it.
// Pair channels are ordered by the kinds and spins of their two operators before their
// orbitals: channels that differ only in orbitals combine the same local matrix units of a
// site tensor, so keeping them adjacent makes long runs of identical structure (one stacked
// product instead of one product per channel).
std::array<int64_t, 4> key_order(uint64_t k) {
  int t = key_type(k);
  int64_t a = key_a(k), b = key_b(k);
  int64_t sa = a ? (a - 1) >> 2 : -1, sb = b ? (b - 1) >> 2 : -1;
  auto kind = [](int64_t code) -> int64_t { return code ? ((code - 1) & 3) * 2 + (((code - 1) >> 2) & 1) : 0; };
  const int64_t sig = kind(a) * 8 + kind(b);
  switch (t) {
    case K_L1: return {t, sa, a, 0};
    case K_L2: return {t, sig, std::max(sa, sb) * 4096 + std::min(sa, sb), a * 4096 + b};
    case K_R2: return {t, sig, std::min(sa, sb) * 4096 + std::max(sa, sb), a * 4096 + b};
    case K_R1: return {t, sa, a, 0};
    default: return {t, 0, 0, 0};
  }
}

struct Mat4 {
  double m[16] = {0};
};

// 2x2 spin-orbital operators, [out][in].
void op2(int t, bool present, int par, double o[2][2]) {
  double a[2][2] = {{1, 0}, {0, 1}};
  if (present) {
    a[0][0] = a[0][1] = a[1][0] = a[1][1] = 0;
    if (t == OP_C) a[1][0] = 1;
    if (t == OP_A) a[0][1] = 1;
    if (t == OP_N) a[1][1] = 1;
  }
  // right-multiply by P^par: column n' scaled by (-1)^(n' * par)
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) o[r][c] = a[r][c] * ((par && c == 1) ? -1.0 : 1.0);
}

struct TransKey {
  int site;
  uint64_t kin, kout;
  bool operator==(const TransKey& o) const { return site == o.site && kin == o.kin && kout == o.kout; }
};
struct TransHash {
  size_t operator()(const TransKey& k) const {
    uint64_t x = k.kin * 0x9E3779B97F4A7C15ull ^ (k.kout + 0x632BE59BD9B4E019ull) * 0xBF58476D1CE4E5B9ull ^
                 (uint64_t)k.site * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (size_t)x;
  }
};

struct Builder {
  int L, K, imid;
  int adjacent_window = -1;  // cuts i with |i - imid| <= window use the adjacent-operator rule
  std::unordered_map<uint64_t, std::pair<int, int>> range;  // key -> [first cut, last cut]
  std::unordered_map<uint64_t, std::pair<int, int>> range_plain;  // the same under the plain rule
  std::unordered_map<TransKey, Mat4, TransHash> structural;
  std::unordered_map<TransKey, Mat4, TransHash> coeff;      // from two-body terms and e0
  struct OB {
    TransKey tk;
    int p, q;
    Mat4 m;
  };
  std::vector<OB> onebody;

  static void touch_in(std::unordered_map<uint64_t, std::pair<int, int>>& range, uint64_t k, int a, int b) {
    auto it = range.find(k);
    if (it == range.end())
      range.emplace(k, std::make_pair(a, b));
    else {
      it->second.first = std::min(it->second.first, a);
      it->second.second = std::max(it->second.second, b);
    }
  }  void touch(uint64_t k, int a, int b) { touch_in(range, k, a, b); }


  // ops in written order; one-body terms carry (p, q) so their coefficient can be replaced.
  void term(double coef, std::vector<SOp> ops, int obp, int obq) {
    int n = (int)ops.size();
    int sign = 1;
    for (int i = 1; i < n; ++i)
      for (int j = i; j > 0 && ops[j - 1].so > ops[j].so; --j) {
        std::swap(ops[j - 1], ops[j]);
        sign = -sign;
      }
    std::vector<SOp> m;
    for (int i = 0; i < n; ++i) {
      if (!m.empty() && m.back().so == ops[i].so) {
        if (m.back().t == OP_C && ops[i].t == OP_A && m.back().f == 1) {
          m.back().t = OP_N;
          m.back().f = 2;
        } else {
          return;  // a+ a+ or a a on one spin orbital vanishes
        }
      } else {
        m.push_back(ops[i]);
      }
    }
    int total = 0;
    for (auto& o : m) total += o.f;
    auto nl_at = [&](int c) {  // fermion operators on spin orbitals < c
      int s = 0;
      for (auto& o : m)
        if (o.so < c) s += o.f;
      return s;
    };
    auto key_at = [&](int i, int window) -> uint64_t {
      int c = 2 * i;
      int nl = nl_at(c);
      if (nl == 0) return mk_key(K_I, 0, 0);
      if (nl == total) return mk_key(K_H, 0, 0);
      std::vector<uint32_t> lo, ro;
      for (auto& o : m) (o.so < c ? lo : ro).push_back(opcode(o));
      if (nl == 1) return mk_key(K_L1, lo[0], 0);
      if (nl == 3) return mk_key(K_R1, ro[0], 0);
      // two operators on each side: name the pair of the left side (L2) left of the chain
      // centre and that of the right side (R2) right of it, except when the operator nearest
      // to the cut on the named side's opposite side sits on the site next to the cut.  Then
      // the other pair is named, so that the transition on that site is a pure operator and
      // every coefficient crossing of a pair channel happens on a site without operators of
      // the term (all its channels combine the same four diagonal matrix units).
      int last_left = -1, first_right = L;
      for (auto& o : m) {
        const int site = o.so >> 1;
        if (o.so < c) last_left = std::max(last_left, site);
        else first_right = std::min(first_right, site);
      }
      bool left_pair = i < imid;
      if (std::abs(i - imid) <= window) left_pair = i < imid ? first_right != i : last_left == i - 1;
      if (left_pair) return mk_key(K_L2, lo[0], lo.size() > 1 ? lo[1] : 0);
      return mk_key(K_R2, ro[0], ro.size() > 1 ? ro[1] : 0);
    };
    std::vector<uint64_t> keys(L + 1);
    for (int i = 0; i <= L; ++i) keys[i] = key_at(i, adjacent_window);
    // channels of the plain rule (the smallest MPO, 2L^2 + 3L + 2 at the centre): the reference
    // of the algorithmic flop count
    if (adjacent_window >= 0) {
      uint64_t prev = key_at(0, -1);
      int first = 0;
      for (int i = 1; i <= L + 1; ++i) {
        const uint64_t k = i <= L ? key_at(i, -1) : ~0ull;
        if (k != prev) {
          touch_in(range_plain, prev, first, i - 1);
          prev = k;
          first = i;
        }
      }
    }
    // a term crosses from the left-unique channels (I, L1, L2) to the right-unique ones exactly
    // once, where its coefficient sits
    for (int i = 0; i < L; ++i)
      TDMPS_REQUIRE(left_unique(key_type(keys[i])) || !left_unique(key_type(keys[i + 1])), TDMPS_ERR_NUMERIC,
                    "internal: operator automaton returns to a left-unique channel");
    int start = 0;
    for (int i = 1; i <= L + 1; ++i) {
      if (i == L + 1 || keys[i] != keys[start]) {
        touch(keys[start], start, i - 1);
        start = i;
      }
    }
    for (int p = 0; p < L; ++p) {
      if (keys[p] == keys[p + 1]) continue;
      const SOp* up = nullptr;
      const SOp* dn = nullptr;
      for (auto& o : m) {
        if (o.so == 2 * p) up = &o;
        if (o.so == 2 * p + 1) dn = &o;
      }
      double ou[2][2], od[2][2];
      op2(up ? up->t : 0, up != nullptr, nl_at(2 * p + 1) & 1, ou);
      op2(dn ? dn->t : 0, dn != nullptr, nl_at(2 * p + 2) & 1, od);
      Mat4 M;
      for (int s = 0; s < 4; ++s)
        for (int sp = 0; sp < 4; ++sp) M.m[s * 4 + sp] = ou[s & 1][sp & 1] * od[s >> 1][sp >> 1];
      TransKey tk{p, keys[p], keys[p + 1]};
      bool lr = left_unique(key_type(keys[p])) && !left_unique(key_type(keys[p + 1]));
      if (!lr) {
        structural.emplace(tk, M);
      } else if (obp >= 0) {
        OB ob{tk, obp, obq, M};
        for (double& x : ob.m.m) x *= sign;
        onebody.push_back(ob);
      } else {
        Mat4& acc = coeff[tk];
        for (int e = 0; e < 16; ++e) acc.m[e] += coef * sign * M.m[e];
      }
    }
  }
};

}  // namespace

int mpo_channel_kind(uint64_t key, int* so, int* op) {
  const int t = key_type(key);
  if (t == K_I) return 0;
  if (t == K_H) return 1;
  if (t == K_L1 && key_a(key) && !key_b(key)) {
    const uint32_t code = key_a(key) - 1;
    *so = (int)(code >> 2);
    *op = (code & 3) == OP_C ? 0 : ((code & 3) == OP_A ? 1 : 2);
    return 2;
  }
  return 3;
}

MpoHost build_mpo(int L, const double* h, const double* eri, double e0, bool two_body, int adjacent_window) {
  TDMPS_REQUIRE(L >= 2 && L <= 64, TDMPS_ERR_ARG, "L must be in [2, 64]");
  for (int64_t i = 0; i < (int64_t)L * L; ++i)
    TDMPS_REQUIRE(std::isfinite(h[i]), TDMPS_ERR_NUMERIC, "non-finite one-body integral");
  if (two_body)
    for (int64_t i = 0; i < (int64_t)L * L * L * L; ++i)
      TDMPS_REQUIRE(std::isfinite(eri[i]), TDMPS_ERR_NUMERIC, "non-finite two-body integral");
  TDMPS_REQUIRE(std::isfinite(e0), TDMPS_ERR_NUMERIC, "non-finite e0");

  Builder b;
  b.L = L;
  b.K = 2 * L;
  b.imid = L / 2;
  b.adjacent_window = adjacent_window;
  // one-body terms: every (p, q, spin) is laid down so that set_one_body can change h
  for (int p = 0; p < L; ++p)
    for (int q = 0; q < L; ++q)
      for (int s = 0; s < 2; ++s)
        b.term(1.0, {{2 * p + s, OP_C, 1}, {2 * q + s, OP_A, 1}}, p, q);
  // two-body: 1/2 sum (ik|jl) c+_{i s} c+_{j t} c_{l t} c_{k s}; the pair (is,k) <-> (jt,l)
  // exchange maps a term onto itself, so each unordered pair of pairs is taken once.
  if (two_body) {
    const int64_t L2 = (int64_t)L * L, L3 = L2 * L;
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < L; ++i)
        for (int k = 0; k < L; ++k)
          for (int t = 0; t < 2; ++t)
            for (int j = 0; j < L; ++j)
              for (int l = 0; l < L; ++l) {
                int P1 = ((s * L + i) * L + k), P2 = ((t * L + j) * L + l);
                if (P2 < P1) continue;
                double v = eri[i * L3 + k * L2 + j * L + l];
                if (P1 == P2) continue;  // a+_{is} a+_{is} = 0
                if (v == 0.0) continue;
                b.term(v, {{2 * i + s, OP_C, 1}, {2 * j + t, OP_C, 1}, {2 * l + t, OP_A, 1}, {2 * k + s, OP_A, 1}},
                       -1, -1);
              }
  }
  // constant e0 on the first site
  {
    TransKey tk{0, mk_key(K_I, 0, 0), mk_key(K_H, 0, 0)};
    Mat4& acc = b.coeff[tk];
    for (int s = 0; s < 4; ++s) acc.m[s * 4 + s] += e0;
    b.touch(mk_key(K_I, 0, 0), 0, 0);
    b.touch(mk_key(K_H, 0, 0), 1, L);
  }

  MpoHost M;
  M.L = L;
  M.cut.resize(L + 1);
  M.plain_cls.resize(L + 1);
  if (adjacent_window >= 0) {
    std::vector<std::map<Charge, int>> cnt(L + 1);
    for (auto& kv : b.range_plain)
      for (int c = kv.second.first; c <= kv.second.second; ++c) cnt[c][key_charge(kv.first)]++;
    for (int c = 0; c <= L; ++c)
      for (auto& kv : cnt[c]) M.plain_cls[c].push_back(kv);
  }
  std::vector<std::unordered_map<uint64_t, int>> index(L + 1);
  std::vector<std::vector<uint64_t>> alive(L + 1);
  for (auto& kv : b.range)
    for (int c = kv.second.first; c <= kv.second.second; ++c) alive[c].push_back(kv.first);
  for (int c = 0; c <= L; ++c) {
    auto& ks = alive[c];
    std::sort(ks.begin(), ks.end(), [](uint64_t x, uint64_t y) {
      Charge cx = key_charge(x), cy = key_charge(y);
      if (cx != cy) return cx < cy;
      return key_order(x) < key_order(y);
    });
    MpoCut& cu = M.cut[c];
    cu.key = ks;
    for (size_t k = 0; k < ks.size(); ++k) {
      index[c][ks[k]] = (int)k;
      cu.q.push_back(key_charge(ks[k]));
      cu.parity.push_back((int8_t)key_parity(ks[k]));
      if (cu.cls_q.empty() || cu.cls_q.back() != cu.q.back()) {
        cu.cls_q.push_back(cu.q.back());
        cu.cls_start.push_back((int)k);
        cu.cls_count.push_back(0);
      }
      cu.cls_count.back()++;
      cu.cls_of.push_back((int)cu.cls_q.size() - 1);
    }
    if (adjacent_window < 0)
      for (size_t k = 0; k < cu.cls_q.size(); ++k) M.plain_cls[c].push_back({cu.cls_q[k], cu.cls_count[k]});
  }

  // assemble per-site transitions: structural + pass-through + coefficient sums
  struct Rec {
    double fixed[16];
    bool used[16];
  };
  std::vector<std::unordered_map<uint64_t, Rec>> recs(L);
  auto rec_at = [&](int p, uint64_t kin, uint64_t kout) -> Rec& {
    uint64_t key = (uint64_t)index[p + 1].at(kout) << 32 | (uint32_t)index[p].at(kin);
    auto it = recs[p].find(key);
    if (it == recs[p].end()) {
      Rec r;
      for (int e = 0; e < 16; ++e) {
        r.fixed[e] = 0;
        r.used[e] = false;
      }
      it = recs[p].emplace(key, r).first;
    }
    return it->second;
  };
  for (auto& kv : b.structural) {
    Rec& r = rec_at(kv.first.site, kv.first.kin, kv.first.kout);
    for (int e = 0; e < 16; ++e)
      if (kv.second.m[e] != 0.0) {
        r.fixed[e] = kv.second.m[e];
        r.used[e] = true;
      }
  }
  b.structural.clear();
  for (int p = 0; p < L; ++p)
    for (auto& kv : index[p]) {
      auto it = index[p + 1].find(kv.first);
      if (it == index[p + 1].end()) continue;
      Rec& r = rec_at(p, kv.first, kv.first);
      int par = key_parity(kv.first);
      for (int s = 0; s < 4; ++s) {
        r.fixed[s * 4 + s] = (par && local_parity(s)) ? -1.0 : 1.0;
        r.used[s * 4 + s] = true;
      }
    }
  for (auto& kv : b.coeff) {
    Rec& r = rec_at(kv.first.site, kv.first.kin, kv.first.kout);
    for (int e = 0; e < 16; ++e)
      if (kv.second.m[e] != 0.0) {
        r.fixed[e] += kv.second.m[e];
        r.used[e] = true;
      }
  }
  b.coeff.clear();
  for (auto& ob : b.onebody) {
    Rec& r = rec_at(ob.tk.site, ob.tk.kin, ob.tk.kout);
    for (int e = 0; e < 16; ++e)
      if (ob.m.m[e] != 0.0) r.used[e] = true;
  }
  M.W.resize(L);
  M.c_fixed.resize(L);
  for (int p = 0; p < L; ++p) {
    std::vector<std::pair<uint64_t, const Rec*>> sorted;
    sorted.reserve(recs[p].size());
    for (auto& kv : recs[p]) sorted.push_back({kv.first, &kv.second});
    std::sort(sorted.begin(), sorted.end(), [](auto& x, auto& y) { return x.first < y.first; });
    for (auto& sr : sorted) {
      int w = (int)(uint32_t)sr.first, v = (int)(sr.first >> 32);
      for (int e = 0; e < 16; ++e)
        if (sr.second->used[e]) {
          M.W[p].push_back({w, v, (int8_t)(e / 4), (int8_t)(e % 4), sr.second->fixed[e]});
          M.c_fixed[p].push_back(sr.second->fixed[e]);
        }
    }
    recs[p].clear();
  }
  auto entry_index = [&](int p, int w, int v, int e) {
    const auto& Wp = M.W[p];
    auto it = std::lower_bound(Wp.begin(), Wp.end(), std::make_tuple(v, w, e), [](const MpoEntry& x, const std::tuple<int, int, int>& k) {
      return std::make_tuple(x.v, x.w, x.s * 4 + x.sp) < k;
    });
    TDMPS_REQUIRE(it != Wp.end() && it->v == v && it->w == w && it->s * 4 + it->sp == e, TDMPS_ERR_NUMERIC,
                  "internal: one-body entry not found");
    return (int)(it - Wp.begin());
  };
  for (auto& ob : b.onebody) {
    int p = ob.tk.site;
    int w = index[p].at(ob.tk.kin), v = index[p + 1].at(ob.tk.kout);
    for (int e = 0; e < 16; ++e)
      if (ob.m.m[e] != 0.0) M.onebody.push_back({p, entry_index(p, w, v, e), (int16_t)ob.p, (int16_t)ob.q, ob.m.m[e]});
  }
  mpo_set_one_body(M, h);
  return M;
}

void mpo_set_one_body(MpoHost& m, const double* h) {
  const int L = m.L;
  for (int64_t i = 0; i < (int64_t)L * L; ++i)
    TDMPS_REQUIRE(std::isfinite(h[i]), TDMPS_ERR_NUMERIC, "non-finite one-body integral");
  m.h.assign(h, h + (size_t)L * L);
  for (int p = 0; p < L; ++p)
    for (size_t e = 0; e < m.W[p].size(); ++e) m.W[p][e].c = m.c_fixed[p][e];
  for (auto& r : m.onebody) m.W[r.site][r.entry].c += h[r.p * L + r.q] * r.factor;
  m.version = next_mpo_version();
}

uint64_t next_mpo_version() {
  static std::atomic<uint64_t> counter{0};
  return ++counter;
}

// Dense operator by contracting the channels left to right (tiny L only).
void mpo_to_dense(const MpoHost& m, double* out) {
  const int L = m.L;
  TDMPS_REQUIRE(L <= 6, TDMPS_ERR_ARG, "mpo_to_dense supports L <= 6");
  std::vector<std::vector<double>> T(1, std::vector<double>(1, 1.0));  // channel -> dim x dim
  int64_t dim = 1;
  for (int p = 0; p < L; ++p) {
    int64_t nd = dim * 4;
    std::vector<std::vector<double>> U(m.cut[p + 1].size(), std::vector<double>(nd * nd, 0.0));
    for (auto& e : m.W[p]) {
      const auto& A = T[e.w];
      auto& B = U[e.v];
      for (int64_t r = 0; r < dim; ++r)
        for (int64_t c = 0; c < dim; ++c) {
          double a = A[r * dim + c];
          if (a == 0.0) continue;
          B[(r * 4 + e.s) * nd + (c * 4 + e.sp)] += a * e.c;
        }
    }
    T.swap(U);
    dim = nd;
  }
  std::copy(T[0].begin(), T[0].end(), out);
}

double mpo_det_element(const MpoHost& m, const uint8_t* bra, const uint8_t* ket) {
  std::vector<double> env(1, 1.0);
  for (int p = 0; p < m.L; ++p) {
    TDMPS_REQUIRE(bra[p] < 4 && ket[p] < 4, TDMPS_ERR_ARG, "occupation codes must be 0..3");
    std::vector<double> nxt(m.cut[p + 1].size(), 0.0);
    for (auto& e : m.W[p])
      if (e.s == bra[p] && e.sp == ket[p]) nxt[e.v] += env[e.w] * e.c;
    env.swap(nxt);
  }
  return env[0];
}

}  // namespace tdmps
