// One-particle reduced density matrix gamma_pq = sum_s <psi|a+_{ps} a_{qs}|psi> / <psi|psi>
// (the accuracy measure of the time-evolved states in the H2O results) for all p, q in one
// left-to-right sweep.
//
// The state is brought into right-canonical form, so the part right of any cut contracts to
// the identity.  The left environments of the one-body MPO with all coefficients equal to one
// then carry, in each channel with a single open operator a+_{ps} (or a_{ps}) left of the cut,
// the partial contraction of that operator with its Jordan-Wigner string.  At site q every
// transition of the MPO that completes a term (open operator -> complete, or identity ->
// complete for the on-site terms) is redirected to an output channel of its own; one
// environment update with these transitions gives, per output channel, a matrix whose trace
// is the expectation value of that term.  The cost is one environment update per site for the
// propagation and one for the closing, O(L^2 D^3) over the sweep instead of O(L^3 D^3) for L^2
// separate expectation values.
#include <algorithm>
#include <cmath>
#include <complex>
#include <memory>

#include "drivers.h"

namespace tdmps {
namespace {

using zd = std::complex<double>;

// Closing operator at site q: cut q of O, and at cut q + 1 one channel per completing term.
// kind_out[c] / p_out[c]: 0 = gamma_{p q} (open creator p), 1 = gamma_{q p} (open annihilator
// p), 2 = gamma_{q q}.
MpoHost closing_mpo(const MpoHost& O, int q, std::vector<int>& kind_out, std::vector<int>& p_out) {
  MpoHost X;
  X.L = O.L;
  X.cut = O.cut;
  X.W.resize(O.L);
  X.c_fixed.resize(O.L);
  const MpoCut& in = O.cut[q];
  const MpoCut& out = O.cut[q + 1];
  int hch = -1;
  for (int v = 0; v < out.size(); ++v) {
    int so, op;
    if (mpo_channel_kind(out.key[v], &so, &op) == 1) hch = v;
  }
  TDMPS_REQUIRE(hch >= 0, TDMPS_ERR_ARG, "internal: no complete channel in the one-body operator");
  // output channel per source channel (open operator or identity)
  std::vector<int> dst(in.size(), -1);
  kind_out.clear();
  p_out.clear();
  for (const MpoEntry& e : O.W[q]) {
    if (e.v != hch || dst[e.w] >= 0) continue;
    int so = 0, op = 0;
    const int k = mpo_channel_kind(in.key[e.w], &so, &op);
    if (k == 0) {
      kind_out.push_back(2);
      p_out.push_back(q);
    } else if (k == 2 && op <= 1) {
      kind_out.push_back(op);
      p_out.push_back(so >> 1);
    } else {
      continue;  // completed terms from the left (H -> H) are not wanted
    }
    dst[e.w] = (int)kind_out.size() - 1;
  }
  MpoCut oc;
  const int n = (int)kind_out.size();
  for (int c = 0; c < n; ++c) {
    oc.key.push_back((uint64_t)c);
    oc.q.push_back(Charge(0, 0));
    oc.parity.push_back(0);
    oc.cls_of.push_back(0);
  }
  if (n > 0) {
    oc.cls_q = {Charge(0, 0)};
    oc.cls_start = {0};
    oc.cls_count = {n};
  }
  X.cut[q + 1] = oc;
  for (const MpoEntry& e : O.W[q])
    if (e.v == hch && dst[e.w] >= 0) {
      MpoEntry f = e;
      f.v = dst[e.w];
      X.W[q].push_back(f);
      X.c_fixed[q].push_back(e.c);
    }
  std::sort(X.W[q].begin(), X.W[q].end(), [](const MpoEntry& a, const MpoEntry& b) {
    if (a.v != b.v) return a.v < b.v;
    if (a.w != b.w) return a.w < b.w;
    if (a.s != b.s) return a.s < b.s;
    return a.sp < b.sp;
  });
  return X;
}

}  // namespace

std::vector<zd> one_rdm(Contractor& C, const Mps* psi) {
  const int L = psi->L;
  std::unique_ptr<Mps> rc(mps_clone(psi));
  right_canonicalize(C, rc.get(), 0.0);
  const double n2 = overlap(C, rc.get(), rc.get()).x;
  TDMPS_REQUIRE(n2 > 0 && std::isfinite(n2), TDMPS_ERR_NUMERIC, "state has zero or non-finite norm");
  std::vector<double> ones((size_t)L * L, 1.0);
  const MpoHost O = build_mpo(L, ones.data(), nullptr, 0.0, false);
  std::vector<zd> g((size_t)L * L, zd(0));
  Env E = env_left_boundary(C.ctx, rc->bond[0], rc->bond[0]);
  const Mps* m = rc.get();
  for (int q = 0; q < L; ++q) {
    std::vector<int> kind, pp;
    const MpoHost X = closing_mpo(O, q, kind, pp);
    if (!kind.empty()) {
      SideOps ops = premix_left(C, E, X, q);
      Env out = env_left_update(C, ops, m, m->site[q].c(), m->lay[q], m->bond[q], m->bond[q + 1], m->site[q].c(),
                                m->lay[q], m->bond[q], m->bond[q + 1], X);
      // trace of every output channel over the bond (bra and ket bases coincide)
      std::vector<cplx> h((size_t)out.b.size);
      if (out.b.size) dev_d2h(h.data(), out.b.data.p, h.size() * sizeof(cplx), C.ctx->stream);
      const Bond& b = m->bond[q + 1];
      const StackGroup& sg = out.b.grp[0];
      for (int c = 0; c < (int)kind.size(); ++c) {
        zd tr = 0;
        for (int s = 0; s < b.nsec(); ++s) {
          if (sg.off[s] < 0) continue;
          const int64_t D = b.dim[s];
          const cplx* blk = h.data() + sg.off[s] + (int64_t)c * D * D;
          for (int64_t i = 0; i < D; ++i) tr += zd(blk[i * D + i].x, blk[i * D + i].y);
        }
        const int p = pp[c];
        if (kind[c] == 0)
          g[(size_t)p * L + q] += tr;
        else if (kind[c] == 1)
          g[(size_t)q * L + p] += tr;
        else
          g[(size_t)q * L + q] += tr;
      }
    }
    SideOps ops = premix_left(C, E, O, q);
    Env nxt = env_left_update(C, ops, m, m->site[q].c(), m->lay[q], m->bond[q], m->bond[q + 1], m->site[q].c(),
                              m->lay[q], m->bond[q], m->bond[q + 1], O);
    E = std::move(nxt);
  }
  for (auto& x : g) x /= n2;
  return g;
}

}  // namespace tdmps
