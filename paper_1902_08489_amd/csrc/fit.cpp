// Variational fit (Methods, Eq. (add_min)): C ~ alpha H psi + sum_j beta_j phi_j.
//
// Two-site sweeps with C kept in mixed-canonical form.  At bond (i, i+1) the optimal
// two-site tensor is the projection of the target on the local basis, obtained from the
// left/right environments of <C|H|psi> and <C|phi_j>:
//   theta_C = alpha H_eff theta_psi + sum_j beta_j L^{C phi_j} theta_phi_j R^{C phi_j},
// which is then truncated by SVD and split.  A sweep is a left-to-right pass over the
// bonds followed by a right-to-left pass.  The initial guess is the first operand,
// right-canonicalised.  With grow_on_h the first left-to-right pass projects alpha H psi
// alone: a target orthogonal to psi (the orthogonal Krylov vectors) has no projection on the
// bases of a product-state guess, so the bases are first grown on H psi, which contains psi.
#include <algorithm>
#include <cmath>
#include <memory>

#include "engine.h"

namespace tdmps {
namespace {

struct Term {
  const MpoHost* op;
  const Mps* ket;
  cplx coef;
  std::vector<std::unique_ptr<Env>> Lenv, Renv;  // indexed by bond
};

Env build_left(Contractor& C, const MpoHost& O, const Env& E, int i, const Mps* bra, const Mps* ket,
               std::unique_ptr<SideOps>* keep) {
  auto ops = std::make_unique<SideOps>(premix_left(C, E, O, i));
  Env N = env_left_update(C, *ops, bra, bra->site[i].c(), bra->lay[i], bra->bond[i], bra->bond[i + 1],
                          ket->site[i].c(), ket->lay[i], ket->bond[i], ket->bond[i + 1], O);
  if (keep) *keep = std::move(ops);
  return N;
}

Env build_right(Contractor& C, const MpoHost& O, const Env& E, int i, const Mps* bra, const Mps* ket) {
  SideOps ops = premix_right(C, E, O, i);
  return env_right_update(C, ops, bra->site[i].c(), bra->lay[i], bra->bond[i], bra->bond[i + 1], ket->site[i].c(),
                          ket->lay[i], ket->bond[i], ket->bond[i + 1], O);
}

}  // namespace

Mps* fit(Contractor& C, const MpoHost* H, cplx alpha, const Mps* psi, const std::vector<FitTerm>& terms,
         const tdmps_fit_params& prm, FitOut* info, bool grow_on_h) {
  TDMPS_REQUIRE(H || !terms.empty(), TDMPS_ERR_ARG, "nothing to fit");
  const Mps* first = H ? psi : terms[0].phi;
  const int L = first->L;
  TDMPS_REQUIRE(L >= 2, TDMPS_ERR_ARG, "L must be >= 2");
  TDMPS_REQUIRE(prm.Dmax >= 1 && prm.n_sweeps >= 1, TDMPS_ERR_ARG, "Dmax and n_sweeps must be >= 1");
  for (auto& t : terms) {
    TDMPS_REQUIRE(t.phi->L == L, TDMPS_ERR_ARG, "operands differ in length");
    TDMPS_REQUIRE(t.phi->total == first->total, TDMPS_ERR_SECTOR, "operands differ in total charge");
  }
  if (H) TDMPS_REQUIRE(H->L == L, TDMPS_ERR_ARG, "operator and state differ in length");
  std::unique_ptr<Mps> Cm(mps_clone(first));
  right_canonicalize(C, Cm.get(), prm.svd_cutoff);
  std::vector<MpoHost> idm;
  idm.push_back(identity_mpo(L));
  std::vector<Term> T;
  if (H) T.push_back({H, psi, alpha, {}, {}});
  for (auto& t : terms) T.push_back({&idm[0], t.phi, t.beta, {}, {}});
  for (auto& t : T) {
    t.Lenv.resize(L + 1);
    t.Renv.resize(L + 1);
    t.Lenv[0].reset(new Env(env_left_boundary(C.ctx, Cm->bond[0], t.ket->bond[0])));
    t.Renv[L].reset(new Env(env_right_boundary(C.ctx, Cm->bond[L], t.ket->bond[L], L)));
    for (int i = L - 1; i >= 2; --i)
      t.Renv[i].reset(new Env(build_right(C, *t.op, *t.Renv[i + 1], i, Cm.get(), t.ket)));
  }
  FitOut out;
  double prev = -1;
  for (int sweep = 0; sweep < prm.n_sweeps; ++sweep) {
    out.disc_sum = 0;
    double last_norm = 0;
    for (int dir = 0; dir < 2; ++dir) {
      for (int step = 0; step < L - 1; ++step) {
        int i = dir == 0 ? step : L - 2 - step;
        TwoLayout bl;
        bl.build(Cm->bond[i], Cm->bond[i + 2]);
        DevBuf theta(std::max<int64_t>(bl.size, 1) * sizeof(cplx));
        std::vector<std::unique_ptr<SideOps>> lkeep(T.size()), rkeep(T.size());
        // at the last local problem of a sweep, every term's output alone (for <out|H|psi> and
        // <out|phi_j>); the two-site tensors there are tiny (bond 0 has dimension one)
        const bool last_bond = dir == 1 && i == 0;
        std::vector<std::vector<cplx>> local(last_bond ? T.size() : 0);
        bool first_term = true;
        const bool h_only = grow_on_h && H && sweep == 0 && dir == 0;
        for (size_t k = 0; k < T.size(); ++k) {
          Term& t = T[k];
          if (h_only && k > 0) {  // left environment of the term still advances with the sweep
            lkeep[k] = std::make_unique<SideOps>(premix_left(C, *t.Lenv[i], *t.op, i));
            continue;
          }
          TwoLayout kl;
          kl.build(t.ket->bond[i], t.ket->bond[i + 2]);
          DevBuf tin(std::max<int64_t>(kl.size, 1) * sizeof(cplx));
          form_theta(C, t.ket, i, tin.c(), kl);
          lkeep[k] = std::make_unique<SideOps>(premix_left(C, *t.Lenv[i], *t.op, i));
          rkeep[k] = std::make_unique<SideOps>(premix_right(C, *t.Renv[i + 2], *t.op, i + 1));
          if (last_bond && bl.size) {
            DevBuf part(bl.size * sizeof(cplx));
            heff_apply(C, *lkeep[k], *rkeep[k], tin.c(), kl, t.ket->bond[i], t.ket->bond[i + 2], part.c(), bl,
                       Cm->bond[i], Cm->bond[i + 2], cplx{1, 0}, false, nullptr);
            local[k].resize(bl.size);
            dev_d2h(local[k].data(), part.c(), bl.size * sizeof(cplx), C.ctx->stream);
          }
          double alg = 0;
          heff_apply(C, *lkeep[k], *rkeep[k], tin.c(), kl, t.ket->bond[i], t.ket->bond[i + 2], theta.c(), bl,
                     Cm->bond[i], Cm->bond[i + 2], t.coef, !first_term, t.op == H ? &alg : nullptr);
          C.heff_alg_flops += alg;
          first_term = false;
        }
        TruncResult tr = split_theta(C, theta.c(), bl, Cm.get(), i, prm.Dmax, prm.svd_cutoff, dir == 0);
        if (last_bond) {
          // bonds 0 and 2 of the result are unchanged by the split, so the final two-site
          // tensor has the layout of theta
          std::vector<cplx> fin(bl.size);
          if (bl.size) {
            DevBuf tf(bl.size * sizeof(cplx));
            form_theta(C, Cm.get(), 0, tf.c(), bl);
            dev_d2h(fin.data(), tf.c(), bl.size * sizeof(cplx), C.ctx->stream);
          }
          auto dot = [&](const std::vector<cplx>& v) {
            double re = 0, im = 0;
            for (int64_t x = 0; x < (int64_t)v.size(); ++x) {
              re += fin[x].x * v[x].x + fin[x].y * v[x].y;
              im += fin[x].x * v[x].y - fin[x].y * v[x].x;
            }
            return cplx{re, im};
          };
          out.term_overlaps.clear();
          for (size_t k = 0; k < T.size(); ++k) {
            const cplx d = dot(local[k]);
            if (H && k == 0)
              out.h_out_psi = d;
            else
              out.term_overlaps.push_back(d);
          }
        }
        out.disc_max = std::max(out.disc_max, tr.discarded);
        out.disc_sum += tr.discarded;
        last_norm = tr.norm2;
        for (size_t k = 0; k < T.size(); ++k) {
          Term& t = T[k];
          if (dir == 0) {
            t.Lenv[i + 1].reset(new Env(env_left_update(
                C, *lkeep[k], Cm.get(), Cm->site[i].c(), Cm->lay[i], Cm->bond[i], Cm->bond[i + 1], t.ket->site[i].c(),
                t.ket->lay[i], t.ket->bond[i], t.ket->bond[i + 1], *t.op)));
          } else {
            t.Renv[i + 1].reset(new Env(env_right_update(
                C, *rkeep[k], Cm->site[i + 1].c(), Cm->lay[i + 1], Cm->bond[i + 1], Cm->bond[i + 2],
                t.ket->site[i + 1].c(), t.ket->lay[i + 1], t.ket->bond[i + 1], t.ket->bond[i + 2], *t.op)));
          }
        }
      }
    }
    out.sweeps = sweep + 1;
    out.norm2 = last_norm;
    if (prm.conv_tol > 0 && prev >= 0 && std::fabs(last_norm - prev) <= prm.conv_tol * std::max(last_norm, 1e-300))
      break;
    prev = last_norm;
  }
  C.fit_discarded += out.disc_sum;
  if (info) *info = out;
  return Cm.release();
}

}  // namespace tdmps
