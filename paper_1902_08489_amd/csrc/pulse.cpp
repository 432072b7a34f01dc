// Field-driven RK4 propagation and the gradient of a final dipole with respect to the pulse
// amplitude, by the adjoint of the discrete RK4 map with checkpointed recomputation.
//
// H(t) = H0 + E(t) M with E(t) = A sin(omega t) exp(-(t - tc)^2 / (2 tau^2)): the field enters
// through the one-body integrals of Eq. (hamil), h(t) = h0 + E(t) m.  Observable after N steps
// (the RK4 stage definitions and Eq. (rk_add)): D = <psi_N|mu|psi_N> / <psi_N|psi_N>.
//
// Every step is linear, psi_{n+1} = P_n psi_n, so dD/dA = sum_n 2 Re <lam_{n+1}| dP_n/dA psi_n>
// with lam_N = (mu - D) psi_N / |psi_N|^2 and lam_n = P_n^H lam_{n+1}.  Reverse mode through
// the stages (A_s = -i dt H(t_s), k_s = A_s u_s) gives the stage adjoints
//   kb4 = lam/6, ub4 = A_4^H kb4, kb3 = lam/3 + ub4, ub3 = A_3^H kb3, kb2 = lam/3 + ub3/2,
//   ub2 = A_2^H kb2, kb1 = lam/6 + ub2/2, lam_n = lam + ub2 + ub3 + ub4 + A_1^H kb1,
// and the step's contribution sum_s 2 dt f(t_s) Im <kb_s|M|u_s>.  A_s^H = +i dt H(t_s) since
// H is Hermitian, so the adjoint of an H application is an H application: the backward pass
// runs the same fits, environments and H_eff products as the forward pass.  With MPS at
// full bond dimension the result is the exact derivative of the discrete map.  Below it every
// adjoint stage (A_s^H applied to an MPS, and each sum of MPS) is a fit of its own, truncated
// to Dmax like the forward stages: the result approximates the derivative of the truncated
// map, with an error of the order of the truncation, and does not include the variation of
// the kept singular subspaces with the amplitude.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "pulse.h"

namespace tdmps {
namespace {

double shape(const PulseRun& r, double t) {
  return std::sin(r.omega * t) * std::exp(-(t - r.t_center) * (t - r.t_center) / (2 * r.width * r.width));
}

// H(t) into H: one-body integrals h0 + A f(t) m
void set_field(PulseRun& r, MpoHost& H, double t) {
  const double e = r.amplitude * shape(r, t);
  std::vector<double> h(r.h0.size());
  for (size_t i = 0; i < h.size(); ++i) h[i] = r.h0[i] + e * r.m[i];
  const uint64_t old = H.version;
  mpo_set_one_body(H, h.data());
  bool shared = false;  // the pool starts with copies of H0, all of H0's version
  for (const auto& f : r.field) shared |= &f != &H && f.version == old;
  if (!shared) premix_cache_forget(old);
}

// H at time half * dt / 2 (the RK4 stage times are whole and half steps), from the pool
const MpoHost* field_at(PulseRun& r, int64_t half) {
  int slot = -1;
  for (int i = 0; i < PulseRun::NFIELD; ++i)
    if (r.field_key[i] == half) slot = i;
  if (slot < 0) {
    slot = 0;
    for (int i = 1; i < PulseRun::NFIELD; ++i)
      if (r.field_used[i] < r.field_used[slot]) slot = i;
    set_field(r, r.field[slot], half * r.dt / 2);
    r.field_key[slot] = half;
  }
  r.field_used[slot] = ++r.field_clock;
  return &r.field[slot];
}

Mps* step(Contractor& C, PulseRun& r, const Mps* psi, int n) {
  // three lookups in a pool of four: none of them evicts another of this step
  const MpoHost* Ht = field_at(r, 2 * (int64_t)n);
  const MpoHost* Hm = field_at(r, 2 * (int64_t)n + 1);
  const MpoHost* Ht1 = field_at(r, 2 * (int64_t)n + 2);
  FitOut fo;
  return rk4_step(C, Ht, Hm, Ht1, psi, r.dt, r.prm, &fo);
}

Mps* combine(Contractor& C, const std::vector<FitTerm>& terms, const tdmps_fit_params& prm) {
  return fit(C, nullptr, cplx{1, 0}, nullptr, terms, prm, nullptr);
}

}  // namespace

void pulse_forward(Contractor& C, PulseRun& r, const Mps* psi0) {
  TDMPS_REQUIRE(r.nsteps >= 1 && r.every >= 1, TDMPS_ERR_ARG, "need nsteps >= 1 and checkpoint interval >= 1");
  r.ckpt.clear();
  // optional progress lines on stderr (TDMPS_PROGRESS set): one per checkpoint interval
  const bool progress = std::getenv("TDMPS_PROGRESS") != nullptr;
  const double t0 = wall_seconds();
  std::unique_ptr<Mps> psi(mps_clone(psi0));
  for (int n = 0; n < r.nsteps; ++n) {
    if (n % r.every == 0) r.ckpt.emplace_back(mps_clone(psi.get()));
    psi.reset(step(C, r, psi.get(), n));
    if (progress && ((n + 1) % r.every == 0 || n + 1 == r.nsteps))
      std::fprintf(stderr, "pulse: forward step %d of %d after %.1f s\n", n + 1, r.nsteps, wall_seconds() - t0);
  }
  r.last = std::move(psi);
  r.norm2 = overlap(C, r.last.get(), r.last.get()).x;
  TDMPS_REQUIRE(r.norm2 > 0 && std::isfinite(r.norm2), TDMPS_ERR_NUMERIC, "propagated state has zero norm");
  r.value = sandwich(C, r.mu, r.last.get(), r.last.get()).x / r.norm2;
}

double pulse_backward(Contractor& C, PulseRun& r) {
  TDMPS_REQUIRE(r.last && !r.ckpt.empty(), TDMPS_ERR_ARG, "no forward trajectory");
  const double dt = r.dt;
  // lam_N = (mu - D) psi_N / |psi_N|^2
  std::unique_ptr<Mps> lam(fit(C, &r.mu, cplx{1.0 / r.norm2, 0}, r.last.get(),
                               {{cplx{-r.value / r.norm2, 0}, r.last.get()}}, r.prm, nullptr));
  double grad = 0;
  const cplx adj{0.0, dt};  // A_s^H = +i dt H(t_s)
  const cplx fwd{0.0, -dt};
  const bool progress = std::getenv("TDMPS_PROGRESS") != nullptr;
  const double t0 = wall_seconds();
  for (int seg = (int)r.ckpt.size() - 1; seg >= 0; --seg) {
    if (progress)
      std::fprintf(stderr, "pulse: adjoint segment %d of %d after %.1f s\n", (int)r.ckpt.size() - seg,
                   (int)r.ckpt.size(), wall_seconds() - t0);
    const int n0 = seg * r.every, n1 = std::min(r.nsteps, n0 + r.every);
    // recompute psi_n0 .. psi_{n1-1} from the checkpoint
    std::vector<std::unique_ptr<Mps>> states;
    states.emplace_back(mps_clone(r.ckpt[seg].get()));
    for (int n = n0; n + 1 < n1; ++n) states.emplace_back(step(C, r, states.back().get(), n));
    for (int n = n1 - 1; n >= n0; --n) {
      const Mps* psi = states[n - n0].get();
      const double t = n * dt;
      const MpoHost* Ht = field_at(r, 2 * (int64_t)n);
      const MpoHost* Hm = field_at(r, 2 * (int64_t)n + 1);
      const MpoHost* Ht1 = field_at(r, 2 * (int64_t)n + 2);
      // forward stages
      std::unique_ptr<Mps> k1(fit(C, Ht, fwd, psi, {}, r.prm, nullptr));
      std::unique_ptr<Mps> u2(combine(C, {{cplx{1, 0}, psi}, {cplx{0.5, 0}, k1.get()}}, r.prm));
      k1.reset();
      std::unique_ptr<Mps> k2(fit(C, Hm, fwd, u2.get(), {}, r.prm, nullptr));
      std::unique_ptr<Mps> u3(combine(C, {{cplx{1, 0}, psi}, {cplx{0.5, 0}, k2.get()}}, r.prm));
      k2.reset();
      std::unique_ptr<Mps> k3(fit(C, Hm, fwd, u3.get(), {}, r.prm, nullptr));
      std::unique_ptr<Mps> u4(combine(C, {{cplx{1, 0}, psi}, {cplx{1, 0}, k3.get()}}, r.prm));
      k3.reset();
      // stage adjoints
      std::unique_ptr<Mps> kb4(mps_clone(lam.get()));
      scale_mps(C.ctx, kb4.get(), cplx{1.0 / 6, 0});
      std::unique_ptr<Mps> ub4(fit(C, Ht1, adj, kb4.get(), {}, r.prm, nullptr));
      std::unique_ptr<Mps> kb3(combine(C, {{cplx{1.0 / 3, 0}, lam.get()}, {cplx{1, 0}, ub4.get()}}, r.prm));
      std::unique_ptr<Mps> ub3(fit(C, Hm, adj, kb3.get(), {}, r.prm, nullptr));
      std::unique_ptr<Mps> kb2(combine(C, {{cplx{1.0 / 3, 0}, lam.get()}, {cplx{0.5, 0}, ub3.get()}}, r.prm));
      std::unique_ptr<Mps> ub2(fit(C, Hm, adj, kb2.get(), {}, r.prm, nullptr));
      std::unique_ptr<Mps> kb1(combine(C, {{cplx{1.0 / 6, 0}, lam.get()}, {cplx{0.5, 0}, ub2.get()}}, r.prm));
      // gradient of this step: 2 dt sum_s f(t_s) Im <kb_s|M|u_s>
      // the stage times of the operators above (half-step indices 2n, 2n + 1, 2n + 1, 2n + 2)
      const double th = (2 * (int64_t)n + 1) * dt / 2, t1 = (2 * (int64_t)n + 2) * dt / 2;
      const double fs[4] = {shape(r, t), shape(r, th), shape(r, th), shape(r, t1)};
      const Mps* kb[4] = {kb1.get(), kb2.get(), kb3.get(), kb4.get()};
      const Mps* us[4] = {psi, u2.get(), u3.get(), u4.get()};
      for (int s = 0; s < 4; ++s)
        if (fs[s] != 0.0) grad += 2 * dt * fs[s] * sandwich(C, r.M, kb[s], us[s]).y;
      // lam_n = lam + ub2 + ub3 + ub4 + A_1^H kb1
      std::unique_ptr<Mps> a1(fit(C, Ht, adj, kb1.get(), {}, r.prm, nullptr));
      lam.reset(combine(C,
                        {{cplx{1, 0}, lam.get()},
                         {cplx{1, 0}, ub2.get()},
                         {cplx{1, 0}, ub3.get()},
                         {cplx{1, 0}, ub4.get()},
                         {cplx{1, 0}, a1.get()}},
                        r.prm));
    }
  }
  return grad;
}

}  // namespace tdmps
