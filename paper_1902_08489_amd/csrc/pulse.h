// Field-driven RK4 propagation and its amplitude gradient (adjoint of the discrete map).
#pragma once

#include <memory>
#include <vector>

#include "drivers.h"

namespace tdmps {

struct PulseRun {
  // H(t) = H0 + A f(t) M, f(t) = sin(omega t) exp(-(t - t_center)^2 / (2 width^2))
  double amplitude = 0, omega = 0, t_center = 0, width = 1;
  double dt = 0;
  int nsteps = 0, every = 1;  // RK4 steps, checkpoint interval
  tdmps_fit_params prm{};
  std::vector<double> h0, m;  // one-body integrals of H0 and of the coupling M (L x L)
  // H at the stage times, one operator per half-step index (time = index * dt / 2): a pool of
  // four whose least recently used member is rewritten, so that H(t + dt) of one step is H(t)
  // of the next (and of the previous one in the adjoint pass) without a new operator version
  static constexpr int NFIELD = 4;
  MpoHost field[NFIELD];
  int64_t field_key[NFIELD] = {-1, -1, -1, -1};
  uint64_t field_used[NFIELD] = {0, 0, 0, 0};
  uint64_t field_clock = 0;
  MpoHost M, mu;              // coupling operator and observable
  std::vector<std::unique_ptr<Mps>> ckpt;  // psi_0, psi_every, ...
  std::unique_ptr<Mps> last;               // psi_N
  double value = 0, norm2 = 0;             // D and |psi_N|^2
};

// Propagates psi0 over r.nsteps RK4 steps, keeping checkpoints; sets r.value = D.
void pulse_forward(Contractor& C, PulseRun& r, const Mps* psi0);
// dD/dA of the last forward run.
double pulse_backward(Contractor& C, PulseRun& r);

}  // namespace tdmps
