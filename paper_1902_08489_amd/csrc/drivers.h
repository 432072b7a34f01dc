// RK4 and Krylov time steps on top of the fit.
#pragma once

#include <complex>

#include "engine.h"

namespace tdmps {

std::vector<std::complex<double>> krylov_coefficients(int m, const std::vector<std::complex<double>>& N,
                                                      const std::vector<std::complex<double>>& H, double dt,
                                                      bool orthogonal);

Mps* rk4_step(Contractor& C, const MpoHost* Ht, const MpoHost* Hm, const MpoHost* Ht1, const Mps* psi, double dt,
              const tdmps_fit_params& prm, FitOut* info);

Mps* krylov_step(Contractor& C, const MpoHost* H, const Mps* psi, double dt, int m, bool orthogonal,
                 const tdmps_fit_params& prm, std::vector<std::complex<double>>* N,
                 std::vector<std::complex<double>>* Hm);

// gamma_pq = sum_s <psi|a+_{ps} a_{qs}|psi> / <psi|psi>, L*L row-major.
std::vector<std::complex<double>> one_rdm(Contractor& C, const Mps* psi);

}  // namespace tdmps
