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

// Lowest generalised eigenpair of the Krylov matrices: coefficients c (c^H N c = 1) and energy.
std::vector<std::complex<double>> krylov_lowest(int m, const std::vector<std::complex<double>>& N,
                                                const std::vector<std::complex<double>>& H, bool orthogonal,
                                                double* energy);

// Ground state by restarted Krylov (Lanczos) iterations: each restart builds an orthogonal
// basis of m states from the current iterate and replaces it by the lowest Ritz state
// (normalised); energy = the last Ritz value.
Mps* krylov_ground(Contractor& C, const MpoHost* H, const Mps* psi, int m, int restarts, const tdmps_fit_params& prm,
                   double* energy);

// c_{site, spin} psi (spin 0 = up, 1 = down), exact: sign strings on the sites left of site,
// the local annihilator on site, bonds right of site relabelled by the removed charge.
Mps* mps_annihilate(Ctx* ctx, const Mps* psi, int site, int spin);

// gamma_pq = sum_s <psi|a+_{ps} a_{qs}|psi> / <psi|psi>, L*L row-major.
std::vector<std::complex<double>> one_rdm(Contractor& C, const Mps* psi);

}  // namespace tdmps
