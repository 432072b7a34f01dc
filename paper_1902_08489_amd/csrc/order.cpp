// Orbital ordering by a Fiedler reduction of the band width of the coupling between orbitals
// (the ordering used for the molecular orbitals of the H2O results).  The coupling of
// orbitals i != j is w_ij = |h_ij| + |(ij|ji)| (one-body hopping and exchange); the ordering
// sorts the orbitals by the components of the Fiedler vector, the eigenvector of the second
// smallest eigenvalue of the graph Laplacian diag(sum_j w_ij) - w, which places strongly
// coupled orbitals next to each other (small band width of w in the new order).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"

namespace tdmps {
namespace {

// Cyclic Jacobi eigen-decomposition of a real symmetric n x n matrix (row-major):
// A = Q diag(w) Q^T.
void sym_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto at = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) (r == c ? tot : off) += at(r, c) * at(r, c);
    if (off <= 1e-30 * (tot + off) || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double g = at(p, q);
        if (g == 0.0) continue;
        const double zeta = (at(q, q) - at(p, p)) / (2 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        const double c = 1 / std::sqrt(1 + t * t), s = c * t;
        for (int k = 0; k < n; ++k) {
          const double x = at(k, p), y = at(k, q);
          at(k, p) = c * x - s * y;
          at(k, q) = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = at(p, k), y = at(q, k);
          at(p, k) = c * x - s * y;
          at(q, k) = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = Q[(size_t)k * n + p], y = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = c * x - s * y;
          Q[(size_t)k * n + q] = s * x + c * y;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = at(i, i);
}

}  // namespace

std::vector<int> fiedler_order(int L, const double* h, const double* eri) {
  TDMPS_REQUIRE(L >= 1, TDMPS_ERR_ARG, "need L >= 1");
  std::vector<int> perm(L);
  std::iota(perm.begin(), perm.end(), 0);
  if (L <= 2) return perm;
  const int64_t L2 = (int64_t)L * L, L3 = L2 * L;
  std::vector<double> lap((size_t)L * L, 0.0);
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      if (i == j) continue;
      double w = std::fabs(h[(size_t)i * L + j]);
      if (eri) w += std::fabs(eri[i * L3 + j * L2 + j * L + i]);  // exchange (ij|ji)
      TDMPS_REQUIRE(std::isfinite(w), TDMPS_ERR_NUMERIC, "non-finite integral");
      lap[(size_t)i * L + j] -= w;
      lap[(size_t)i * L + i] += w;
    }
  std::vector<double> ev, Q;
  sym_eig(L, lap, ev, Q);
  std::vector<int> idx(L);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ev[a] < ev[b]; });
  const int f = idx[1];
  std::vector<double> v(L);
  for (int i = 0; i < L; ++i) v[i] = Q[(size_t)i * L + f];
  // fix the sign so that the result does not depend on the solver: first orbital goes first
  if (v[0] > v[L - 1]) for (double& x : v) x = -x;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return v[a] < v[b]; });
  return perm;
}

}  // namespace tdmps
