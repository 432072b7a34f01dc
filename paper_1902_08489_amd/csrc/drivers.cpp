// Time steps built from the fit: RK4 (the RK4 stage definitions and Eq. (rk_add)) and Krylov (Eqs. (kry_non),
// (kry_orth), (krylov_evo)).  The m x m Krylov algebra runs on the host in FP64.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <memory>

#include "drivers.h"

namespace tdmps {

using zd = std::complex<double>;

namespace {

// Cyclic Jacobi for a Hermitian n x n matrix (row-major): A = Q diag(w) Q^H.
void herm_eig(int n, std::vector<zd> A, std::vector<double>& w, std::vector<zd>& Q) {
  Q.assign((size_t)n * n, zd(0));
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  auto at = [&](int r, int c) -> zd& { return A[(size_t)r * n + c]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) (r == c ? tot : off) += std::norm(at(r, c));
    if (off <= 1e-30 * (tot + off) || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        zd g = at(p, q);
        double ag = std::abs(g);
        if (ag == 0.0) continue;
        double a = at(p, p).real(), b = at(q, q).real();
        zd ph = g / ag;  // e^{i phi}
        double zeta = (b - a) / (2 * ag);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        double c = 1 / std::sqrt(1 + t * t), s = c * t;
        // J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
        zd em = std::conj(ph);
        for (int k = 0; k < n; ++k) {  // columns: A <- A J
          zd x = at(k, p), y = at(k, q);
          at(k, p) = c * x - s * em * y;
          at(k, q) = s * x + c * em * y;
        }
        for (int k = 0; k < n; ++k) {  // rows: A <- J^H A
          zd x = at(p, k), y = at(q, k);
          at(p, k) = c * x - s * ph * y;
          at(q, k) = s * x + c * ph * y;
        }
        for (int k = 0; k < n; ++k) {
          zd x = Q[(size_t)k * n + p], y = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = c * x - s * em * y;
          Q[(size_t)k * n + q] = s * x + c * em * y;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = at(i, i).real();
}

}  // namespace

namespace {

// Generalised Hermitian eigenproblem of the Krylov matrices, H V = N V diag(lam), V^H N V = 1,
// on the directions where N is not numerically singular (orthogonal mode: all of them).
void krylov_eig(int m, const std::vector<zd>& Nin, const std::vector<zd>& Hin, bool orthogonal, std::vector<zd>& V,
                std::vector<double>& lam, int& r, std::vector<zd>& Nsym) {
  std::vector<zd> N(Nin), H(Hin);
  for (int a = 0; a < m; ++a)
    for (int c = a; c < m; ++c) {
      zd x = 0.5 * (N[a * m + c] + std::conj(N[c * m + a]));
      N[a * m + c] = x;
      N[c * m + a] = std::conj(x);
      zd y = 0.5 * (H[a * m + c] + std::conj(H[c * m + a]));
      H[a * m + c] = y;
      H[c * m + a] = std::conj(y);
    }
  std::vector<double> nw;
  std::vector<zd> Q;
  herm_eig(m, N, nw, Q);
  double nmax = 0;
  for (double x : nw) nmax = std::max(nmax, x);
  TDMPS_REQUIRE(nmax > 0, TDMPS_ERR_SINGULAR, "Krylov overlap matrix is zero");
  std::vector<int> keep;
  for (int i = 0; i < m; ++i) {
    if (nw[i] > 1e-12 * nmax)
      keep.push_back(i);
    else
      TDMPS_REQUIRE(!orthogonal, TDMPS_ERR_SINGULAR, "Krylov overlap matrix is not positive definite");
  }
  r = (int)keep.size();
  // X = Q_keep diag(n^-1/2): X^H N X = 1
  std::vector<zd> X((size_t)m * r);
  for (int a = 0; a < m; ++a)
    for (int j = 0; j < r; ++j) X[a * r + j] = Q[a * m + keep[j]] / std::sqrt(nw[keep[j]]);
  std::vector<zd> Hp((size_t)r * r, zd(0));
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      zd s = 0;
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) s += std::conj(X[a * r + i]) * H[a * m + b] * X[b * r + j];
      Hp[i * r + j] = s;
    }
  std::vector<zd> Y;
  herm_eig(r, Hp, lam, Y);
  V.assign((size_t)m * r, zd(0));
  for (int a = 0; a < m; ++a)
    for (int j = 0; j < r; ++j) {
      zd s = 0;
      for (int i = 0; i < r; ++i) s += X[a * r + i] * Y[i * r + j];
      V[a * r + j] = s;
    }
  Nsym = N;
}

}  // namespace

std::vector<zd> krylov_coefficients(int m, const std::vector<zd>& Nin, const std::vector<zd>& Hin, double dt,
                                    bool orthogonal) {
  std::vector<zd> V, N;
  std::vector<double> lam;
  int r = 0;
  krylov_eig(m, Nin, Hin, orthogonal, V, lam, r, N);
  // c = V exp(-i dt lam) V^H N e0
  std::vector<zd> y(r);
  for (int j = 0; j < r; ++j) {
    zd s = 0;
    for (int a = 0; a < m; ++a) s += std::conj(V[a * r + j]) * N[a * m + 0];
    y[j] = s * std::exp(zd(0, -dt * lam[j]));
  }
  std::vector<zd> c(m);
  for (int a = 0; a < m; ++a) {
    zd s = 0;
    for (int j = 0; j < r; ++j) s += V[a * r + j] * y[j];
    c[a] = s;
  }
  return c;
}

std::vector<zd> krylov_lowest(int m, const std::vector<zd>& Nin, const std::vector<zd>& Hin, bool orthogonal,
                              double* energy) {
  std::vector<zd> V, N;
  std::vector<double> lam;
  int r = 0;
  krylov_eig(m, Nin, Hin, orthogonal, V, lam, r, N);
  int jmin = 0;
  for (int j = 1; j < r; ++j)
    if (lam[j] < lam[jmin]) jmin = j;
  if (energy) *energy = lam[jmin];
  std::vector<zd> c(m);
  for (int a = 0; a < m; ++a) c[a] = V[a * r + jmin];
  return c;
}

Mps* rk4_step(Contractor& C, const MpoHost* Ht, const MpoHost* Hm, const MpoHost* Ht1, const Mps* psi, double dt,
              const tdmps_fit_params& prm, FitOut* info) {
  cplx a{0.0, -dt};
  FitOut fo, acc;
  auto track = [&](const FitOut& f) {
    acc.sweeps = std::max(acc.sweeps, f.sweeps);
    acc.disc_max = std::max(acc.disc_max, f.disc_max);
    acc.disc_sum += f.disc_sum;
  };
  std::unique_ptr<Mps> k1(fit(C, Ht, a, psi, {}, prm, &fo));
  track(fo);
  std::unique_ptr<Mps> u2(fit(C, nullptr, a, nullptr, {{cplx{1, 0}, psi}, {cplx{0.5, 0}, k1.get()}}, prm, &fo));
  track(fo);
  std::unique_ptr<Mps> k2(fit(C, Hm, a, u2.get(), {}, prm, &fo));
  track(fo);
  u2.reset();
  std::unique_ptr<Mps> u3(fit(C, nullptr, a, nullptr, {{cplx{1, 0}, psi}, {cplx{0.5, 0}, k2.get()}}, prm, &fo));
  track(fo);
  std::unique_ptr<Mps> k3(fit(C, Hm, a, u3.get(), {}, prm, &fo));
  track(fo);
  u3.reset();
  std::unique_ptr<Mps> u4(fit(C, nullptr, a, nullptr, {{cplx{1, 0}, psi}, {cplx{1, 0}, k3.get()}}, prm, &fo));
  track(fo);
  std::unique_ptr<Mps> k4(fit(C, Ht1, a, u4.get(), {}, prm, &fo));
  track(fo);
  u4.reset();
  Mps* out = fit(C, nullptr, a, nullptr,
                 {{cplx{1, 0}, psi},
                  {cplx{1.0 / 6, 0}, k1.get()},
                  {cplx{1.0 / 3, 0}, k2.get()},
                  {cplx{1.0 / 3, 0}, k3.get()},
                  {cplx{1.0 / 6, 0}, k4.get()}},
                 prm, &fo);
  track(fo);
  acc.norm2 = fo.norm2;
  if (info) *info = acc;
  return out;
}

// Krylov basis of Eqs. (kry_orth)/(kry_non): phi^0 = psi/|psi|, each next vector fitted from
// H phi^k (minus the projections on all previous vectors in the orthogonal mode) and
// normalised; N and H (m x m, row-major) from overlaps and sandwiches.  The orthogonal basis
// stops early when the space is invariant: when the component of H phi^k orthogonal to the
// basis is below 1e-10 of H phi^k (e.g. psi an eigenstate), only meff = k + 1 vectors are
// kept (unused rows and columns of N and H stay 0).
struct KrylovBasis {
  std::vector<std::unique_ptr<Mps>> phi;
  std::vector<zd> N, H;
  int meff = 0;
  double s0 = 0;  // |psi|
};

static KrylovBasis krylov_basis(Contractor& C, const MpoHost* H, const Mps* psi, int m, bool orthogonal,
                                const tdmps_fit_params& prm) {
  TDMPS_REQUIRE(m >= 2 && m <= 64, TDMPS_ERR_ARG, "Krylov dimension must be in [2, 64]");
  auto z = [](cplx c) { return zd(c.x, c.y); };
  // optional progress lines on stderr (TDMPS_PROGRESS set): one per Krylov vector
  const bool progress = std::getenv("TDMPS_PROGRESS") != nullptr;
  const double t_start = wall_seconds();
  KrylovBasis K;
  double n0 = overlap(C, psi, psi).x;
  TDMPS_REQUIRE(n0 > 0 && std::isfinite(n0), TDMPS_ERR_NUMERIC, "state has zero or non-finite norm");
  K.s0 = std::sqrt(n0);
  auto& phi = K.phi;
  phi.emplace_back(mps_clone(psi));
  scale_mps(C.ctx, phi[0].get(), cplx{1.0 / K.s0, 0.0});
  std::vector<zd>& N = K.N;
  std::vector<zd>& Hm = K.H;
  N.assign((size_t)m * m, zd(0));
  Hm.assign((size_t)m * m, zd(0));
  N[0] = z(overlap(C, phi[0].get(), phi[0].get()));
  MpoHost I = identity_mpo(psi->L);
  auto bras = [&](int n) {
    std::vector<const Mps*> b;
    for (int j = 0; j < n; ++j) b.push_back(phi[j].get());
    return b;
  };
  // Column k of H: <phi_j|H|phi_k> for all j <= k in one batched sweep, except j = k - 1,
  // which the fit that produced phi_k already gave exactly (FitOut::h_out_psi)
  auto column = [&](int k, bool have_prev) {
    std::vector<const Mps*> b;
    std::vector<int> idx;
    for (int j = 0; j <= k; ++j)
      if (!(have_prev && j == k - 1)) {
        b.push_back(phi[j].get());
        idx.push_back(j);
      }
    const std::vector<cplx> hk = sandwich_many(C, *H, b, phi[k].get());
    for (size_t q = 0; q < idx.size(); ++q) {
      const int j = idx[q];
      Hm[j * m + k] = z(hk[q]);
      Hm[k * m + j] = std::conj(Hm[j * m + k]);
    }
  };
  int meff = m;
  for (int k = 0; k < m - 1; ++k) {
    column(k, k > 0);
    double proj = 0;
    for (int j = 0; j <= k; ++j) proj += std::norm(Hm[j * m + k]) / N[j * m + j].real();
    std::vector<FitTerm> terms;
    if (orthogonal)
      for (int j = 0; j <= k; ++j) {
        zd b = -Hm[j * m + k] / N[j * m + j];
        terms.push_back({cplx{b.real(), b.imag()}, phi[j].get()});
      }
    FitOut fo;
    // the orthogonalised target has no overlap with the guess phi_k: grow the bases on H phi_k
    // first (the first left-to-right pass), then fit the whole target
    std::unique_ptr<Mps> nxt(fit(C, H, cplx{1, 0}, phi[k].get(), terms, prm, &fo, orthogonal));
    if (progress)
      std::fprintf(stderr, "krylov: vector %d of %d after %.1f s\n", k + 1, m - 1, wall_seconds() - t_start);
    double nn = overlap(C, nxt.get(), nxt.get()).x;
    TDMPS_REQUIRE(nn >= 0 && std::isfinite(nn), TDMPS_ERR_NUMERIC, "Krylov vector is not finite");
    if (orthogonal && nn <= 1e-20 * (proj + nn)) {
      meff = k + 1;
      break;
    }
    TDMPS_REQUIRE(nn > 0, TDMPS_ERR_SINGULAR, "Krylov vector vanished");
    scale_mps(C.ctx, nxt.get(), cplx{1.0 / std::sqrt(nn), 0.0});
    phi.push_back(std::move(nxt));
    // <phi_{k+1}|H|phi_k> of the normalised vector
    Hm[(k + 1) * m + k] = z(fo.h_out_psi) / std::sqrt(nn);
    Hm[k * m + k + 1] = std::conj(Hm[(k + 1) * m + k]);
    if (orthogonal && fo.term_overlaps.size() == (size_t)(k + 1)) {
      // the fit's terms were phi_0 .. phi_k: their overlaps with the result are exact
      for (int j = 0; j <= k; ++j) {
        N[(k + 1) * m + j] = z(fo.term_overlaps[j]) / std::sqrt(nn);
        N[j * m + k + 1] = std::conj(N[(k + 1) * m + j]);
      }
      N[(k + 1) * m + k + 1] = z(overlap(C, phi[k + 1].get(), phi[k + 1].get()));
    } else {
      const std::vector<cplx> nk = sandwich_many(C, I, bras(k + 2), phi[k + 1].get());
      for (int j = 0; j <= k + 1; ++j) {
        N[j * m + k + 1] = z(nk[j]);
        N[(k + 1) * m + j] = std::conj(N[j * m + k + 1]);
      }
    }
  }
  if (meff == m) column(m - 1, true);
  K.meff = meff;
  return K;
}

static void sub_matrices(const KrylovBasis& K, int m, std::vector<zd>& Ns, std::vector<zd>& Hs) {
  const int e = K.meff;
  Ns.assign((size_t)e * e, zd(0));
  Hs.assign((size_t)e * e, zd(0));
  for (int r = 0; r < e; ++r)
    for (int q = 0; q < e; ++q) {
      Ns[r * e + q] = K.N[r * m + q];
      Hs[r * e + q] = K.H[r * m + q];
    }
}

Mps* krylov_step(Contractor& C, const MpoHost* H, const Mps* psi, double dt, int m, bool orthogonal,
                 const tdmps_fit_params& prm, std::vector<zd>* Nout, std::vector<zd>* Hout) {
  KrylovBasis K = krylov_basis(C, H, psi, m, orthogonal, prm);
  std::vector<zd> Ns, Hs;
  sub_matrices(K, m, Ns, Hs);
  auto c = krylov_coefficients(K.meff, Ns, Hs, dt, orthogonal);
  std::vector<FitTerm> terms;
  for (int k = 0; k < K.meff; ++k)
    terms.push_back({cplx{K.s0 * c[k].real(), K.s0 * c[k].imag()}, K.phi[k].get()});
  Mps* out = fit(C, nullptr, cplx{1, 0}, nullptr, terms, prm, nullptr);
  if (Nout) *Nout = K.N;
  if (Hout) *Hout = K.H;
  return out;
}

Mps* krylov_ground(Contractor& C, const MpoHost* H, const Mps* psi, int m, int restarts, const tdmps_fit_params& prm,
                   double* energy) {
  TDMPS_REQUIRE(restarts >= 1, TDMPS_ERR_ARG, "need at least one restart");
  std::unique_ptr<Mps> cur(mps_clone(psi));
  double E = 0;
  for (int r = 0; r < restarts; ++r) {
    KrylovBasis K = krylov_basis(C, H, cur.get(), m, true, prm);
    std::vector<zd> Ns, Hs;
    sub_matrices(K, m, Ns, Hs);
    auto c = krylov_lowest(K.meff, Ns, Hs, true, &E);
    std::vector<FitTerm> terms;
    for (int k = 0; k < K.meff; ++k) terms.push_back({cplx{c[k].real(), c[k].imag()}, K.phi[k].get()});
    std::unique_ptr<Mps> nxt(fit(C, nullptr, cplx{1, 0}, nullptr, terms, prm, nullptr));
    const double nn = overlap(C, nxt.get(), nxt.get()).x;
    TDMPS_REQUIRE(nn > 0 && std::isfinite(nn), TDMPS_ERR_NUMERIC, "ground-state iterate vanished");
    scale_mps(C.ctx, nxt.get(), cplx{1.0 / std::sqrt(nn), 0.0});
    cur = std::move(nxt);
  }
  if (energy) *energy = E;
  return cur.release();
}

}  // namespace tdmps
