// Batched Householder QR (FP64) used to precondition the Jacobi SVD.
//
// One-sided Jacobi on a matrix G converges slowly when the singular values of G are graded
// (an entanglement spectrum decays exponentially) or G is rank deficient.  Running it on
// X = R^H instead, where G = Q R is a QR factorisation, removes most of those sweeps
// (preconditioned Jacobi SVD of Drmac and Veselic).  G is ell x k with n = min(ell, k); R is
// n x k (upper trapezoidal) and X = R^H is k x n.  With X V = W (orthogonal columns of norms
// sigma) the SVD of G is G = (Q [V; 0]) Sigma (W Sigma^{-1})^H: the ell-side vectors Q [V; 0]
// are orthonormal to rounding, the k-side ones W Sigma^{-1} only to eps sigma_max / sigma.
//
// Reflectors H = I - tau v v^H with real tau = 2 / |v|^2 and v[j] = 1 (H Hermitian and unitary);
// H maps column x (rows j..ell-1) to beta e_j with beta = -e^{i arg x_j} |x|.  Columns are
// factorised in panels of 16; the panel product H_1 ... H_16 = I - V T V^H (compact WY, T upper
// triangular) is kept per panel so that the trailing columns and later Q itself can be applied
// with 16 x 16 MFMA tiles.
#include <hip/hip_runtime.h>

#include <string>

#include "common.h"
#include "kernels.h"

namespace tdmps {
namespace {

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(TDMPS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int QB = QR_PANEL;  // panel width
static_assert(QB == 16, "16 x 16 MFMA tiles");

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Factorise columns j0 .. j0+nb-1 < n of every matrix (one workgroup of 256 threads per matrix):
// reflectors overwrite the panel below the diagonal, R its upper part, and T of the panel is
// written to m.T[j0 / 16].  Columns right of the panel are left for qr_apply_kernel.
__global__ __launch_bounds__(256) void qr_panel_kernel(const QrMat* __restrict__ mats, int j0) {
  const QrMat m = mats[blockIdx.x];
  if (j0 >= m.nsv) return;  // uniform
  const int nb = min(QB, m.nsv - j0);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double2* G = (double2*)m.G;
  const int64_t ld = m.ell;
  __shared__ double part[4][2 * QB];
  __shared__ double2 red[QB];
  __shared__ double2 Ts[QB][QB];
  __shared__ double tau_s[QB];
  for (int e = t; e < QB * QB; e += 256) Ts[e / QB][e % QB] = make_double2(0.0, 0.0);
  for (int j = 0; j < nb; ++j) {
    const int col = j0 + j;
    double2* x = G + col * ld;
    // |x[col+1 ..]|^2
    double s = 0;
    for (int r = col + 1 + t; r < m.ell; r += 256) s += x[r].x * x[r].x + x[r].y * x[r].y;
    s = wsum(s);
    __syncthreads();  // previous users of part[] are done
    if (lane == 0) part[wave][0] = s;
    __syncthreads();
    const double xs = (part[0][0] + part[1][0]) + (part[2][0] + part[3][0]);
    const double2 alpha = x[col];
    const double aa = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);
    double tau = 0;
    double2 inv0 = make_double2(0.0, 0.0);
    if (xs > 0) {
      const double nrm = sqrt(aa * aa + xs);
      const double2 ph = aa > 0 ? make_double2(alpha.x / aa, alpha.y / aa) : make_double2(1.0, 0.0);
      const double v0m = aa + nrm;  // v0 = ph * (|alpha| + |x|)
      // 1 / v0 = conj(ph) / (|alpha| + |x|)
      inv0 = make_double2(ph.x / v0m, -ph.y / v0m);
      tau = 2.0 / (1.0 + xs / (v0m * v0m));
      __syncthreads();
      if (t == 0) x[col] = make_double2(-ph.x * nrm, -ph.y * nrm);  // beta
      for (int r = col + 1 + t; r < m.ell; r += 256) {
        const double2 v = x[r];
        x[r] = make_double2(v.x * inv0.x - v.y * inv0.y, v.x * inv0.y + v.y * inv0.x);
      }
    }
    if (t == 0) tau_s[j] = tau;
    __syncthreads();
    // dots: d_c = v^H g_c for the panel columns right of j, e_i = v_i^H v for i < j
    const int nd = nb - 1;  // (nb - 1 - j) columns + j reflectors
    if (nd > 0) {
      double acc[2 * (QB - 1)];
#pragma unroll
      for (int q = 0; q < 2 * (QB - 1); ++q) acc[q] = 0;
      if (tau != 0) {
        for (int r = col + t; r < m.ell; r += 256) {
          const double2 v = r == col ? make_double2(1.0, 0.0) : x[r];
#pragma unroll
          for (int q = 0; q < QB - 1; ++q) {
            if (q < nd) {
              // q < j: reflector i = q (rows > j0 + i below the unit entry; r > j0 + q here);
              // else panel column j0 + 1 + q
              const double2 y = G[(j0 + q + (q < j ? 0 : 1)) * ld + r];
              const double2 z = q < j ? cmulc(y, v) : cmulc(v, y);  // v_i^H v or v^H g_c
              acc[2 * q] += z.x;
              acc[2 * q + 1] += z.y;
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 2 * (QB - 1); ++q) {
        if (q < 2 * nd) {
          const double v = wsum(acc[q]);
          if (lane == 0) part[wave][q] = v;
        }
      }
      __syncthreads();
      if (t < nd) red[t] = make_double2((part[0][2 * t] + part[1][2 * t]) + (part[2][2 * t] + part[3][2 * t]),
                                        (part[0][2 * t + 1] + part[1][2 * t + 1]) +
                                            (part[2][2 * t + 1] + part[3][2 * t + 1]));
      __syncthreads();
      // g_c -= tau v d_c for the remaining panel columns
      if (tau != 0) {
        for (int c = j + 1; c < nb; ++c) {
          const double2 d = red[c - 1];
          const double2 f = make_double2(tau * d.x, tau * d.y);
          double2* g = G + (j0 + c) * ld;
          for (int r = col + t; r < m.ell; r += 256) {
            const double2 v = r == col ? make_double2(1.0, 0.0) : x[r];
            const double2 gv = g[r];
            g[r] = make_double2(gv.x - (v.x * f.x - v.y * f.y), gv.y - (v.x * f.y + v.y * f.x));
          }
        }
      }
    }
    // T[0:j, j] = -tau_j T[0:j, 0:j] e, T[j][j] = tau_j
    if (t == 0) {
      for (int a = 0; a < j; ++a) {
        double sr = 0, si = 0;
        for (int b = a; b < j; ++b) {
          const double2 tv = Ts[a][b], ev = red[b];
          sr += tv.x * ev.x - tv.y * ev.y;
          si += tv.x * ev.y + tv.y * ev.x;
        }
        Ts[a][j] = make_double2(-tau * sr, -tau * si);
      }
      Ts[j][j] = make_double2(tau, 0.0);
    }
    __syncthreads();
  }
  double2* T = (double2*)m.T + (int64_t)(j0 / QB) * QB * QB;
  for (int e = t; e < QB * QB; e += 256) T[e] = Ts[e / QB][e % QB];
}

// Register-resident variant of qr_panel_kernel for panels of at most 256 * RPT rows (RPT <= 4;
// taller panels would spill and use qr_panel_kernel): thread t
// holds rows j0 + t + 256 i (i < RPT) of the 16 panel columns, so a reflector step costs two
// workgroup reductions and no memory traffic; the panel is read once and written once.
template <int RPT>
__global__ __launch_bounds__(256) void qr_panel_reg_kernel(const QrMat* __restrict__ mats, int j0) {
  const QrMat m = mats[blockIdx.x];
  if (j0 >= m.nsv) return;  // uniform
  const int nb = min(QB, m.nsv - j0);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double2* G = (double2*)m.G;
  const int64_t ld = m.ell;
  __shared__ double part[4][2 * QB];
  __shared__ double2 red[QB];
  __shared__ double2 Ts[QB][QB];
  __shared__ double2 bc;
  double2 x[RPT][QB];
#pragma clang loop unroll(full)
  for (int i = 0; i < RPT; ++i) {
    const int row = j0 + t + 256 * i;
#pragma clang loop unroll(full)
    for (int c = 0; c < QB; ++c)
      x[i][c] = (row < m.ell && c < nb) ? G[(j0 + c) * ld + row] : make_double2(0.0, 0.0);
  }
  for (int e = t; e < QB * QB; e += 256) Ts[e / QB][e % QB] = make_double2(0.0, 0.0);
#pragma clang loop unroll(full)
  for (int j = 0; j < QB; ++j) {
    if (j < nb) {
      const int col = j0 + j;
      // |x[col+1 ..]|^2 and the diagonal element
      double s = 0;
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i) {
        const int row = j0 + t + 256 * i;
        if (row > col && row < m.ell) s += x[i][j].x * x[i][j].x + x[i][j].y * x[i][j].y;
      }
      s = wsum(s);
      __syncthreads();  // previous users of part[], bc and red[] are done
      if (lane == 0) part[wave][0] = s;
#pragma clang loop unroll(full)
      for (int i = 0; i < RPT; ++i)
        if (j0 + t + 256 * i == col) bc = x[i][j];
      __syncthreads();
      const double xs = (part[0][0] + part[1][0]) + (part[2][0] + part[3][0]);
      const double2 alpha = bc;
      const double aa = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);
      double tau = 0;
      if (xs > 0) {
        const double nrm = sqrt(aa * aa + xs);
        const double2 ph = aa > 0 ? make_double2(alpha.x / aa, alpha.y / aa) : make_double2(1.0, 0.0);
        const double v0m = aa + nrm;
        const double2 inv0 = make_double2(ph.x / v0m, -ph.y / v0m);
        tau = 2.0 / (1.0 + xs / (v0m * v0m));
#pragma clang loop unroll(full)
        for (int i = 0; i < RPT; ++i) {
          const int row = j0 + t + 256 * i;
          const double2 v = x[i][j];
          if (row == col)
            x[i][j] = make_double2(-ph.x * nrm, -ph.y * nrm);
          else if (row > col)
            x[i][j] = make_double2(v.x * inv0.x - v.y * inv0.y, v.x * inv0.y + v.y * inv0.x);
        }
      }
      const int nd = nb - 1;
      if (nd > 0) {
        double acc[2 * (QB - 1)];
#pragma clang loop unroll(full)
        for (int q = 0; q < 2 * (QB - 1); ++q) acc[q] = 0;
        if (tau != 0) {
#pragma clang loop unroll(full)
          for (int i = 0; i < RPT; ++i) {
            const int row = j0 + t + 256 * i;
            if (row >= col && row < m.ell) {
              const double2 v = row == col ? make_double2(1.0, 0.0) : x[i][j];
#pragma clang loop unroll(full)
              for (int q = 0; q < QB - 1; ++q) {
                if (q < nd) {
                  // q < j: reflector q (row > j0 + q here); else panel column q + 1
                  const double2 y = x[i][q < j ? q : q + 1];
                  const double2 z = q < j ? cmulc(y, v) : cmulc(v, y);
                  acc[2 * q] += z.x;
                  acc[2 * q + 1] += z.y;
                }
              }
            }
          }
        }
#pragma clang loop unroll(full)
        for (int q = 0; q < 2 * (QB - 1); ++q) {
          if (q < 2 * nd) {
            const double v = wsum(acc[q]);
            if (lane == 0) part[wave][q] = v;
          }
        }
        __syncthreads();
        if (t < nd)
          red[t] = make_double2((part[0][2 * t] + part[1][2 * t]) + (part[2][2 * t] + part[3][2 * t]),
                                (part[0][2 * t + 1] + part[1][2 * t + 1]) + (part[2][2 * t + 1] + part[3][2 * t + 1]));
        __syncthreads();
        if (tau != 0) {
#pragma clang loop unroll(full)
          for (int c = j + 1; c < QB; ++c) {
            if (c < nb) {
              const double2 d = red[c - 1];
              const double2 f = make_double2(tau * d.x, tau * d.y);
#pragma clang loop unroll(full)
              for (int i = 0; i < RPT; ++i) {
                const int row = j0 + t + 256 * i;
                if (row >= col && row < m.ell) {
                  const double2 v = row == col ? make_double2(1.0, 0.0) : x[i][j];
                  x[i][c] = make_double2(x[i][c].x - (v.x * f.x - v.y * f.y), x[i][c].y - (v.x * f.y + v.y * f.x));
                }
              }
            }
          }
        }
      }
      // T[0:j, j] = -tau_j T[0:j, 0:j] e, T[j][j] = tau_j
      if (t == 0) {
        for (int a = 0; a < j; ++a) {
          double sr = 0, si = 0;
          for (int b = a; b < j; ++b) {
            const double2 tv = Ts[a][b], ev = red[b];
            sr += tv.x * ev.x - tv.y * ev.y;
            si += tv.x * ev.y + tv.y * ev.x;
          }
          Ts[a][j] = make_double2(-tau * sr, -tau * si);
        }
        Ts[j][j] = make_double2(tau, 0.0);
      }
    }
  }
#pragma clang loop unroll(full)
  for (int i = 0; i < RPT; ++i) {
    const int row = j0 + t + 256 * i;
    if (row < m.ell)
#pragma clang loop unroll(full)
      for (int c = 0; c < QB; ++c)
        if (c < nb) G[(j0 + c) * ld + row] = x[i][c];
  }
  __syncthreads();
  double2* T = (double2*)m.T + (int64_t)(j0 / QB) * QB * QB;
  for (int e = t; e < QB * QB; e += 256) T[e] = Ts[e / QB][e % QB];
}

// Apply the block reflector of panel j0 to 16-column blocks.  mode 0: trailing columns of G,
// A <- (I - V T V^H)^H A for the columns j0 + nb .. k-1 right of the panel; mode 1:
// A <- (I - V T V^H) A on the n columns of m.B (ell x n).  Only rows j0 .. ell-1 change.  Y = V^H A and the update A -= V Z (Z = T^H Y
// or T Y) run on the f64 MFMA units; lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[l/16 + 4e][l%16].
__global__ __launch_bounds__(256) void qr_apply_kernel(const QrMat* __restrict__ mats, int nmats, int j0, int mode) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double2 Yp[4][QB][QB + 1];
  __shared__ double2 Zs[QB][QB + 1];
  int lo = 0, hi = nmats - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mats[mid].cb_base <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const QrMat m = mats[lo];
  const int c0 = QB * ((int)blockIdx.x - m.cb_base);
  if (j0 >= m.nsv) return;
  const int nb = min(QB, m.nsv - j0);
  if (mode == 0 && c0 + QB <= j0 + nb) return;  // block inside the panel
  const int ncol = mode == 0 ? m.k : m.nsv;
  if (c0 >= ncol) return;
  const int cmin = mode == 0 ? j0 + nb : 0;  // first column to update
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int64_t ld = m.ell;
  const double2* Vp = (const double2*)m.G + j0 * ld;  // reflector j of the panel: column j0 + j
  double2* A = (double2*)(mode == 0 ? m.G : m.B);
  auto vget = [&](int r, int j) -> double2 {  // V[r][j], r absolute row
    if (j >= nb) return make_double2(0.0, 0.0);
    const int d = j0 + j;
    if (r < d || r >= m.ell) return make_double2(0.0, 0.0);
    if (r == d) return make_double2(1.0, 0.0);
    return Vp[j * ld + r];
  };
  auto aget = [&](int r, int c) -> double2 {
    return (r < m.ell && c < ncol) ? A[(int64_t)c * ld + r] : make_double2(0.0, 0.0);
  };
  // Y = V^H A over rows j0 .. ell-1, 4-row steps split over the waves
  {
    v4d r1 = {0, 0, 0, 0}, r2 = r1, i1 = r1, i2 = r1;
    const int nsteps = (m.ell - j0 + 3) >> 2;
    for (int s = wave; s < nsteps; s += 4) {
      const int r = j0 + 4 * s + lq;
      const double2 v = vget(r, l16), a = aget(r, c0 + l16);
      r1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, a.x, r1, 0, 0, 0);
      r2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v.y, a.y, r2, 0, 0, 0);
      i1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, a.y, i1, 0, 0, 0);
      i2 = __builtin_amdgcn_mfma_f64_16x16x4f64(-v.y, a.x, i2, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Yp[wave][lq + 4 * e][l16] = make_double2(r1[e] + r2[e], i1[e] + i2[e]);
  }
  __syncthreads();
  {
    const int a = t >> 4, b = t & 15;
    const double2* T = (const double2*)m.T + (int64_t)(j0 / QB) * QB * QB;
    double zr = 0, zi = 0;
    for (int c = 0; c < QB; ++c) {
      const double2 y0 = Yp[0][c][b], y1 = Yp[1][c][b], y2 = Yp[2][c][b], y3 = Yp[3][c][b];
      const double yr = (y0.x + y1.x) + (y2.x + y3.x), yi = (y0.y + y1.y) + (y2.y + y3.y);
      double2 tv;
      if (mode == 0) {  // (T^H)[a][c] = conj(T[c][a])
        tv = T[c * QB + a];
        tv.y = -tv.y;
      } else {
        tv = T[a * QB + c];
      }
      zr += tv.x * yr - tv.y * yi;
      zi += tv.x * yi + tv.y * yr;
    }
    Zs[a][b] = make_double2(zr, zi);
  }
  __syncthreads();
  // A -= V Z in 16-row tiles
  double zr[4], zi[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 z = Zs[4 * s + lq][l16];
    zr[s] = z.x;
    zi[s] = z.y;
  }
  const int ntiles = (m.ell - j0 + 15) >> 4;
  for (int tile = wave; tile < ntiles; tile += 4) {
    const int rbase = j0 + 16 * tile;
    v4d ar = {0, 0, 0, 0}, ai = ar, br = ar, bi = ar;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double2 v = vget(rbase + l16, 4 * s + lq);
      ar = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, zr[s], ar, 0, 0, 0);
      ai = __builtin_amdgcn_mfma_f64_16x16x4f64(v.x, zi[s], ai, 0, 0, 0);
      br = __builtin_amdgcn_mfma_f64_16x16x4f64(v.y, -zi[s], br, 0, 0, 0);
      bi = __builtin_amdgcn_mfma_f64_16x16x4f64(v.y, zr[s], bi, 0, 0, 0);
    }
    const int c = c0 + l16;
    if (c < ncol && c >= cmin) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rbase + lq + 4 * e;
        if (r < m.ell) {
          double2* p = A + (int64_t)c * ld + r;
          const double2 o = *p;
          *p = make_double2(o.x - (ar[e] + br[e]), o.y - (ai[e] + bi[e]));
        }
      }
    }
  }
}

// X = R^H (k x n, column-major, lower trapezoidal) from the R factor in the upper part of G.
__global__ __launch_bounds__(256) void qr_rt_kernel(const QrMat* __restrict__ mats) {
  const QrMat m = mats[blockIdx.x];
  const double2* G = (const double2*)m.G;
  double2* X = (double2*)m.X;
  const int64_t n = (int64_t)m.k * m.nsv;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int c = (int)(e / m.k), r = (int)(e - (int64_t)c * m.k);
    double2 v = make_double2(0.0, 0.0);
    if (r >= c) {
      v = G[(int64_t)r * m.ell + c];  // R[c][r]
      v.y = -v.y;
    }
    X[e] = v;
  }
}

// After the Jacobi sweeps on X (accumulated rotations in m.V, n x n): B = [V; 0] (ell x n) and
// X <- X Sigma^{-1} (columns of norm sigma_c > 0 become unit vectors; zero columns stay zero).
__global__ __launch_bounds__(256) void qr_finish_kernel(const QrMat* __restrict__ mats, const double* __restrict__ sigma,
                                                        int max_k) {
  const QrMat m = mats[blockIdx.x];
  const double* sg = sigma + (int64_t)blockIdx.x * max_k;
  double2* X = (double2*)m.X;
  const double2* V = (const double2*)m.V;
  double2* B = (double2*)m.B;
  const int64_t nx = (int64_t)m.k * m.nsv;
  for (int64_t e = threadIdx.x; e < nx; e += blockDim.x) {
    const int c = (int)(e / m.k);
    const double s = sg[c];
    const double inv = s > 0 ? 1.0 / s : 0.0;
    const double2 x = X[e];
    X[e] = make_double2(x.x * inv, x.y * inv);
  }
  const int64_t nb = (int64_t)m.ell * m.nsv;
  for (int64_t e = threadIdx.x; e < nb; e += blockDim.x) {
    const int c = (int)(e / m.ell), r = (int)(e - (int64_t)c * m.ell);
    B[e] = r < m.nsv ? V[(int64_t)c * m.nsv + r] : make_double2(0.0, 0.0);
  }
}

}  // namespace

void launch_qr_panel(const QrMat* mats, int nmats, int j0, int max_rows, void* stream) {
  if (nmats <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  if (max_rows <= 256)
    hipLaunchKernelGGL(qr_panel_reg_kernel<1>, dim3(nmats), dim3(256), 0, s, mats, j0);
  else if (max_rows <= 512)
    hipLaunchKernelGGL(qr_panel_reg_kernel<2>, dim3(nmats), dim3(256), 0, s, mats, j0);
  else if (max_rows <= 1024)
    hipLaunchKernelGGL(qr_panel_reg_kernel<4>, dim3(nmats), dim3(256), 0, s, mats, j0);
  else
    hipLaunchKernelGGL(qr_panel_kernel, dim3(nmats), dim3(256), 0, s, mats, j0);
  check(hipGetLastError(), "qr panel launch");
}

void launch_qr_apply(const QrMat* mats, int nmats, int total_blocks, int j0, int mode, void* stream) {
  if (nmats <= 0 || total_blocks <= 0) return;
  hipLaunchKernelGGL(qr_apply_kernel, dim3(total_blocks), dim3(256), 0, (hipStream_t)stream, mats, nmats, j0, mode);
  check(hipGetLastError(), "qr apply launch");
}

void launch_qr_rt(const QrMat* mats, int nmats, void* stream) {
  if (nmats <= 0) return;
  hipLaunchKernelGGL(qr_rt_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, mats);
  check(hipGetLastError(), "qr rt launch");
}

void launch_qr_finish(const QrMat* mats, int nmats, const double* sigma, int max_k, void* stream) {
  if (nmats <= 0) return;
  hipLaunchKernelGGL(qr_finish_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, mats, sigma, max_k);
  check(hipGetLastError(), "qr finish launch");
}

}  // namespace tdmps
