// Strided block copies and the batched block one-sided Jacobi SVD (FP64).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <string>

#include "common.h"
#include "kernels.h"

namespace tdmps {
namespace {

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(TDMPS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr int COPY_SPLIT = 8;

__global__ __launch_bounds__(256) void copy_kernel(const CopyTask* __restrict__ tasks) {
  const CopyTask t = tasks[blockIdx.x];
  const int64_t n = (int64_t)t.rows * t.cols;
  const double2* src = (const double2*)t.src;
  double2* dst = (double2*)t.dst;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.y * blockDim.x) {
    int r = (int)(e / t.cols), c = (int)(e - (int64_t)r * t.cols);
    int64_t rr = t.ridx ? t.ridx[r] : r, cc = t.cidx ? t.cidx[c] : c;
    double2 v = src[rr * t.src_rs + cc * t.src_cs];
    if (t.flags & 1) v.y = -v.y;
    double s = 1.0;
    if (t.rscale) s *= t.rscale[r];
    if (t.cscale) s *= t.cscale[c];
    v.x *= s;
    v.y *= s;
    double2* d = dst + (int64_t)r * t.dst_ld + c;
    if (t.flags & 2) {
      double2 o = *d;
      v.x += o.x;
      v.y += o.y;
    }
    *d = v;
  }
}

__global__ void svd_init_kernel(const SvdMat* __restrict__ mats) {
  const SvdMat m = mats[blockIdx.x];
  const int64_t n = (int64_t)m.k * m.k;
  double2* V = (double2*)m.V;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    int a = (int)(e / m.k), b = (int)(e - (int64_t)a * m.k);
    V[e] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int find_mat(const SvdMat* __restrict__ mats, int n, int64_t pair) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (mats[mid].pair_base <= pair)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Circle schedule on n (even) items: pair i of round r is (n-1, r) for i = 0 and
// ((r+i) mod (n-1), (r-i) mod (n-1)) otherwise; every pair meets once in n-1 rounds.
__device__ __forceinline__ void circle_pair(int n, int r, int i, int& p, int& q) {
  if (i == 0) {
    p = n - 1;
    q = r;
  } else {
    p = (r + i) % (n - 1);
    q = (r - i + (n - 1)) % (n - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

constexpr int SVD_PW = 2 * SVD_BLOCK;  // columns of a block pair

// 1/sqrt(x) and 1/x for normal positive x: hardware estimate refined by two Newton steps
// (each step doubles the number of correct bits of the estimate).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

// Rotation that makes columns p, q of a pair orthogonal, from a = |g_p|^2, b = |g_q|^2 and
// gamma = g_p^H g_q: g_p' = c g_p - s e^{-i phi} g_q, g_q' = s g_p + c e^{-i phi} g_q with
// gamma = |gamma| e^{i phi} (the smaller of the two angles that zero the overlap).  A pair is
// rotated iff |gamma| > tol sqrt(a b) and |gamma| > thr sqrt(max(a, b)), tested on squares;
// overlaps below 1e-145 in modulus count as zero.
struct Rot {
  double c, s, er, ei;  // (er, ei) = e^{-i phi}
};

__device__ __forceinline__ bool make_rot(double a, double b, double gr, double gi, double tol, double thr, Rot& R) {
  const double g2 = gr * gr + gi * gi;
  if (!(g2 > tol * tol * (a * b)) || !(g2 > thr * thr * fmax(a, b)) || !(g2 > 1e-290)) return false;
  const double ri = rsq_nr(g2);  // 1 / |gamma|
  const double zeta = 0.5 * (b - a) * ri;
  const double az = fabs(zeta);
  double t;
  if (az > 1e100) {
    t = 0.5 * rcp_nr(az);
  } else {
    const double q = 1.0 + az * az;
    t = rcp_nr(az + q * rsq_nr(q));
  }
  if (zeta < 0) t = -t;
  R.c = rsq_nr(1.0 + t * t);
  R.s = R.c * t;
  R.er = gr * ri;
  R.ei = -gi * ri;
  return true;
}

// One round of the block one-sided Jacobi method.  The columns of every matrix are cut into
// blocks of SVD_BLOCK; workgroup i of round r >= 0 owns block pair i of the circle schedule over
// the blocks, workgroup i of the diagonal round (r < 0) the blocks 2i and 2i + 1, i.e. 16
// columns P.  It forms the Gram matrix M = P^H P on the FP64 MFMA units, rotates the column
// pairs of its round in LDS (M <- J^H M J and Q <- Q J for every pair whose overlap exceeds
// the tolerance, with the same test and rotation as the scalar method) and, if any pair was
// rotated, overwrites P by P Q and the matching 16 columns of V by V Q, again on the MFMA
// units.  M is formed afresh from the columns at every visit, so a sweep without rotations
// certifies the pairwise test on the columns.
//
// MFMA f64 16x16x4 lane layout: lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[l/16 + 4e][l%16] in register e.  For the Gram matrix both operands are the element
// P[4s + l/16][l%16] of the 4-row step s.  Every wave issues the loads of a whole batch of
// steps (tiles) before its first MFMA, so a block pair's panel is in flight at once.
constexpr int SVD_GB = 16;  // Gram: 4-row steps per wave and batch
constexpr int SVD_UB = 4;   // update: 16-row tiles per wave and batch

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVES waves per workgroup (4 or 8): the Gram matrix and the column update are split over
// the waves, the 16 x 16 rotation sweep runs on wave 0.  Small matrices run faster with 4
// (fewer idle waves per barrier), large ones gain nothing from either.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void svd_block_round_kernel(const SvdMat* __restrict__ mats, int nmats,
                                                                         int round, double tol,
                                                                         int32_t* __restrict__ counter,
                                                                         const int32_t* __restrict__ prev) {
  static_assert(SVD_PW == 16, "one 16 x 16 MFMA tile per block pair");
  static_assert(WAVES >= 4, "the Gram reduction uses one thread per element of the 16 x 16 matrix");
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double2 Mp[WAVES][SVD_PW][SVD_PW + 1];  // per-wave partial Gram matrices
  __shared__ double2 Ms[SVD_PW][SVD_PW + 1];
  __shared__ double2 Qs[SVD_PW][SVD_PW + 1];
  __shared__ int col[SVD_PW];
  __shared__ int rotated;
  if (prev != nullptr && *prev == 0) return;  // converged in an earlier sweep (uniform)
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int j = find_mat(mats, nmats, blockIdx.x);
  const SvdMat m = mats[j];
  const int i = (int)(blockIdx.x - m.pair_base);
  const bool diag = round < 0;
  if (round >= m.nblk - 1 || i >= m.nblk / 2) return;  // uniform over the workgroup
  int bI = 2 * i, bJ = 2 * i + 1;
  if (!diag) circle_pair(m.nblk, round, i, bI, bJ);
  if (t < SVD_PW) {
    const int c = (t < SVD_BLOCK ? bI : bJ) * SVD_BLOCK + (t % SVD_BLOCK);
    col[t] = c < m.k ? c : -1;
  }
  if (t == 0) rotated = 0;
  __syncthreads();

  // Gram matrix: wave w takes the 4-row steps w, w + WAVES, ...
  {
    const double2* G = (const double2*)m.G;
    const int c = col[l16];
    const int nsteps = (m.ell + 3) >> 2;
    v4d r1 = {0, 0, 0, 0}, r2 = r1, i1 = r1, i2 = r1;
    for (int s0 = wave; s0 < nsteps; s0 += WAVES * SVD_GB) {
      double2 v[SVD_GB];
#pragma unroll
      for (int u = 0; u < SVD_GB; ++u) {
        const int row = 4 * (s0 + WAVES * u) + lq;
        v[u] = (c >= 0 && row < m.ell) ? G[(int64_t)c * m.ell + row] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < SVD_GB; ++u) {
        r1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u].x, v[u].x, r1, 0, 0, 0);
        i1 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u].x, v[u].y, i1, 0, 0, 0);
        r2 = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u].y, v[u].y, r2, 0, 0, 0);
        i2 = __builtin_amdgcn_mfma_f64_16x16x4f64(-v[u].y, v[u].x, i2, 0, 0, 0);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Mp[wave][lq + 4 * e][l16] = make_double2(r1[e] + r2[e], i1[e] + i2[e]);
  }
  __syncthreads();
  if (t < SVD_PW * SVD_PW) {
    const int a = t >> 4, b = t & 15;
    double sr = 0, si = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      sr += Mp[w][a][b].x;
      si += Mp[w][a][b].y;
    }
    Ms[a][b] = make_double2(sr, a == b ? 0.0 : si);
    Qs[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  // Rotations on M by wave 0 (wave-synchronous LDS): lane l serves pair l / 8; the column step
  // rotates rows l%8 and l%8 + 8 of M and Q, the row step columns l%8, l%8 + 8.  A block-pair
  // round rotates the 64 cross pairs (p in I, q in J) in 8 rounds of 8; the diagonal round of
  // a sweep rotates the pairs inside I and inside J (7 rounds of 4 + 4).  Every column pair
  // is thus rotated once per sweep (a cyclic Jacobi ordering).
  if (wave == 0) {
    const int pr = lane >> 3, sub = lane & 7;
    bool any = false;
    const int nr = diag ? SVD_BLOCK - 1 : SVD_BLOCK;
    for (int r = 0; r < nr; ++r) {
      int p, q;
      if (diag) {
        circle_pair(SVD_BLOCK, r, pr & 3, p, q);
        if (pr >= 4) {
          p += SVD_BLOCK;
          q += SVD_BLOCK;
        }
      } else {
        p = pr;
        q = SVD_BLOCK + ((pr + r) & (SVD_BLOCK - 1));
      }
      Rot R;
      const double2 g = Ms[p][q];
      const bool rot = make_rot(Ms[p][p].x, Ms[q][q].x, g.x, g.y, tol, m.thr, R);
      any |= rot;
      wave_sync();
      if (rot) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double2(*X)[SVD_PW + 1] = u < 2 ? Ms : Qs;
          const int x = sub + 8 * (u & 1);
          const double2 a = X[x][p], b = X[x][q];
          const double br = R.er * b.x - R.ei * b.y, bi = R.er * b.y + R.ei * b.x;  // e^{-i phi} b
          X[x][p] = make_double2(R.c * a.x - R.s * br, R.c * a.y - R.s * bi);
          X[x][q] = make_double2(R.s * a.x + R.c * br, R.s * a.y + R.c * bi);
        }
      }
      wave_sync();
      if (rot) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int y = sub + 8 * u;
          const double2 a = Ms[p][y], b = Ms[q][y];
          const double br = R.er * b.x + R.ei * b.y, bi = R.er * b.y - R.ei * b.x;  // e^{+i phi} b
          Ms[p][y] = make_double2(R.c * a.x - R.s * br, R.c * a.y - R.s * bi);
          Ms[q][y] = make_double2(R.s * a.x + R.c * br, R.s * a.y + R.c * bi);
        }
      }
      wave_sync();
    }
    if (__any(any) && lane == 0) rotated = 1;
  }
  __syncthreads();
  if (!rotated) return;  // uniform: read after the barrier
  if (t == 0) atomicAdd(counter, 1);

  // P <- P Q and V <- V Q in 16-row tiles, wave w taking tiles w, w + WAVES, ...; k-step
  // s of a tile reads column 4s + l/16 at row l%16 (A operand) and keeps Q[4s + l/16][l%16]
  double qr[4], qi[4];
  int cin[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 qv = Qs[4 * s + lq][l16];
    qr[s] = qv.x;
    qi[s] = qv.y;
    cin[s] = col[4 * s + lq];
  }
  const int cout = col[l16];
  for (int pass = 0; pass < 2; ++pass) {
    double2* X = (double2*)(pass == 0 ? m.G : m.V);
    const int len = pass == 0 ? m.ell : m.k;
    const int ntiles = (len + 15) >> 4;
    for (int t0 = wave; t0 < ntiles; t0 += WAVES * SVD_UB) {
      double2 v[SVD_UB][4];
#pragma unroll
      for (int u = 0; u < SVD_UB; ++u) {
        const int row = 16 * (t0 + WAVES * u) + l16;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          v[u][s] = (cin[s] >= 0 && row < len) ? X[(int64_t)cin[s] * len + row] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < SVD_UB; ++u) {
        v4d ar = {0, 0, 0, 0}, ai = ar, br = ar, bi = ar;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          ar = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][s].x, qr[s], ar, 0, 0, 0);
          ai = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][s].x, qi[s], ai, 0, 0, 0);
          br = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][s].y, -qi[s], br, 0, 0, 0);
          bi = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][s].y, qr[s], bi, 0, 0, 0);
        }
        const int tile = t0 + WAVES * u;
        if (cout >= 0) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = 16 * tile + lq + 4 * e;
            if (row < len) X[(int64_t)cout * len + row] = make_double2(ar[e] + br[e], ai[e] + bi[e]);
          }
        }
      }
    }
  }
}

// One workgroup row per task; the y dimension strides over the elements of the block.
__global__ __launch_bounds__(256) void share_kernel(const ShareTask* __restrict__ tasks,
                                                    const double* __restrict__ coef) {
  const ShareTask t = tasks[blockIdx.x];
  const double* cf = coef + t.coff;
  const double2* X = (const double2*)t.X;
  double2* T = (double2*)t.T;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < t.blk; e += (int64_t)gridDim.y * 256) {
    double2 x[SHARE_MAXQ];
#pragma unroll
    for (int q = 0; q < SHARE_MAXQ; ++q) x[q] = q < t.nq ? X[q * t.blk + e] : make_double2(0.0, 0.0);
    for (int j = 0; j < t.nrun; ++j) {
      float2* T32 = (float2*)t.T + j * t.blk + e;  // out32: the FP32 storage of the mixed precisions
      double2 s = make_double2(0.0, 0.0);
      if (t.accum) {
        if (t.out32)
          s = make_double2(T32->x, T32->y);
        else
          s = T[j * t.blk + e];
      }
#pragma unroll
      for (int q = 0; q < SHARE_MAXQ; ++q)
        if (q < t.nq) {
          const double c = cf[j * t.nq + q];
          s.x += c * x[q].x;
          s.y += c * x[q].y;
        }
      if (t.out32)
        *T32 = make_float2((float)s.x, (float)s.y);
      else
        T[j * t.blk + e] = s;
    }
  }
}

__global__ __launch_bounds__(256) void svd_norms_kernel(const SvdMat* __restrict__ mats, int nmats, int maxk,
                                                        double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (gw >= (int64_t)nmats * maxk) return;
  const int j = (int)(gw / maxk), col = (int)(gw - (int64_t)j * maxk);
  const SvdMat m = mats[j];
  if (col >= m.k) return;
  const double2* g = (const double2*)m.G + (int64_t)col * m.ell;
  double s = 0;
  for (int e = lane; e < m.ell; e += 64) s += g[e].x * g[e].x + g[e].y * g[e].y;
  s = wave_sum(s);
  if (lane == 0) out[gw] = sqrt(s);
}

}  // namespace

void launch_copy(const CopyTask* tasks, int ntasks, void* stream) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(ntasks, COPY_SPLIT), dim3(256), 0, (hipStream_t)stream, tasks);
  check(hipGetLastError(), "copy launch");
}

void launch_share(const ShareTask* tasks, const double* coef, int ntasks, int64_t max_blk, void* stream) {
  if (ntasks <= 0 || max_blk <= 0) return;
  const int64_t y = std::min<int64_t>(64, (max_blk + 1023) / 1024);
  hipLaunchKernelGGL(share_kernel, dim3(ntasks, (unsigned)std::max<int64_t>(1, y)), dim3(256), 0, (hipStream_t)stream,
                     tasks, coef);
  check(hipGetLastError(), "share launch");
}

void launch_svd_init(const SvdMat* mats, int nmats, void* stream) {
  if (nmats <= 0) return;
  hipLaunchKernelGGL(svd_init_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, mats);
  check(hipGetLastError(), "svd init launch");
}

void launch_svd_round(const SvdMat* mats, int nmats, int64_t total_pairs, int round, double tol, int32_t* counter,
                      const int32_t* prev, int waves, void* stream) {
  if (nmats <= 0 || total_pairs <= 0) return;
  TDMPS_REQUIRE(waves == 4 || waves == 8, TDMPS_ERR_ARG, "svd round: waves must be 4 or 8");
  if (waves == 4)
    hipLaunchKernelGGL(svd_block_round_kernel<4>, dim3((unsigned)total_pairs), dim3(64 * 4), 0, (hipStream_t)stream,
                       mats, nmats, round, tol, counter, prev);
  else
    hipLaunchKernelGGL(svd_block_round_kernel<8>, dim3((unsigned)total_pairs), dim3(64 * 8), 0, (hipStream_t)stream,
                       mats, nmats, round, tol, counter, prev);
  check(hipGetLastError(), "svd round launch");
}

void launch_svd_norms(const SvdMat* mats, int nmats, int maxk, double* out, void* stream) {
  if (nmats <= 0 || maxk <= 0) return;
  int64_t waves = (int64_t)nmats * maxk;
  hipLaunchKernelGGL(svd_norms_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, (hipStream_t)stream, mats,
                     nmats, maxk, out);
  check(hipGetLastError(), "svd norms launch");
}

}  // namespace tdmps
