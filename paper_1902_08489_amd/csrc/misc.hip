// Strided block copies and the batched one-sided Jacobi SVD (FP64).
#include <hip/hip_runtime.h>

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

__device__ __forceinline__ void rotate(double2* x, double2* y, int n, int lane, double c, double s, double emr,
                                       double emi) {
  for (int e = lane; e < n; e += 64) {
    double2 a = x[e], b = y[e];
    // b' = e^{-i phi} b
    double br = emr * b.x - emi * b.y, bi = emr * b.y + emi * b.x;
    x[e] = make_double2(c * a.x - s * br, c * a.y - s * bi);
    y[e] = make_double2(s * a.x + c * br, s * a.y + c * bi);
  }
}

// One round of the circle schedule: pair i of round r is (np-1, r) for i = 0 and
// ((r+i) mod (np-1), (r-i) mod (np-1)) otherwise; every pair meets once per sweep.
__global__ __launch_bounds__(256) void svd_round_kernel(const SvdMat* __restrict__ mats, int nmats,
                                                        int64_t total_pairs, int round, double tol,
                                                        int32_t* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (gw >= total_pairs) return;
  const int j = find_mat(mats, nmats, gw);
  const SvdMat m = mats[j];
  const int i = (int)(gw - m.pair_base);
  const int np = m.kpad;
  if (round >= np - 1 || i >= np / 2) return;
  int p, q;
  if (i == 0) {
    p = np - 1;
    q = round;
  } else {
    p = (round + i) % (np - 1);
    q = (round - i + (np - 1)) % (np - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
  if (q >= m.k) return;
  double2* gp = (double2*)m.G + (int64_t)p * m.ell;
  double2* gq = (double2*)m.G + (int64_t)q * m.ell;
  double a = 0, b = 0, gr = 0, gi = 0;
  for (int e = lane; e < m.ell; e += 64) {
    double2 x = gp[e], y = gq[e];
    a += x.x * x.x + x.y * x.y;
    b += y.x * y.x + y.y * y.y;
    gr += x.x * y.x + x.y * y.y;  // conj(x) y
    gi += x.x * y.y - x.y * y.x;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  gr = wave_sum(gr);
  gi = wave_sum(gi);
  const double ag = sqrt(gr * gr + gi * gi);
  if (!(ag > tol * sqrt(a * b)) || !(ag > m.thr * sqrt(fmax(a, b))) || ag == 0.0) return;
  if (lane == 0) atomicAdd(counter, 1);
  const double zeta = (b - a) / (2.0 * ag);
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  const double emr = gr / ag, emi = -gi / ag;  // e^{-i phi}
  rotate(gp, gq, m.ell, lane, c, s, emr, emi);
  rotate((double2*)m.V + (int64_t)p * m.k, (double2*)m.V + (int64_t)q * m.k, m.k, lane, c, s, emr, emi);
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

void launch_svd_init(const SvdMat* mats, int nmats, void* stream) {
  if (nmats <= 0) return;
  hipLaunchKernelGGL(svd_init_kernel, dim3(nmats), dim3(256), 0, (hipStream_t)stream, mats);
  check(hipGetLastError(), "svd init launch");
}

void launch_svd_round(const SvdMat* mats, int nmats, int64_t total_pairs, int round, double tol, int32_t* counter,
                      void* stream) {
  if (nmats <= 0 || total_pairs <= 0) return;
  int64_t blocks = (total_pairs + 3) / 4;
  hipLaunchKernelGGL(svd_round_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, mats, nmats,
                     total_pairs, round, tol, counter);
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
