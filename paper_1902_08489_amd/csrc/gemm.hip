// Grouped complex block GEMM on CDNA4 matrix cores.
//
// One launch executes every block product of a contraction stage: the grid enumerates the
// output tiles of all tasks (task found by binary search over the tile prefix), and each
// tile loops over the task's segments (operand pairs, optionally a reduction batch over
// MPO channels) and k chunks.  Complex products are done as real MFMA products of the
// "realified" operands (4M): A' = [Re A | Im A] interleaved along k (exactly the storage
// of interleaved complex rows) and B' with 2x2 real blocks [[Re B, Im B], [-Im B, Re B]],
// so C' = A' B' is the interleaved complex result.  Tiles are staged through LDS; the
// segment scale alpha and conjugations are applied while staging.
#include <hip/hip_runtime.h>

#include <string>

#include "common.h"
#include "kernels.h"

namespace tdmps {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int find_task(const GemmTask* __restrict__ tasks, int ntasks, int64_t tile) {
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_base <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmTask* __restrict__ tasks,
                                                       const GemmSeg* __restrict__ segs, int ntasks) {
  constexpr int BK = 8;            // complex k per LDS stage
  constexpr int WM = BM / 2;       // complex rows per wave
  constexpr int WN = BN / 2;       // complex columns per wave
  constexpr int TM = WM / 16;      // 16x16 MFMA tiles along m
  constexpr int TN = (2 * WN) / 16;  // along real n
  __shared__ double2 As[BM][BK + 1];
  __shared__ double2 Bs[BK][BN + 1];

  const int64_t tile = blockIdx.x;
  const int ti = find_task(tasks, ntasks, tile);
  const GemmTask T = tasks[ti];
  const int64_t local = tile - T.tile_base;
  const int per = T.tiles_m * T.tiles_n;
  const int bidx = (int)(local / per);
  const int rem = (int)(local - (int64_t)bidx * per);
  const int m0 = (rem / T.tiles_n) * BM;
  const int n0 = (rem % T.tiles_n) * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int l16 = lane & 15, lq = lane >> 4;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int s = T.seg0; s < T.seg0 + T.nseg; ++s) {
    const GemmSeg S = segs[s];
    const double2 alpha = make_double2(S.alpha.x, S.alpha.y);
    const bool conjA = S.opA == OP_C || S.opA == OP_J;
    const bool transA = S.opA == OP_T || S.opA == OP_C;
    const bool conjB = S.opB == OP_C || S.opB == OP_J;
    const bool transB = S.opB == OP_T || S.opB == OP_C;
    for (int r = 0; r < S.nred; ++r) {
      const double2* A = (const double2*)S.A + bidx * S.bsA + r * S.rsA;
      const double2* B = (const double2*)S.B + bidx * S.bsB + r * S.rsB;
      for (int k0 = 0; k0 < S.k; k0 += BK) {
        // stage A (op(A) is m x k)
        for (int e = tid; e < BM * BK; e += 256) {
          int rr, kk;
          if (!transA) {
            rr = e / BK;
            kk = e - rr * BK;
          } else {
            kk = e / BM;
            rr = e - kk * BM;
          }
          int gr = m0 + rr, gk = k0 + kk;
          double2 v = make_double2(0.0, 0.0);
          if (gr < T.m && gk < S.k) {
            v = transA ? A[(int64_t)gk * S.lda + gr] : A[(int64_t)gr * S.lda + gk];
            if (conjA) v.y = -v.y;
            v = cmul(v, alpha);
          }
          As[rr][kk] = v;
        }
        // stage B (op(B) is k x n)
        for (int e = tid; e < BK * BN; e += 256) {
          int kk, cc;
          if (!transB) {
            kk = e / BN;
            cc = e - kk * BN;
          } else {
            cc = e / BK;
            kk = e - cc * BK;
          }
          int gk = k0 + kk, gc = n0 + cc;
          double2 v = make_double2(0.0, 0.0);
          if (gk < S.k && gc < T.n) {
            v = transB ? B[(int64_t)gc * S.ldb + gk] : B[(int64_t)gk * S.ldb + gc];
            if (conjB) v.y = -v.y;
          }
          Bs[kk][cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kr = 0; kr < 2 * BK; kr += 4) {
          const int kreal = kr + lq;
          const int kc = kreal >> 1, kp = kreal & 1;
          double a[TM], bb[TN];
#pragma unroll
          for (int i = 0; i < TM; ++i) {
            double2 av = As[wm + i * 16 + l16][kc];
            a[i] = kp ? av.y : av.x;
          }
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const int rc = 2 * wn + j * 16 + l16;
            double2 bv = Bs[kc][rc >> 1];
            const int cp = rc & 1;
            bb[j] = kp == 0 ? (cp == 0 ? bv.x : bv.y) : (cp == 0 ? -bv.y : bv.x);
          }
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
      }
    }
  }
  // epilogue: register e of a lane holds row lq + 4 e of each 16x16 tile, real column l16
  // (lane layout of v_mfma_f64_16x16x4f64 on gfx950: A[l%16][l/16], B[l/16][l%16])
  double2* C = (double2*)T.C + bidx * T.bsC;
  const bool accum = T.flags & GEMM_ACCUM;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int rc = 2 * wn + j * 16 + l16;
      const int gc = n0 + (rc >> 1);
      const int part = rc & 1;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gr = m0 + wm + i * 16 + lq + 4 * e;
        if (gr < T.m && gc < T.n) {
          double* p = (double*)(C + (int64_t)gr * T.ldc + gc) + part;
          *p = accum ? *p + acc[i][j][e] : acc[i][j][e];
        }
      }
    }
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(TDMPS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

int gemm_tile_m(int cfg) { return cfg == 0 ? 64 : 32; }
int gemm_tile_n(int cfg) { return cfg == 0 ? 64 : 32; }

void launch_gemm(const GemmTask* tasks, const GemmSeg* segs, int ntasks, int64_t total_tiles, int cfg, int precision,
                 void* stream) {
  if (ntasks <= 0 || total_tiles <= 0) return;
  TDMPS_REQUIRE(total_tiles < (int64_t)1 << 31, TDMPS_ERR_ARG, "too many GEMM tiles in one launch");
  (void)precision;
  dim3 grid((unsigned)total_tiles), block(256);
  if (cfg == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<64, 64>), grid, block, 0, (hipStream_t)stream, tasks, segs, ntasks);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<32, 32>), grid, block, 0, (hipStream_t)stream, tasks, segs, ntasks);
  check(hipGetLastError(), "gemm launch");
}

}  // namespace tdmps
