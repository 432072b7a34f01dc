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

// Iteration over the flattened (segment, channel, k-chunk) steps of one task.
struct StepIt {
  int s, r, k0;
};

template <int BM, int BN, int BK>
struct Stage {
  // per-thread prefetch registers: BM*BK/256 A elements and BK*BN/256 B elements
  static constexpr int NA = BM * BK / 256;
  static constexpr int NB = BK * BN / 256;
  double2 ra[NA], rb[NB];

  __device__ __forceinline__ void load(const GemmSeg& S, const GemmTask& T, int bidx, int r, int k0, int m0, int n0,
                                       int tid) {
    const bool conjA = S.opA == OP_C || S.opA == OP_J;
    const bool transA = S.opA == OP_T || S.opA == OP_C;
    const bool conjB = S.opB == OP_C || S.opB == OP_J;
    const bool transB = S.opB == OP_T || S.opB == OP_C;
    const double2* A = (const double2*)S.A + bidx * S.bsA + r * S.rsA;
    const double2* B = (const double2*)S.B + bidx * S.bsB + r * S.rsB;
    const double2 alpha = make_double2(S.alpha.x, S.alpha.y);
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      int rr, kk;
      if (!transA) {
        rr = e / BK;
        kk = e - rr * BK;
      } else {
        kk = e / BM;
        rr = e - kk * BM;
      }
      const int gr = m0 + rr, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gr < T.m && gk < S.k) {
        v = transA ? A[(int64_t)gk * S.lda + gr] : A[(int64_t)gr * S.lda + gk];
        if (conjA) v.y = -v.y;
        v = cmul(v, alpha);
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      int kk, cc;
      if (!transB) {
        kk = e / BN;
        cc = e - kk * BN;
      } else {
        cc = e / BK;
        kk = e - cc * BK;
      }
      const int gk = k0 + kk, gc = n0 + cc;
      double2 v = make_double2(0.0, 0.0);
      if (gk < S.k && gc < T.n) {
        v = transB ? B[(int64_t)gc * S.ldb + gk] : B[(int64_t)gk * S.ldb + gc];
        if (conjB) v.y = -v.y;
      }
      rb[q] = v;
    }
  }

  __device__ __forceinline__ void store(double2 (*As)[BK + 1], double2 (*Bs)[BN + 1], const GemmSeg& S, int tid) {
    const bool transA = S.opA == OP_T || S.opA == OP_C;
    const bool transB = S.opB == OP_T || S.opB == OP_C;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      int rr, kk;
      if (!transA) {
        rr = e / BK;
        kk = e - rr * BK;
      } else {
        kk = e / BM;
        rr = e - kk * BM;
      }
      As[rr][kk] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      int kk, cc;
      if (!transB) {
        kk = e / BN;
        cc = e - kk * BN;
      } else {
        cc = e / BK;
        kk = e - cc * BK;
      }
      Bs[kk][cc] = rb[q];
    }
  }
};

__device__ __forceinline__ bool next_step(const GemmSeg* __restrict__ segs, const GemmTask& T, StepIt& it, int BK) {
  it.k0 += BK;
  const GemmSeg& S = segs[it.s];
  if (it.k0 < S.k) return true;
  it.k0 = 0;
  if (++it.r < S.nred) return true;
  it.r = 0;
  return ++it.s < T.seg0 + T.nseg;
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmTask* __restrict__ tasks,
                                                       const GemmSeg* __restrict__ segs,
                                                       const int32_t* __restrict__ tile_task, int64_t total_tiles) {
  constexpr int BK = 16;             // complex k per LDS stage
  constexpr int WM = BM / 2;         // complex rows per wave
  constexpr int WN = BN / 2;         // complex columns per wave
  constexpr int TM = WM / 16;        // 16x16 MFMA tiles along m
  constexpr int TN = (2 * WN) / 16;  // along real n
  __shared__ double2 As[BM][BK + 1];
  __shared__ double2 Bs[BK][BN + 1];

  // One tile per workgroup.  Workgroup w runs on XCD w % 8; tiles are numbered so that
  // each XCD takes a contiguous range, keeping neighbouring tiles of a task in one L2.
  const int64_t per_xcd = (total_tiles + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= total_tiles) return;
  {
  const int ti = tile_task[tile];
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

  Stage<BM, BN, BK> st;
  StepIt it{T.seg0, 0, 0};
  bool have = T.nseg > 0;
  // skip empty segments
  while (have && (segs[it.s].k <= 0 || segs[it.s].nred <= 0)) {
    if (++it.s >= T.seg0 + T.nseg) have = false;
  }
  if (have) st.load(segs[it.s], T, bidx, it.r, it.k0, m0, n0, tid);
  while (have) {
    st.store(As, Bs, segs[it.s], tid);
    __syncthreads();
    StepIt nx = it;
    bool more = next_step(segs, T, nx, BK);
    while (more && (segs[nx.s].k <= 0 || segs[nx.s].nred <= 0)) {
      nx.k0 = 0;
      nx.r = 0;
      more = ++nx.s < T.seg0 + T.nseg;
    }
    if (more) st.load(segs[nx.s], T, bidx, nx.r, nx.k0, m0, n0, tid);
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
    it = nx;
    have = more;
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
  __syncthreads();
  }
}

// Deterministic split-K reduction: C (+)= sum_s parts[s] in fixed order.
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceTask* __restrict__ tasks) {
  const ReduceTask t = tasks[blockIdx.x];
  const int64_t n = (int64_t)t.m * t.n;
  const int64_t stride = (int64_t)t.m * t.n;
  const double2* P = (const double2*)t.parts;
  double2* C = (double2*)t.C;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.y * blockDim.x) {
    double2 s = P[e];
    for (int q = 1; q < t.nparts; ++q) {
      double2 v = P[q * stride + e];
      s.x += v.x;
      s.y += v.y;
    }
    const int r = (int)(e / t.n), c = (int)(e - (int64_t)r * t.n);
    double2* d = C + (int64_t)r * t.ldc + c;
    if (t.accum) {
      double2 o = *d;
      s.x += o.x;
      s.y += o.y;
    }
    *d = s;
  }
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(TDMPS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace


void launch_reduce(const ReduceTask* tasks, int ntasks, void* stream) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3(ntasks, 8), dim3(256), 0, (hipStream_t)stream, tasks);
  check(hipGetLastError(), "reduce launch");
}

int gemm_tile_m(int cfg) { return cfg == 0 ? 64 : (cfg == 1 ? 32 : 128); }
int gemm_tile_n(int cfg) { return cfg == 0 ? 64 : 32; }

void launch_gemm(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int cfg,
                 int precision, void* stream) {
  if (total_tiles <= 0) return;
  (void)precision;
  const int64_t grid = 8 * ((total_tiles + 7) / 8);
  TDMPS_REQUIRE(grid < ((int64_t)1 << 31), TDMPS_ERR_ARG, "too many GEMM tiles in one launch");
  dim3 g((unsigned)grid), block(256);
  if (cfg == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<64, 64>), g, block, 0, (hipStream_t)stream, tasks, segs, tile_task, total_tiles);
  else if (cfg == 1)
    hipLaunchKernelGGL((gemm_f64_kernel<32, 32>), g, block, 0, (hipStream_t)stream, tasks, segs, tile_task, total_tiles);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<128, 32>), g, block, 0, (hipStream_t)stream, tasks, segs, tile_task, total_tiles);
  check(hipGetLastError(), "gemm launch");
}

}  // namespace tdmps
