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
#include <type_traits>

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

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Precision of the products (operands are FP64 complex in HBM in every mode):
//   P64  : FP64 MFMA 16x16x4               (LDS: double2)
//   P32  : FP32 MFMA 16x16x4, FP32 accumulate (LDS: float2)
//   PBF3 : bf16 split x = hi + lo of the FP32-rounded operand, products hi*hi + hi*lo + lo*hi
//          on the 16x16x32 bf16 MFMA with FP32 accumulate (LDS: realified hi / lo planes)
enum { P64 = 0, P32 = 1, PBF3 = 2 };

template <int BM, int BN, int PREC>
struct Smem;
template <int BM, int BN>
struct Smem<BM, BN, P64> {
  double2 A[BM][9];
  double2 B[8][BN + 1];
};
template <int BM, int BN>
struct Smem<BM, BN, P32> {
  float2 A[BM][17];
  float2 B[16][BN + 1];
};
template <int BM, int BN>
struct Smem<BM, BN, PBF3> {
  // A' rows (realified k, 32 per stage) and B'^T rows (realified column, 32 k), hi and lo
  __bf16 Ah[BM][40], Al[BM][40];
  __bf16 Bh[2 * BN][40], Bl[2 * BN][40];
};

__device__ __forceinline__ void split_bf16(double x, __bf16& h, __bf16& l) {
  const float f = (float)x;
  h = (__bf16)f;
  l = (__bf16)(f - (float)h);
}

template <int BM, int BN, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void gemm_kernel(const GemmTask* __restrict__ tasks,
                                                   const GemmSeg* __restrict__ segs,
                                                   const int32_t* __restrict__ tile_task, int64_t total_tiles) {
  constexpr int BK = PREC == P64 ? 8 : 16;  // complex k per LDS stage (FP64: fewer live registers)
  constexpr int WM = BM / 2;                 // complex rows per wave
  constexpr int WN = BN / 2;                 // complex columns per wave
  constexpr int TM = WM / 16;                // 16x16 MFMA tiles along m
  constexpr int TN = (2 * WN) / 16;          // along real n
  typedef typename std::conditional<PREC == P64, d4, f4>::type acc_t;
  __shared__ Smem<BM, BN, PREC> sm;

  // One tile per workgroup.  Workgroup w runs on XCD w % 8; tiles are numbered so that
  // each XCD takes a contiguous range, keeping neighbouring tiles of a task in one L2.
  const int64_t per_xcd = (total_tiles + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= total_tiles) return;
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

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  Stage<BM, BN, BK> st;
  StepIt it{T.seg0, 0, 0};
  bool have = T.nseg > 0;
  while (have && (segs[it.s].k <= 0 || segs[it.s].nred <= 0)) {
    if (++it.s >= T.seg0 + T.nseg) have = false;
  }
  if (have) st.load(segs[it.s], T, bidx, it.r, it.k0, m0, n0, tid);
  while (have) {
    // registers -> LDS in the precision's layout
    {
      const GemmSeg& S = segs[it.s];
      const bool transA = S.opA == OP_T || S.opA == OP_C;
      const bool transB = S.opB == OP_T || S.opB == OP_C;
#pragma unroll
      for (int q = 0; q < Stage<BM, BN, BK>::NA; ++q) {
        const int e = tid + q * 256;
        int rr, kk;
        if (!transA) {
          rr = e / BK;
          kk = e - rr * BK;
        } else {
          kk = e / BM;
          rr = e - kk * BM;
        }
        const double2 v = st.ra[q];
        if constexpr (PREC == P64) {
          sm.A[rr][kk] = v;
        } else if constexpr (PREC == P32) {
          sm.A[rr][kk] = make_float2((float)v.x, (float)v.y);
        } else {
          split_bf16(v.x, sm.Ah[rr][2 * kk], sm.Al[rr][2 * kk]);
          split_bf16(v.y, sm.Ah[rr][2 * kk + 1], sm.Al[rr][2 * kk + 1]);
        }
      }
#pragma unroll
      for (int q = 0; q < Stage<BM, BN, BK>::NB; ++q) {
        const int e = tid + q * 256;
        int kk, cc;
        if (!transB) {
          kk = e / BN;
          cc = e - kk * BN;
        } else {
          cc = e / BK;
          kk = e - cc * BK;
        }
        const double2 v = st.rb[q];
        if constexpr (PREC == P64) {
          sm.B[kk][cc] = v;
        } else if constexpr (PREC == P32) {
          sm.B[kk][cc] = make_float2((float)v.x, (float)v.y);
        } else {
          // B' = [[Re, Im], [-Im, Re]] per complex element, stored transposed (column-major)
          __bf16 rh, rl, ih, il, nh, nl;
          split_bf16(v.x, rh, rl);
          split_bf16(v.y, ih, il);
          split_bf16(-v.y, nh, nl);
          sm.Bh[2 * cc][2 * kk] = rh;
          sm.Bl[2 * cc][2 * kk] = rl;
          sm.Bh[2 * cc + 1][2 * kk] = ih;
          sm.Bl[2 * cc + 1][2 * kk] = il;
          sm.Bh[2 * cc][2 * kk + 1] = nh;
          sm.Bl[2 * cc][2 * kk + 1] = nl;
          sm.Bh[2 * cc + 1][2 * kk + 1] = rh;
          sm.Bl[2 * cc + 1][2 * kk + 1] = rl;
        }
      }
    }
    __syncthreads();
    StepIt nx = it;
    bool more = next_step(segs, T, nx, BK);
    while (more && (segs[nx.s].k <= 0 || segs[nx.s].nred <= 0)) {
      nx.k0 = 0;
      nx.r = 0;
      more = ++nx.s < T.seg0 + T.nseg;
    }
    if (more) st.load(segs[nx.s], T, bidx, nx.r, nx.k0, m0, n0, tid);
    if constexpr (PREC == PBF3) {
      bf8 ah[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = *(const bf8*)&sm.Ah[wm + i * 16 + l16][8 * lq];
        al[i] = *(const bf8*)&sm.Al[wm + i * 16 + l16][8 * lq];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int rc = 2 * wn + j * 16 + l16;
        const bf8 bh = *(const bf8*)&sm.Bh[rc][8 * lq];
        const bf8 bl = *(const bf8*)&sm.Bl[rc][8 * lq];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int kr = 0; kr < 2 * BK; kr += 4) {
        const int kreal = kr + lq;
        const int kc = kreal >> 1, kp = kreal & 1;
        typedef typename std::conditional<PREC == P64, double, float>::type r_t;
        r_t a[TM], bb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const auto av = sm.A[wm + i * 16 + l16][kc];
          a[i] = kp ? av.y : av.x;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int rc = 2 * wn + j * 16 + l16;
          const auto bv = sm.B[kc][rc >> 1];
          const int cp = rc & 1;
          bb[j] = kp == 0 ? (cp == 0 ? bv.x : bv.y) : (cp == 0 ? -bv.y : bv.x);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (PREC == P64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    __syncthreads();
    it = nx;
    have = more;
  }
  // Epilogue.  Output lane layouts on gfx950 (read off the hardware): register e of lane l
  // holds row l/16 + 4e of a 16x16 tile for the f64 MFMA and row 4(l/16) + e for the f32
  // and bf16 MFMAs; column l%16 in all cases.
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
        const int row = PREC == P64 ? lq + 4 * e : 4 * lq + e;
        const int gr = m0 + wm + i * 16 + row;
        if (gr < T.m && gc < T.n) {
          double* p = (double*)(C + (int64_t)gr * T.ldc + gc) + part;
          const double v = (double)acc[i][j][e];
          *p = accum ? *p + v : v;
        }
      }
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

template <int BM, int BN>
void launch_cfg(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int precision,
                hipStream_t stream) {
  const int64_t grid = 8 * ((total_tiles + 7) / 8);
  TDMPS_REQUIRE(grid < ((int64_t)1 << 31), TDMPS_ERR_ARG, "too many GEMM tiles in one launch");
  dim3 g((unsigned)grid), block(256);
  if (precision == TDMPS_FP32)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P32>), g, block, 0, stream, tasks, segs, tile_task, total_tiles);
  else if (precision == TDMPS_BF16X3)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, PBF3>), g, block, 0, stream, tasks, segs, tile_task, total_tiles);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P64>), g, block, 0, stream, tasks, segs, tile_task, total_tiles);
}

void launch_gemm(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int cfg,
                 int precision, void* stream) {
  if (total_tiles <= 0) return;
  if (cfg == 0)
    launch_cfg<64, 64>(tasks, segs, tile_task, total_tiles, precision, (hipStream_t)stream);
  else if (cfg == 1)
    launch_cfg<32, 32>(tasks, segs, tile_task, total_tiles, precision, (hipStream_t)stream);
  else
    launch_cfg<128, 32>(tasks, segs, tile_task, total_tiles, precision, (hipStream_t)stream);
  check(hipGetLastError(), "gemm launch");
}

}  // namespace tdmps
