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

// Position in the flattened (segment, channel, k-chunk) steps of one task.  The segment
// descriptor is read only when the cursor enters a new segment; a k step only moves k0.
// E: operand element type (double2 = FP64 complex storage, float2 = FP32 complex storage).
template <typename E>
struct Cursor {
  const GemmSeg* segs;
  int s, se, r, k0, K, nred;
  int64_t lda, ldb, rsA, rsB;
  const E* A;  // operands of channel r of the current segment
  const E* B;
  double2 alpha;
  bool tA, cA, tB, cB;

  __device__ __forceinline__ bool open(int64_t bidx) {
    for (; s < se; ++s) {
      const GemmSeg& S = segs[s];
      if (S.k <= 0 || S.nred <= 0) continue;
      K = S.k;
      nred = S.nred;
      lda = S.lda;
      ldb = S.ldb;
      rsA = S.rsA;
      rsB = S.rsB;
      A = (const E*)S.A + bidx * S.bsA;
      B = (const E*)S.B + bidx * S.bsB;
      alpha = make_double2(S.alpha.x, S.alpha.y);
      tA = S.opA == OP_T || S.opA == OP_C;
      cA = S.opA == OP_C || S.opA == OP_J;
      tB = S.opB == OP_T || S.opB == OP_C;
      cB = S.opB == OP_C || S.opB == OP_J;
      r = 0;
      k0 = 0;
      return true;
    }
    return false;
  }
  __device__ __forceinline__ bool advance(int64_t bidx, int bk) {
    k0 += bk;
    if (k0 < K) return true;
    k0 = 0;
    if (++r < nred) {
      A += rsA;
      B += rsB;
      return true;
    }
    ++s;
    return open(bidx);
  }
};

// Operands are read through global-address-space pointers: generic (flat) loads would also
// count against the LDS wait counter, so every LDS read of the MFMA loop would wait for the
// prefetch of the next stage.
template <typename E>
struct GPtr;
template <>
struct GPtr<double2> {
  typedef const __attribute__((address_space(1))) double* type;
};
template <>
struct GPtr<float2> {
  typedef const __attribute__((address_space(1))) float* type;
};

// Element -> thread mapping of the B stage, whatever the operand's storage: BMAP_N puts
// adjacent threads on adjacent columns, BMAP_K on adjacent k.  The LDS layout decides, not
// the global one: FP64 / FP32 store B' row-major, where threads adjacent along k would
// write rows 2 apart on the same banks (BMAP_N: the final H_eff stage, whose B is
// transposed, 16.8 -> 12.8 ms at L = 24, D = 1024); the bf16 planes store B'^T, where
// adjacent k are adjacent words (BMAP_K: 39.9 -> 36.8 ms for the whole H_eff).
enum { BMAP_N = 1, BMAP_K = 2 };

template <int BM, int BN, int BK, int BMAP, typename E>
struct Stage {
  // per-thread prefetch registers: ceil(BM*BK/256) A elements and ceil(BK*BN/256) B elements,
  // raw as loaded (conjugation and the segment scale are applied when they are written to LDS,
  // so that nothing waits for the loads before the MFMAs of the current stage are issued)
  static constexpr int NA = (BM * BK + 255) / 256;
  static constexpr int NB = (BK * BN + 255) / 256;
  static constexpr bool FULLA = BM * BK % 256 == 0;
  static constexpr bool FULLB = BK * BN % 256 == 0;
  typedef typename GPtr<E>::type gptr;
  E ra[NA], rb[NB];

  __device__ __forceinline__ void load(const Cursor<E>& c, const GemmTask& T, int m0, int n0, int tid) {
    const gptr A = (gptr)c.A;
    const gptr B = (gptr)c.B;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      int rr, kk;
      if (!c.tA) {
        rr = e / BK;
        kk = e - rr * BK;
      } else {
        kk = e / BM;
        rr = e - kk * BM;
      }
      const int gr = m0 + rr, gk = c.k0 + kk;
      E v = {0, 0};
      if ((FULLA || e < BM * BK) && gr < T.m && gk < c.K) {
        const gptr p = A + 2 * (c.tA ? (int64_t)gk * c.lda + gr : (int64_t)gr * c.lda + gk);
        v.x = p[0];
        v.y = p[1];
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      int kk, cc;
      if (BMAP == BMAP_N) {
        kk = e / BN;
        cc = e - kk * BN;
      } else {
        cc = e / BK;
        kk = e - cc * BK;
      }
      const int gk = c.k0 + kk, gc = n0 + cc;
      E v = {0, 0};
      if ((FULLB || e < BK * BN) && gk < c.K && gc < T.n) {
        const gptr p = B + 2 * (c.tB ? (int64_t)gc * c.ldb + gk : (int64_t)gk * c.ldb + gc);
        v.x = p[0];
        v.y = p[1];
      }
      rb[q] = v;
    }
  }
};

// Staging of a real-A product (FP64 only): C = A B with A real (the real parts of the stored
// complex A, non-transposed) and B complex, non-transposed.  One LDS stage then covers 2 * BK
// values of k: the A' rows hold A's real values at the realified-k positions and B' row k holds
// (Re, Im) of B's complex row k, so the same MFMA loop forms C' = A' B' = the interleaved
// complex result with half the products of the complex form.
template <int BM, int BN, int BK>
struct StageRA {
  static constexpr int KR = 2 * BK;  // k values per stage
  static constexpr int NA = (BM * KR + 255) / 256;
  static constexpr int NB = (KR * BN + 255) / 256;
  static constexpr bool FULLA = BM * KR % 256 == 0;
  static constexpr bool FULLB = KR * BN % 256 == 0;
  typedef const __attribute__((address_space(1))) double* gptr;
  double ra[NA];
  double2 rb[NB];

  __device__ __forceinline__ void load(const Cursor<double2>& c, const GemmTask& T, int m0, int n0, int tid) {
    const gptr A = (gptr)c.A;
    const gptr B = (gptr)c.B;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      const int rr = e / KR, kk = e - rr * KR;
      const int gr = m0 + rr, gk = c.k0 + kk;
      double v = 0.0;
      if ((FULLA || e < BM * KR) && gr < T.m && gk < c.K) v = A[2 * ((int64_t)gr * c.lda + gk)];
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      const int kk = e / BN, cc = e - kk * BN;
      const int gk = c.k0 + kk, gc = n0 + cc;
      double2 v = make_double2(0.0, 0.0);
      if ((FULLB || e < KR * BN) && gk < c.K && gc < T.n) {
        const gptr p = B + 2 * ((int64_t)gk * c.ldb + gc);
        v.x = p[0];
        v.y = p[1];
      }
      rb[q] = v;
    }
  }
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Precision of the products (operands are FP64 complex in HBM in every mode):
//   P64  : FP64 MFMA 16x16x4               (LDS: double2)
//   P32  : FP32 MFMA 16x16x4, FP32 accumulate (LDS: float2)
//   PBF3 : bf16 split x = hi + lo of the FP32-rounded operand, products hi*hi + hi*lo + lo*hi
//          on the 16x16x32 bf16 MFMA with FP32 accumulate (LDS: realified hi / lo planes)
//   PBF6 : three-term split x = hi + mid + lo (all 24 bits of the FP32 value), products
//          hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid (every term down to 2^-16 of the
//          leading one; the dropped ones are 2^-24 and below), FP32 accumulate
enum { P64 = 0, P32 = 1, PBF3 = 2, PBF6 = 3 };


template <int BM, int BN, int PREC>
struct Smem;
// FP64 / FP32: operands are kept realified in LDS so that every MFMA operand is one plain
// LDS read: A' rows hold (Re, Im) interleaved along k (the complex row itself), B' holds the
// 2 x 2 real block [[Re, Im], [-Im, Re]] of every complex element (row = realified k,
// column = realified n).  Row paddings put the B' rows read by one instruction (realified k
// = lane / 16) on distinct LDS banks: row strides of 16 (mod 32) doubles, 16 (mod 64) floats.
constexpr int bpad64(int bn) { return ((16 - 2 * bn) % 32 + 32) % 32; }
constexpr int bpad32(int bn) { return ((16 - 2 * bn) % 64 + 64) % 64; }
template <int BM, int BN>
struct Smem<BM, BN, P64> {
  double A[BM][2 * 8 + 2];
  double B[2 * 8][2 * BN + bpad64(BN)];
};
template <int BM, int BN>
struct Smem<BM, BN, P32> {
  float A[BM][2 * 16 + 4];
  float B[2 * 16][2 * BN + bpad32(BN)];
};
template <int BM, int BN>
struct Smem<BM, BN, PBF3> {
  // A' rows (realified k, 32 per stage) and B'^T rows (realified column, 32 k), hi and lo
  __bf16 Ah[BM][40], Al[BM][40];
  __bf16 Bh[2 * BN][40], Bl[2 * BN][40];
};
template <int BM, int BN>
struct Smem<BM, BN, PBF6> {
  // as PBF3 with a third (mid) plane
  __bf16 Ah[BM][40], Am[BM][40], Al[BM][40];
  __bf16 Bh[2 * BN][40], Bm[2 * BN][40], Bl[2 * BN][40];
};

__device__ __forceinline__ void split_bf16(float f, __bf16& h, __bf16& l) {
  h = (__bf16)f;
  l = (__bf16)(f - (float)h);
}

// f = h + m + l: each difference is exact in FP32 (it keeps at most 16, then 8, significant bits)
__device__ __forceinline__ void split3_bf16(float f, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)f;
  const float r = f - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

__device__ __forceinline__ double2 scale(double2 v, bool conj, double2 alpha) {
  if (conj) v.y = -v.y;
  return cmul(v, alpha);
}
__device__ __forceinline__ float2 scale(float2 v, bool conj, double2 alpha) {
  if (conj) v.y = -v.y;
  const float ar = (float)alpha.x, ai = (float)alpha.y;
  return make_float2(v.x * ar - v.y * ai, v.x * ai + v.y * ar);
}

// two bf16 as one 32-bit LDS word (the first at the lower address)
__device__ __forceinline__ uint32_t pack_bf16(__bf16 lo, __bf16 hi) {
  return (uint32_t)__builtin_bit_cast(unsigned short, lo) | ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
}

// S32: operands stored as FP32 complex (FP32 and BF16-split precisions); RA: real A (FP64)
template <int BM, int BN, int PREC, bool S32, bool RA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void gemm_kernel(const GemmTask* __restrict__ tasks,
                                                   const GemmSeg* __restrict__ segs,
                                                   const int32_t* __restrict__ tile_task, int64_t total_tiles,
                                                   int64_t tile_offset) {
  constexpr int BK = PREC == P64 ? 8 : 16;  // complex k per LDS stage (FP64: fewer live registers)
  constexpr bool BF = PREC == PBF3 || PREC == PBF6;
  constexpr int BMAP = BF ? BMAP_K : BMAP_N;
  static_assert(!(S32 && PREC == P64), "FP64 products read FP64 operands");
  static_assert(!RA || (PREC == P64 && !S32), "real-A products are FP64");
  typedef typename std::conditional<S32, float2, double2>::type E;
  typedef typename std::conditional<RA, StageRA<BM, BN, BK>, Stage<BM, BN, BK, BMAP, E>>::type St;
  constexpr int KSTEP = RA ? 2 * BK : BK;  // k values per LDS stage
  constexpr int WM = BM / 2;                 // complex rows per wave
  constexpr int WN = BN / 2;                 // complex columns per wave
  constexpr int TM = WM / 16;                // 16x16 MFMA tiles along m
  constexpr int TN = (2 * WN) / 16;          // along real n
  typedef typename std::conditional<PREC == P64, d4, f4>::type acc_t;
  __shared__ Smem<BM, BN, PREC> sm;

  // One tile per workgroup.  Workgroup w runs on XCD w % 8; tiles are numbered so that
  // each XCD takes a contiguous range, keeping neighbouring tiles of a task in one L2.
  const int64_t per_xcd = (total_tiles + 7) / 8;
  const int64_t tile0 = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile0 >= total_tiles) return;
  const int64_t tile = tile0 + tile_offset;
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
  // A wave whose quadrant of the tile lies outside the block (ragged tiles) would only
  // multiply zero padding: it stages operands and takes the barriers but issues no MFMA.  The
  // FP64 32x48 shape (long final-stage reductions) keeps every wave's MFMAs and every k step
  // (below): the H_eff apply at L = 24, D = 1024 measured faster that way.
  constexpr bool FULL = PREC == P64 && BM == 32 && BN == 48;
  const bool wlive = FULL || (__builtin_amdgcn_readfirstlane(wm) < T.m - m0 &&
                              __builtin_amdgcn_readfirstlane(wn) < T.n - n0);

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  St st;
  Cursor<E> cur;
  cur.segs = segs;
  cur.s = T.seg0;
  cur.se = T.seg0 + T.nseg;
  bool have = cur.open(bidx);
  if (have) st.load(cur, T, m0, n0, tid);
  while (have) {
    // registers -> LDS in the precision's layout
    if constexpr (RA) {
#pragma unroll
      for (int q = 0; q < St::NA; ++q) {
        const int e = tid + q * 256;
        if (!St::FULLA && e >= BM * St::KR) continue;
        const int rr = e / St::KR, kk = e - rr * St::KR;
        sm.A[rr][kk] = st.ra[q] * cur.alpha.x;
      }
#pragma unroll
      for (int q = 0; q < St::NB; ++q) {
        const int e = tid + q * 256;
        if (!St::FULLB && e >= St::KR * BN) continue;
        const int kk = e / BN, cc = e - kk * BN;
        *(double2*)&sm.B[kk][2 * cc] = st.rb[q];
      }
    } else {
      const bool transA = cur.tA;
#pragma unroll
      for (int q = 0; q < St::NA; ++q) {
        const int e = tid + q * 256;
        if (!St::FULLA && e >= BM * BK) continue;
        int rr, kk;
        if (!transA) {
          rr = e / BK;
          kk = e - rr * BK;
        } else {
          kk = e / BM;
          rr = e - kk * BM;
        }
        const E v = scale(st.ra[q], cur.cA, cur.alpha);
        if constexpr (PREC == P64) {
          *(double2*)&sm.A[rr][2 * kk] = v;
        } else if constexpr (PREC == P32) {
          *(float2*)&sm.A[rr][2 * kk] = make_float2((float)v.x, (float)v.y);
        } else if constexpr (PREC == PBF6) {
          __bf16 xh, xm, xl, yh, ym, yl;
          split3_bf16(v.x, xh, xm, xl);
          split3_bf16(v.y, yh, ym, yl);
          *(uint32_t*)&sm.Ah[rr][2 * kk] = pack_bf16(xh, yh);
          *(uint32_t*)&sm.Am[rr][2 * kk] = pack_bf16(xm, ym);
          *(uint32_t*)&sm.Al[rr][2 * kk] = pack_bf16(xl, yl);
        } else {
          __bf16 xh, xl, yh, yl;
          split_bf16(v.x, xh, xl);
          split_bf16(v.y, yh, yl);
          *(uint32_t*)&sm.Ah[rr][2 * kk] = pack_bf16(xh, yh);
          *(uint32_t*)&sm.Al[rr][2 * kk] = pack_bf16(xl, yl);
        }
      }
#pragma unroll
      for (int q = 0; q < St::NB; ++q) {
        const int e = tid + q * 256;
        if (!St::FULLB && e >= BK * BN) continue;
        int kk, cc;
        if (BMAP == BMAP_N) {
          kk = e / BN;
          cc = e - kk * BN;
        } else {
          cc = e / BK;
          kk = e - cc * BK;
        }
        E v = st.rb[q];
        if (cur.cB) v.y = -v.y;
        if constexpr (PREC == P64) {
          *(double2*)&sm.B[2 * kk][2 * cc] = v;
          *(double2*)&sm.B[2 * kk + 1][2 * cc] = make_double2(-v.y, v.x);
        } else if constexpr (PREC == P32) {
          const float re = (float)v.x, im = (float)v.y;
          *(float2*)&sm.B[2 * kk][2 * cc] = make_float2(re, im);
          *(float2*)&sm.B[2 * kk + 1][2 * cc] = make_float2(-im, re);
        } else if constexpr (PREC == PBF6) {
          // the split of -Im is the negated split of Im (bf16 negation is exact)
          __bf16 rh, rm, rl, ih, im, il;
          split3_bf16(v.x, rh, rm, rl);
          split3_bf16(v.y, ih, im, il);
          *(uint32_t*)&sm.Bh[2 * cc][2 * kk] = pack_bf16(rh, -ih);
          *(uint32_t*)&sm.Bm[2 * cc][2 * kk] = pack_bf16(rm, -im);
          *(uint32_t*)&sm.Bl[2 * cc][2 * kk] = pack_bf16(rl, -il);
          *(uint32_t*)&sm.Bh[2 * cc + 1][2 * kk] = pack_bf16(ih, rh);
          *(uint32_t*)&sm.Bm[2 * cc + 1][2 * kk] = pack_bf16(im, rm);
          *(uint32_t*)&sm.Bl[2 * cc + 1][2 * kk] = pack_bf16(il, rl);
        } else {
          // B' = [[Re, Im], [-Im, Re]] per complex element, stored transposed (column-major)
          __bf16 rh, rl, ih, il, nh, nl;
          split_bf16(v.x, rh, rl);
          split_bf16(v.y, ih, il);
          split_bf16(-v.y, nh, nl);
          *(uint32_t*)&sm.Bh[2 * cc][2 * kk] = pack_bf16(rh, nh);
          *(uint32_t*)&sm.Bl[2 * cc][2 * kk] = pack_bf16(rl, nl);
          *(uint32_t*)&sm.Bh[2 * cc + 1][2 * kk] = pack_bf16(ih, rh);
          *(uint32_t*)&sm.Bl[2 * cc + 1][2 * kk] = pack_bf16(il, rl);
        }
      }
    }
    __syncthreads();
    Cursor<E> nx = cur;
    const bool more = nx.advance(bidx, KSTEP);
    if (more) st.load(nx, T, m0, n0, tid);
    if (!wlive) {
      // the wave's quadrant holds only padding: no MFMA
    } else if constexpr (PREC == PBF6) {
      bf8 ah[TM], am[TM], al[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ah[i] = *(const bf8*)&sm.Ah[wm + i * 16 + l16][8 * lq];
        am[i] = *(const bf8*)&sm.Am[wm + i * 16 + l16][8 * lq];
        al[i] = *(const bf8*)&sm.Al[wm + i * 16 + l16][8 * lq];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int rc = 2 * wn + j * 16 + l16;
        const bf8 bh = *(const bf8*)&sm.Bh[rc][8 * lq];
        const bf8 bm = *(const bf8*)&sm.Bm[rc][8 * lq];
        const bf8 bl = *(const bf8*)&sm.Bl[rc][8 * lq];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          // smallest terms first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bm, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bm, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bh, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    } else if constexpr (PREC == PBF3) {
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
      // realified k of the stage that hold data: the steps past the end of a segment's
      // reduction would only add the zero padding.  The test serialises each step's LDS reads
      // with its MFMAs; for the FP64 32x48 shape (three MFMAs a step) that cost more than the
      // padding saved, and it issues every step.
      const int kval = RA || FULL ? 2 * BK : 2 * min(BK, cur.K - cur.k0);
#pragma unroll
      for (int kr = 0; kr < 2 * BK; kr += 4) {
        if (!FULL && kr >= kval) break;
        const int kreal = kr + lq;
        typedef typename std::conditional<PREC == P64, double, float>::type r_t;
        r_t a[TM], bb[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = sm.A[wm + i * 16 + l16][kreal];
#pragma unroll
        for (int j = 0; j < TN; ++j) bb[j] = sm.B[kreal][2 * wn + j * 16 + l16];
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
    cur = nx;
    have = more;
  }
  // Epilogue.  Output lane layouts on gfx950 (read off the hardware): register e of lane l
  // holds row l/16 + 4e of a 16x16 tile for the f64 MFMA and row 4(l/16) + e for the f32
  // and bf16 MFMAs; column l%16 in all cases.
  typedef __attribute__((address_space(1))) double* gout;
  typedef __attribute__((address_space(1))) float* gout32;
  const bool out32 = T.flags & GEMM_OUT32;  // uniform over the workgroup
  const gout C = (gout)(T.C + bidx * T.bsC);
  const gout32 C32 = (gout32)((float2*)T.C + bidx * T.bsC);
  const bool accum = T.flags & GEMM_ACCUM;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    // one row group at a time: all previous values are loaded before any is needed, so the
    // accumulating epilogue waits once per group instead of once per element
    double old[TN][4];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) old[j][e] = 0.0;
    if (accum) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int rc = 2 * wn + j * 16 + l16;
        const int gc = n0 + (rc >> 1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = PREC == P64 ? lq + 4 * e : 4 * lq + e;
          const int gr = m0 + wm + i * 16 + row;
          if (gr < T.m && gc < T.n) {
            const int64_t at = 2 * ((int64_t)gr * T.ldc + gc) + (rc & 1);
            old[j][e] = out32 ? (double)C32[at] : C[at];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int rc = 2 * wn + j * 16 + l16;
      const int gc = n0 + (rc >> 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = PREC == P64 ? lq + 4 * e : 4 * lq + e;
        const int gr = m0 + wm + i * 16 + row;
        if (gr < T.m && gc < T.n) {
          const int64_t at = 2 * ((int64_t)gr * T.ldc + gc) + (rc & 1);
          if (out32)
            C32[at] = (float)(old[j][e] + (double)acc[i][j][e]);
          else
            C[at] = old[j][e] + (double)acc[i][j][e];
        }
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
    if (t.out32) {
      float2* d = (float2*)t.C + (int64_t)r * t.ldc + c;
      if (t.accum) {
        const float2 o = *d;
        s.x += o.x;
        s.y += o.y;
      }
      *d = make_float2((float)s.x, (float)s.y);
    } else {
      double2* d = C + (int64_t)r * t.ldc + c;
      if (t.accum) {
        double2 o = *d;
        s.x += o.x;
        s.y += o.y;
      }
      *d = s;
    }
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

// Tile shapes (complex rows x complex columns).  With the 2 x 2 wave grid a shape needs rows
// in multiples of 32 and columns in multiples of 16 (one f64 MFMA tile covers 16 rows and 8
// complex columns).  Block dimensions are charge-sector sizes, so the planner picks, per
// task, the shape with the least padded work.
constexpr int CFG_M[GEMM_NCFG] = {64, 32, 128, 64, 96, 128, 32, 96, 96, 64};
constexpr int CFG_N[GEMM_NCFG] = {64, 32, 32, 48, 48, 48, 48, 64, 32, 32};
int gemm_tile_m(int cfg) { return CFG_M[cfg]; }
int gemm_tile_n(int cfg) { return CFG_N[cfg]; }

template <int BM, int BN>
void launch_cfg(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int precision,
                hipStream_t stream, int64_t off, bool ops32, bool real_a) {
  const int64_t grid = 8 * ((total_tiles + 7) / 8);
  TDMPS_REQUIRE(grid < ((int64_t)1 << 31), TDMPS_ERR_ARG, "too many GEMM tiles in one launch");
  TDMPS_REQUIRE(!ops32 || precision == TDMPS_FP32 || precision == TDMPS_BF16X3 || precision == TDMPS_BF16X6,
                TDMPS_ERR_ARG, "FP32 operand storage needs the FP32 or a BF16-split precision");
  TDMPS_REQUIRE(!real_a || (precision == TDMPS_FP64 && !ops32), TDMPS_ERR_ARG, "real-A products are FP64");
  dim3 g((unsigned)grid), block(256);
  if (real_a)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P64, false, true>), g, block, 0, stream, tasks, segs, tile_task, total_tiles,
                       off);
  else if (precision == TDMPS_FP32 && ops32)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P32, true, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else if (precision == TDMPS_FP32)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P32, false, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else if (precision == TDMPS_BF16X3 && ops32)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, PBF3, true, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else if (precision == TDMPS_BF16X3)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, PBF3, false, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else if (precision == TDMPS_BF16X6 && ops32)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, PBF6, true, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else if (precision == TDMPS_BF16X6)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, PBF6, false, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, P64, false, false>), g, block, 0, stream, tasks, segs, tile_task, total_tiles, off);
}

void launch_gemm(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int cfg,
                 int precision, void* stream, int64_t off, bool ops32, bool real_a) {
  if (total_tiles <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  switch (cfg) {
    case 0: launch_cfg<64, 64>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 1: launch_cfg<32, 32>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 2: launch_cfg<128, 32>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 3: launch_cfg<64, 48>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 4: launch_cfg<96, 48>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 5: launch_cfg<128, 48>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 6: launch_cfg<32, 48>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 7: launch_cfg<96, 64>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 8: launch_cfg<96, 32>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    case 9: launch_cfg<64, 32>(tasks, segs, tile_task, total_tiles, precision, s, off, ops32, real_a); break;
    default: throw Error(TDMPS_ERR_ARG, "bad GEMM tile configuration");
  }
  check(hipGetLastError(), "gemm launch");
}

}  // namespace tdmps
