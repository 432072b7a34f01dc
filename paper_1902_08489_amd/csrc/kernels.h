// Interface between the host planner and the device: runtime calls and kernel launchers.
// Every HIP call of the library sits behind these functions (device.hip, gemm.hip,
// misc.hip); the planner and the drivers only see plain pointers and task lists.
#pragma once

#include <cstddef>
#include <cstdint>

namespace tdmps {

struct cplx {
  double x, y;
};

// ---------------------------------------------------------------- grouped complex GEMM
// One task writes (or accumulates into) nbatch independent m x n outputs
//   C_b = [C_b +] sum_seg alpha_seg * sum_{r < nred} op(A_seg + b*bsA + r*rsA) op(B_seg + b*bsB + r*rsB)
// with op in {N, T, C (conjugate transpose), J (conjugate)}; op(A) is m x k, op(B) k x n,
// all row-major with leading dimensions lda, ldb, ldc (in complex elements).
// Element storage: FP64 complex (16 bytes) by default.  A launch with FP32 operands (the mixed
// precisions' storage) reads A and B as FP32 complex (8 bytes; pointers and strides still count
// complex elements); GEMM_OUT32 makes a task write C as FP32 complex.
enum { OP_N = 0, OP_T = 1, OP_C = 2, OP_J = 3 };
enum { GEMM_ACCUM = 1, GEMM_OUT32 = 2 };

struct GemmTask {
  cplx* C;
  int64_t bsC;
  int32_t ldc, m, n, nbatch;
  int32_t seg0, nseg;
  int32_t tiles_m, tiles_n, flags;
  int64_t tile_base;  // exclusive prefix of nbatch*tiles_m*tiles_n over previous tasks
};

struct GemmSeg {
  const cplx* A;
  const cplx* B;
  int64_t bsA, bsB, rsA, rsB;
  int32_t nred, k, lda, ldb, opA, opB;
  cplx alpha;
};

// Split-K partial sums: C (+)= sum_{q < nparts} parts[q] (each part m x n, contiguous, FP64);
// out32: C is FP32 complex.
struct ReduceTask {
  cplx* C;
  const cplx* parts;
  int32_t m, n, ldc, nparts, accum, out32;
};

// ---------------------------------------------------------------- shared-block combination
// T[j * blk + e] (+)= sum_{q < nq} coef[j * nq + q] * X[q * blk + e] for j < nrun, e < blk: the
// contributions of blocks shared by a run of channels, each channel with its own real
// coefficients (nq <= SHARE_MAXQ).
constexpr int SHARE_MAXQ = 8;
struct ShareTask {
  cplx* T;  // FP32 complex if out32
  const cplx* X;
  int64_t coff;  // first coefficient of the task in the coefficient array of the launch
  int64_t blk;
  int32_t nrun, nq, accum, out32;
};

// ---------------------------------------------------------------- strided block copies
// dst[r*dst_ld + c] (+)= op(src[(ridx?ridx[r]:r)*src_rs + (cidx?cidx[c]:c)*src_cs]) * rs[r] * cs[c]
struct CopyTask {
  const cplx* src;
  cplx* dst;
  int64_t src_rs, src_cs;
  const int32_t* ridx;
  const int32_t* cidx;
  const double* rscale;
  const double* cscale;
  int32_t rows, cols, dst_ld, flags;  // flags: 1 = conjugate source, 2 = accumulate
};

// ---------------------------------------------------------------- one-sided Jacobi SVD
// Matrix j holds k vectors of length ell (column-major G, column stride ell) and the k x k
// accumulated rotation V (column-major, column stride k).
// Columns are grouped in blocks of SVD_BLOCK; nblk = number of blocks rounded up to an even
// count (at least 2), pair_base = exclusive prefix of nblk/2 over the matrices of a batch.
constexpr int SVD_BLOCK = 8;
struct SvdMat {
  cplx* G;
  cplx* V;
  int32_t ell, k, nblk, pair_base;
  double thr;  // pairs with |g_p^H g_q| <= thr max(|g_p|, |g_q|) are orthogonal
};

// Batched Householder QR (panels of QR_PANEL columns) of G (ell x k, column-major), n = nsv =
// min(ell, k).  T: per matrix ceil(n / QR_PANEL) row-major QR_PANEL x QR_PANEL compact-WY
// factors; X: k x n; V: n x n; B: ell x n; cb_base: exclusive prefix of ceil(k / QR_PANEL).
constexpr int QR_PANEL = 16;
struct QrMat {
  cplx* G;
  cplx* T;
  cplx* X;
  cplx* V;
  cplx* B;
  int32_t ell, k, nsv, cb_base;
};

// runtime
void dev_set_device(int device);
// Binds the calling thread to (device, stream): later allocations are served from blocks
// released on that stream (or fresh ones).
void dev_bind(int device, void* stream);
void* dev_alloc(size_t bytes);  // returns nullptr when out of memory
void dev_free(void* p);
void dev_alloc_stats(double* count, double* seconds);  // hipMalloc calls and seconds so far (process)
void dev_h2d(void* dst, const void* src, size_t bytes, void* stream);
// H2D copy on the stream straight from host memory (no staging block), returning after the
// stream has completed it
void dev_h2d_wait(void* dst, const void* src, size_t bytes, void* stream);
void dev_d2h(void* dst, const void* src, size_t bytes, void* stream);  // host data valid on return
void dev_d2d(void* dst, const void* src, size_t bytes, void* stream);
void dev_zero(void* dst, size_t bytes, void* stream);  // fill kernel (no memset nodes)
void dev_sync(void* stream);
void* dev_stream_create();
void dev_stream_destroy(void* s);
void* dev_event_create();
void dev_event_destroy(void* e);
void dev_event_record(void* e, void* stream);
float dev_event_elapsed_ms(void* a, void* b);  // synchronises on b
// Stream capture into a HIP graph (the stream must not be the legacy default stream; the
// captured work must hold no allocations, synchronisations or memset nodes).
void graph_begin(void* stream);
void* graph_end(void* stream);    // instantiated graph
void graph_abort(void* stream);   // ends a failed capture and drops it
void graph_launch(void* exec, void* stream);
void graph_destroy(void* exec);

// Scratch of the no-allocation entry point (noalloc.hip): noalloc_init resolves the address of
// the device's copy (call with that device current); noalloc_scratch returns it (nullptr before
// noalloc_init) and its capacity.
void noalloc_init(int device);
void* noalloc_scratch(int device, size_t* cap);

// launchers (all asynchronous on `stream`)
// Runs tiles tile_offset .. tile_offset + total_tiles - 1 of the tile table.
// ops32: A and B are FP32 complex (FP32 and BF16-split precisions only).  real_a: A is real-valued
// (the real parts of the stored complex A are read, A and B not transposed, alpha real; FP64
// only): half the matrix-unit products of the complex form.
void launch_gemm(const GemmTask* tasks, const GemmSeg* segs, const int32_t* tile_task, int64_t total_tiles, int cfg,
                 int precision, void* stream, int64_t tile_offset = 0, bool ops32 = false, bool real_a = false);
void launch_reduce(const ReduceTask* tasks, int ntasks, void* stream);
constexpr int GEMM_NCFG = 10;  // tile shape configurations of launch_gemm
int gemm_tile_m(int cfg);
int gemm_tile_n(int cfg);
void launch_copy(const CopyTask* tasks, int ntasks, void* stream);
void launch_share(const ShareTask* tasks, const double* coef, int ntasks, int64_t max_blk, void* stream);
void launch_svd_init(const SvdMat* mats, int nmats, void* stream);  // V = identity
// One round (block pairs of the circle schedule, round >= 0; or the diagonal round of a sweep,
// round < 0) for all matrices; total_pairs = sum nblk/2; rot_counter is incremented once per
// workgroup that rotated.  A sweep is the diagonal round followed by rounds 0 .. nblk-2.  If
// prev_counter is given and holds 0 (the previous sweep rotated nothing: converged), the
// round does nothing, so sweeps can be queued ahead of the convergence test.
void launch_svd_round(const SvdMat* mats, int nmats, int64_t total_pairs, int round, double tol, int32_t* rot_counter,
                      const int32_t* prev_counter, int waves, void* stream);
void launch_svd_norms(const SvdMat* mats, int nmats, int max_k, double* sigma_out, void* stream);
void launch_scale(cplx* x, int64_t n, cplx alpha, void* stream);
// dst[e] = (FP32 complex) src[e], e < n (dst: 8 bytes per element)
void launch_to_f32(const cplx* src, void* dst, int64_t n, void* stream);
// QR preconditioning of the Jacobi SVD: factor panel j0 (one workgroup per matrix); apply
// panel j0 to the trailing columns of G (mode 0) or Q's panel to B (mode 1) over total_blocks
// = sum ceil(k / QR_PANEL) column blocks; X = R^H; finish: B = [V; 0], X <- X Sigma^{-1} with
// sigma[j * max_n + c] the column norms of X.
void launch_qr_panel(const QrMat* mats, int nmats, int j0, int max_rows, void* stream);  // max_rows >= ell - j0
void launch_qr_apply(const QrMat* mats, int nmats, int total_blocks, int j0, int mode, void* stream);
void launch_qr_rt(const QrMat* mats, int nmats, void* stream);
void launch_qr_finish(const QrMat* mats, int nmats, const double* sigma, int max_k, void* stream);

}  // namespace tdmps
