// Host-side data structures of the block-sparse MPS engine and its internal API.
#pragma once

#include <array>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "mpo.h"

struct tdmps_ctx_s;

namespace tdmps {

const char* last_error_cstr();

// Runs f, converting exceptions to a status code and the thread-local message.
template <class F>
tdmps_status guard(F&& f) {
  try {
    f();
    return TDMPS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return TDMPS_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return TDMPS_ERR_ARG;
  }
}

// ---------------------------------------------------------------- device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool own = true;  // false: a view of memory owned elsewhere (an Arena), never freed
  DevBuf() = default;
  explicit DevBuf(size_t b);
  ~DevBuf();
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), own(o.own) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      own = o.own;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  void release();
  cplx* c() const { return (cplx*)p; }
};

// Bump allocation over a fixed device region (the no-allocation entry point's scratch):
// take() hands out 256-byte aligned pieces and throws TDMPS_ERR_ARG beyond the capacity.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes);
  DevBuf view(size_t bytes);  // non-owning DevBuf over take(bytes)
};

// ---------------------------------------------------------------- bonds and layouts
struct Bond {
  std::vector<Charge> q;  // sorted ascending
  std::vector<int> dim;
  int find(Charge c) const;
  int nsec() const { return (int)q.size(); }
  int total() const {
    int t = 0;
    for (int d : dim) t += d;
    return t;
  }
};

// Site tensor A[a, n, b]: per left sector a row-major panel D_a x width whose columns are
// the blocks n = 0..3 (right sector rs[a][n], column offset col[a][n]).
struct SiteLayout {
  std::vector<int64_t> panel_off;
  std::vector<int> width;
  std::vector<std::array<int, 4>> rs, col;
  int64_t size = 0;
  void build(const Bond& l, const Bond& r);
};

// Two-site tensor theta[a, n1, n2, b] with combined index n = 4 n1 + n2.
struct TwoLayout {
  std::vector<int64_t> panel_off;
  std::vector<int> width;
  std::vector<std::array<int, 16>> rs, col;
  int64_t size = 0;
  void build(const Bond& l, const Bond& r);
};

inline Charge pair_charge(int n) { return local_charge(n >> 2) + local_charge(n & 3); }

// Measured tile shape per block-size bucket of the grouped GEMM (tdmps_ctx_autotune).
// Buckets: output rows and columns by TILE_EDGES (the first edge >= the size), total complex
// reduction length per output by TILE_KEDGES.
constexpr int TILE_NB = 8, TILE_NK = 3;
constexpr int TILE_EDGES[TILE_NB] = {16, 32, 48, 64, 96, 128, 192, 256};
constexpr int TILE_KEDGES[TILE_NK] = {64, 512, 4096};
struct TileTable {
  bool valid = false;
  int8_t cfg[TILE_NB][TILE_NB][TILE_NK] = {};
  float tflops[TILE_NB][TILE_NB][TILE_NK] = {};  // rate of the chosen shape in the tuning run
};
inline int tile_bucket(int64_t x) {
  for (int i = 0; i < TILE_NB; ++i)
    if (x <= TILE_EDGES[i]) return i;
  return TILE_NB - 1;
}
inline int tile_kbucket(int64_t k) {
  for (int i = 0; i < TILE_NK; ++i)
    if (k <= TILE_KEDGES[i]) return i;
  return TILE_NK - 1;
}
// Times every tile shape on synthetic grouped products of each bucket and fills t.
void autotune_tiles(struct ::tdmps_ctx_s* ctx, int precision, TileTable& t);

}  // namespace tdmps

struct tdmps_ctx_s {
  int device = 0;
  void* stream = nullptr;
  bool own_stream = false;
  void* ev[2] = {nullptr, nullptr};
  double counters[TDMPS_NCOUNTERS] = {0};
  // launch mode of the H_eff handle API (tdmps_ctx_set_launch_mode): 0 = one launch per block
  // product, 1 = grouped launches, 2 = grouped launches captured once into a HIP graph and replayed
  int batched = 1;
  // Tile shape of the grouped GEMM: tile_cfg >= 0 forces one configuration for every task;
  // otherwise a tuned table (tdmps_ctx_autotune) is used where present, else the cost model.
  int tile_cfg = -1;
  tdmps::TileTable tune[4];  // per precision
  int tune_gen = 0;  // bumped whenever the tile choice rules change (plans made before are stale)
  // Work of a context is ordered on one stream, so the host synchronises only where it reads
  // device data.  With phase_sync (environment variable TDMPS_PHASE_TIMING set at context
  // creation) every contraction stage also ends in a synchronisation, so that the per-phase
  // wall-clock counters measure device time (at the cost of host / device overlap).
  bool phase_sync = false;
  bool timing = false;
  // FP32 / BF16-split H_eff applies keep their operands and the T intermediate in FP32 storage
  // (converted once per plan; environment variable TDMPS_MIXED_STORAGE=0 at context creation
  // keeps them in FP64 and converts while staging tiles)
  bool mixed_storage = true;
};

struct tdmps_mps_s {
  tdmps_ctx ctx = nullptr;
  int L = 0;
  tdmps::Charge total;
  std::vector<tdmps::Bond> bond;        // L + 1
  std::vector<tdmps::SiteLayout> lay;   // L
  std::vector<tdmps::DevBuf> site;      // L
};

struct tdmps_mpo_s {
  tdmps_ctx ctx = nullptr;
  tdmps::MpoHost host;
};

namespace tdmps {

using Ctx = tdmps_ctx_s;
using Mps = tdmps_mps_s;

// ---------------------------------------------------------------- environment-like data
// Groups of n "channels" with common charge q.  For every ket sector k whose bra sector
// b (q_b = q_k + q) exists, a stack [n][D_b][D_k] (row-major blocks) is stored.
struct StackGroup {
  Charge q;
  int n = 0;
  std::vector<int> bra_of;   // per ket sector
  std::vector<int> ket_of;   // per bra sector
  std::vector<int64_t> off;  // per ket sector, -1 if absent
};

struct Blocks {
  Bond bra, ket;
  std::vector<StackGroup> grp;
  DevBuf data;
  int64_t size = 0;
  void layout(const Bond& b, const Bond& k, const std::vector<std::pair<Charge, int>>& groups);
  cplx* stack(int g, int ks) const { return grp[g].off[ks] < 0 ? nullptr : data.c() + grp[g].off[ks]; }
};

// Environment of an MPO cut: one group per channel class of the cut.
struct Env {
  int cut = 0;
  Blocks b;
};

// Operator of a middle channel for one local matrix unit (s, sp): coef * source[grp][idx].
struct OpRef {
  const Blocks* src = nullptr;
  int grp = 0, idx = 0;
  double coef = 0;
};

struct ChanOps {
  std::vector<int> pat;  // local matrix unit 4*s + sp
  std::vector<OpRef> ref;
};

// Environment operators combined with one site tensor of the MPO, per channel of the
// middle cut and local matrix unit (premix).  Single-source entries alias the
// environment; multi-source ones are linear combinations computed on the device.
struct SideOps {
  int cut = 0;  // middle cut
  const Env* env = nullptr;
  std::vector<ChanOps> ch;
  std::unique_ptr<Blocks> mix;
  std::shared_ptr<DevBuf> wmat;  // premix coefficients (device), alive until the premix plan ran
  // (charge, count) channel classes of the environment's cut under the plain operator rule
  // (MpoHost::plain_cls), for the algorithmic flop count; null: the environment's own classes
  const std::vector<std::pair<Charge, int>>* ref_cls = nullptr;
};

// ---------------------------------------------------------------- GEMM plans
struct GemmPlan {
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
  double flops = 0;  // executed flops (8 per complex multiply-add)
  double host_s = 0;  // host seconds spent in finalize() by run()
  int begin_task(cplx* C, int64_t bsC, int ldc, int m, int n, int nbatch, bool accum);
  void add_seg(const cplx* A, int64_t bsA, int64_t rsA, int lda, int opA, const cplx* B, int64_t bsB, int64_t rsB,
               int ldb, int opB, int k, int nred, cplx alpha);
  // device copies of the task lists (finalize) and asynchronous launch
  static constexpr int NCFG = GEMM_NCFG;
  // all task tables of the plan in one device buffer (one upload)
  DevBuf dtab, wspace;
  // caller data uploaded with the task tables (one upload per plan); device copy at dextra
  std::vector<char> extra;
  const char* dextra = nullptr;
  const GemmSeg* dsegs = nullptr;
  const GemmTask* dtasks[NCFG] = {};
  const int32_t* dtile[NCFG] = {};
  const ReduceTask* dred = nullptr;
  std::vector<int64_t> htile_base[NCFG];  // first tile of every task (per-task launches)
  std::vector<int64_t> red_base;
  int nred_tasks = 0;
  int ntask[NCFG] = {};
  int64_t ntiles[NCFG] = {};
  bool final_ = false;
  // task and segment counts as built (finalize hands the host lists back to a per-thread
  // pool, so that their capacity is reused by the next plan instead of faulted in again)
  size_t ntasks_built = 0, nsegs_built = 0;
  size_t task_count() const { return final_ ? ntasks_built : tasks.size(); }
  size_t seg_count() const { return final_ ? nsegs_built : segs.size(); }
  // with an arena, the split-K workspace and the tables are placed in it and the upload waits
  // for its completion (nothing is allocated)
  Arena* arena = nullptr;
  // operands A and B of every segment are FP32 complex (the mixed precisions' storage)
  bool ops32 = false;
  // every segment's A is real-valued (premix coefficients): FP64 real-A products, 4 flops per
  // multiply-add executed (set before the first add_seg)
  bool real_a = false;
  void finalize(Ctx* ctx, int precision);
  // batched: one grouped launch per tile shape (default); else one launch per task (the
  // per-block baseline the grouped launch is compared with)
  void launch(Ctx* ctx, int precision, bool batched = true);
  void run(Ctx* ctx, int precision, bool batched = true);  // finalize + launch + synchronise
  bool empty() const { return task_count() == 0; }
};

struct CopyPlan {
  std::vector<CopyTask> tasks;
  void add(const cplx* src, int64_t src_rs, int64_t src_cs, cplx* dst, int dst_ld, int rows, int cols, int flags,
           const int32_t* ridx = nullptr, const int32_t* cidx = nullptr, const double* rs = nullptr,
           const double* cs = nullptr);
  void run(Ctx* ctx);
};

// Host vectors copied to the device for the lifetime of an operation.
struct Staging {
  std::vector<DevBuf> bufs;
  template <class T>
  const T* put(Ctx* ctx, const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    bufs.emplace_back(v.size() * sizeof(T));
    dev_h2d(bufs.back().p, v.data(), v.size() * sizeof(T), ctx->stream);
    return (const T*)bufs.back().p;
  }
};

// ---------------------------------------------------------------- engine API
struct Contractor {
  Ctx* ctx;
  int precision = TDMPS_FP64;
  int batched = 1;
  double heff_flops = 0, env_flops = 0, mix_flops = 0;
  double heff_alg_flops = 0;
  // wall-clock seconds per phase (every phase ends with a stream synchronisation)
  double t_heff = 0, t_env = 0, t_mix = 0, t_svd = 0, t_sandwich = 0, t_qr = 0;
  double svd_sweeps = 0, svd_rounds = 0, n_svd = 0, n_heff = 0, n_env = 0, n_sandwich = 0;
  double t_plan = 0;  // host seconds building and finalising GEMM plans (H_eff and environments)
  double fit_discarded = 0;  // sum over the fits of the weight discarded in their last sweep
};

double wall_seconds();

Mps* mps_new(Ctx* ctx, int L, const std::vector<Bond>& bonds);
Mps* mps_clone(const Mps* m);
void mps_from_det(Mps* m, const uint8_t* occ);
MpoHost identity_mpo(int L);

Env env_left_boundary(Ctx* ctx, const Bond& bra0, const Bond& ket0);
Env env_right_boundary(Ctx* ctx, const Bond& braL, const Bond& ketL, int L);

SideOps premix_left(Contractor& C, const Env& L, const MpoHost& W, int site);
SideOps premix_right(Contractor& C, const Env& R, const MpoHost& W, int site);

// Premix structures built so far in the process (misses of the per-operator cache).
double premix_structures_built();
// Drops the cached premix structures of an operator version that no operator holds any more
// (its one-body part was rewritten): they could never be hit again.
void premix_cache_forget(uint64_t version);
Env env_left_update(Contractor& C, const SideOps& ops, const Mps* bra, const cplx* bra_site, const SiteLayout& bl,
                    const Bond& bra_l, const Bond& bra_r, const cplx* ket_site, const SiteLayout& kl,
                    const Bond& ket_l, const Bond& ket_r, const MpoHost& W);
Env env_right_update(Contractor& C, const SideOps& ops, const cplx* bra_site, const SiteLayout& bl, const Bond& bra_l,
                     const Bond& bra_r, const cplx* ket_site, const SiteLayout& kl, const Bond& ket_l,
                     const Bond& ket_r, const MpoHost& W);

// theta_out (bra two-site layout) (+)= alpha * H_eff theta_in (ket two-site layout)
struct HeffPlan {
  // T stage: p1 stacked over runs, p1b products of blocks shared by a run (combined into the
  // channels' rows by the share pass); p2 final stage
  GemmPlan p1, p1b, p2;
  DevBuf T, X;  // T intermediate (FP32 complex with ops32); products of shared blocks (FP64)
  // FP32 storage of the mixed precisions: FP32 copies of the environment operators (made when
  // the plan is built) and of theta_in (made by every launch)
  bool ops32 = false;
  std::vector<DevBuf> shadows;
  DevBuf theta32;
  const cplx* theta_in = nullptr;
  int64_t theta_size = 0;
  std::vector<double> coef_host;
  std::vector<ShareTask> share_host;  // uploaded with p1b's tables: [tasks][coefficients]
  int64_t share_max_blk = 0;
  size_t share_coef_off = 0;  // byte offset of the coefficients in p1b.extra
  cplx* out = nullptr;
  int64_t out_size = 0;
  bool accumulate = false;
  double alg_flops = 0;
  void launch(Ctx* ctx, int precision, bool batched = true);
};
// arena (nullable): intermediates, workspaces and task tables in that region, no allocation
std::unique_ptr<HeffPlan> heff_plan(Contractor& C, const SideOps& lops, const SideOps& rops, const cplx* theta_in,
                                    const TwoLayout& kl, const Bond& ket_l, const Bond& ket_r, cplx* theta_out,
                                    const TwoLayout& bl, const Bond& bra_l, const Bond& bra_r, cplx alpha,
                                    bool accumulate, Arena* arena = nullptr);
void heff_apply(Contractor& C, const SideOps& lops, const SideOps& rops, const cplx* theta_in, const TwoLayout& kl,
                const Bond& ket_l, const Bond& ket_r, cplx* theta_out, const TwoLayout& bl, const Bond& bra_l,
                const Bond& bra_r, cplx alpha, bool accumulate, double* alg_flops);

// theta (two-site) = A_i A_{i+1}
void form_theta(Contractor& C, const Mps* m, int i, cplx* theta, const TwoLayout& tl);

// full left sweep of environments: <bra|O|ket>
cplx sandwich(Contractor& C, const MpoHost& O, const Mps* bra, const Mps* ket);

struct TruncResult {
  Bond mid;
  double discarded = 0, norm2 = 0;
  int kept = 0;
};
// SVD of a two-site tensor (bra layout over bonds l, r), truncation to Dmax, and the
// split into the two site tensors.  move_right: A_i = U, A_{i+1} = S V^H; else A_i = U S,
// A_{i+1} = V^H.  The new site buffers and layouts are written into m at i, i+1.
TruncResult split_theta(Contractor& C, const cplx* theta, const TwoLayout& tl, Mps* m, int i, int Dmax, double cutoff,
                        bool move_right);
void right_canonicalize(Contractor& C, Mps* m, double cutoff);

struct FitTerm {
  cplx beta;
  const Mps* phi;
};
struct FitOut {
  int sweeps = 0;
  double disc_max = 0, disc_sum = 0, norm2 = 0;
  // <out|H|psi> of the returned state (H term only, without alpha), read off the last local
  // problem of the last sweep: at bond (0, 1) the right environment is built from the final
  // sites, so the local projection of H psi dotted with the final two-site tensor is exact.
  // Set when H is given.
  cplx h_out_psi{0, 0};
  // <out|phi_j> for every fit term, read off the same local problem.
  std::vector<cplx> term_overlaps;
};
// out ~ alpha * H psi + sum_j beta_j phi_j  (H may be null: compression only)
// grow_on_h: the first left-to-right pass fits alpha H psi alone (orthogonal Krylov vectors)
Mps* fit(Contractor& C, const MpoHost* H, cplx alpha, const Mps* psi, const std::vector<FitTerm>& terms,
         const tdmps_fit_params& prm, FitOut* info, bool grow_on_h = false);

void scale_mps(Ctx* ctx, Mps* m, cplx alpha);
cplx overlap(Contractor& C, const Mps* a, const Mps* b);
// <bra_j|O|ket> for all bras: the environment sweeps of all bras advance site by site together,
// each premix / environment stage of all bras in one grouped launch.
std::vector<cplx> sandwich_many(Contractor& C, const MpoHost& O, const std::vector<const Mps*>& bras, const Mps* ket);

}  // namespace tdmps
