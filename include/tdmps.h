/*
 * tdmps -- MPS time evolution of the ab-initio electronic Hamiltonian on one MI355X.
 *
 * C ABI of the library.  It follows the method of Frahm & Pfannkuche,
 * "Ultrafast ab-initio Quantum Chemistry Using Matrix Product States" (arXiv:1902.08489):
 * the time-dependent Schroedinger equation on the Fock space (Methods, Eqs. (sg) and
 * (time_evo_opera)) with the Hamiltonian of Eq. (hamil), states stored as matrix
 * product states (Eq. (mps)), and the three MPS operations of the "Operations on MPS"
 * section -- scaling, addition and application of the Hamiltonian, both done by the
 * variational fit of Eq. (add_min) -- composed into RK4 (the RK4 stage definitions and Eq. (rk_add)) and
 * Krylov (Eqs. (kry_non), (kry_orth), (krylov_evo)) time steps.
 *
 * Conventions
 *  - Atomic units (hbar = 1).  L spatial orbitals; orbital p holds the local state
 *    n = n_up + 2 n_dn: |0>, |up>, |dn>, |up dn> = a+_{p up} a+_{p dn} |0>.  Spin orbitals
 *    are ordered 1up, 1dn, 2up, 2dn, ...; a determinant |n_1 ... n_L> is the product of
 *    creators in that order (lowest leftmost) acting on the vacuum.
 *  - Dense state vectors have 4^L complex entries indexed by sum_p n_p 4^(L-1-p)
 *    (orbital 1 most significant).  Complex numbers are interleaved (re, im) doubles.
 *  - States are block sparse by the charge (N_up, N_dn) of the orbitals left of each
 *    bond (U(1) x U(1)).  A site tensor A_i[a, n, b] is stored, for each left sector in
 *    bond order, as a row-major panel of D_a rows whose columns are the blocks
 *    n = 0..3 (those whose right sector exists), each D_b wide.
 *  - Ownership: every `out` handle is new, owned by the caller and released with the
 *    matching *_destroy.  Host arrays passed in are copied and never retained.  Input
 *    handles are never modified except by the explicitly in-place calls.
 *  - Errors: a negative status is returned, `*out` is left NULL and tdmps_last_error()
 *    (thread local) describes the failure.  No C++ exception crosses this boundary.
 *  - Streams: all device work of a context is ordered on its stream.  Calls that return
 *    host scalars or host arrays synchronise that stream before returning.
 *  - Precision: contractions run in the precision of tdmps_fit_params.precision; the
 *    SVD truncation, the Krylov matrices and their exponential are always FP64.
 */
#ifndef TDMPS_H
#define TDMPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdmps_ctx_s* tdmps_ctx;
typedef struct tdmps_mpo_s* tdmps_mpo;
typedef struct tdmps_mps_s* tdmps_mps;
typedef struct tdmps_heff_s* tdmps_heff;
typedef struct tdmps_traj_s* tdmps_traj;
typedef int32_t tdmps_status;

enum {
  TDMPS_OK = 0,
  TDMPS_ERR_ARG = -1,         /* bad argument (size, NULL, occupation code, L)          */
  TDMPS_ERR_SECTOR = -2,      /* charge sectors of the operands do not match            */
  TDMPS_ERR_OOM = -3,         /* device or host allocation failed                       */
  TDMPS_ERR_HIP = -4,         /* a HIP runtime call failed                              */
  TDMPS_ERR_NUMERIC = -5,     /* NaN/Inf in inputs, or an SVD that did not converge      */
  TDMPS_ERR_SINGULAR = -6,    /* Krylov overlap matrix not positive definite            */
  TDMPS_ERR_UNSUPPORTED = -7  /* feature not available in this build                    */
};

/* Contraction precisions: FP64; FP32 products; BF16 split x = hi + lo (16 significant bits
 * per operand, three bf16 products per real product); BF16 three-term split x = hi + mid + lo
 * (all 24 bits of the FP32 value, six bf16 products: FP32 accuracy on the bf16 matrix units).
 * All accumulate in FP32 (the reduced ones) and keep SVD / Krylov algebra in FP64. */
enum { TDMPS_FP64 = 0, TDMPS_FP32 = 1, TDMPS_BF16X3 = 2, TDMPS_BF16X6 = 3 };
enum { TDMPS_KRYLOV_ORTHO = 0, TDMPS_KRYLOV_NONORTHO = 1 };

/* Parameters of the variational fit (Methods, Eq. (add_min)).
 *  Dmax       : maximal bond dimension D kept after every two-site update.
 *  n_sweeps   : maximal number of sweeps; a sweep is a left-to-right pass over the bonds
 *               followed by a right-to-left pass (the paper reports about ten).
 *  conv_tol   : stop when the relative change of |C|^2 between sweeps is below this
 *               (0 = always run n_sweeps).
 *  svd_cutoff : singular values <= svd_cutoff * sigma_max are dropped (at least one kept).
 *  precision  : TDMPS_FP64 / TDMPS_FP32 / TDMPS_BF16X3 / TDMPS_BF16X6 for the block
 *               contractions.  In the reduced precisions the H_eff products keep their operands and their
 *               intermediate in FP32 storage (FP32 copies of the environment operators and of
 *               theta); a context created with the environment variable TDMPS_MIXED_STORAGE=0
 *               keeps FP64 storage.  SVD, QR and the Krylov algebra are FP64 in every mode.
 *  batched    : 1 = one grouped launch per contraction stage (default); 0 = one launch
 *               per block product (reference form used for comparisons). */
typedef struct {
  int32_t Dmax;
  int32_t n_sweeps;
  double conv_tol;
  double svd_cutoff;
  int32_t precision;
  int32_t batched;
} tdmps_fit_params;

typedef struct {
  int32_t sweeps_used;
  int32_t max_bond;
  double discarded_max; /* largest discarded weight of one two-site update */
  double discarded_sum; /* sum over the updates of the last sweep          */
  double norm2;         /* |C|^2 of the result                             */
} tdmps_fit_info;

const char* tdmps_last_error(void);

/* Context: one GPU, one stream.  hip_stream may be NULL (the library creates and owns a
 * stream) or a borrowed hipStream_t that must outlive the context. */
tdmps_status tdmps_ctx_create(int32_t device, void* hip_stream, tdmps_ctx* out);
tdmps_status tdmps_ctx_destroy(tdmps_ctx ctx);
/* Counters of the last operation (fit, time step or expectation value), TDMPS_NCOUNTERS
 * doubles: out[0] = algorithmic flops of the H_eff contractions, out[1] = executed H_eff flops,
 * out[2..6] = wall seconds spent in H_eff, environment updates, SVD truncation (QR included),
 * premix and sandwiches (sandwich time includes its own environment updates and premix;
 * launches are asynchronous, so GPU time is charged to the phase that next waits for the
 * stream unless TDMPS_PHASE_TIMING was set when the context was created, which ends every
 * phase with a synchronisation),
 * out[7] = executed environment-update flops, out[8] = executed premix flops, out[9] / out[10]
 * = Jacobi sweeps / rounds summed over the SVDs, out[11..14] = number of SVD truncations,
 * H_eff applications, environment updates and sandwiches, out[15] = seconds in the QR
 * preconditioning, out[16] = host seconds spent building GEMM plans (included in the H_eff
 * and environment times), out[17] / out[18] = device allocations the caching allocator has
 * made so far in the process and the seconds spent in them, out[19] = premix structures built
 * so far in the process (misses of the cache of per-site coefficient matrices), out[20] =
 * weight discarded by the truncations of the last sweep of every fit of the operation, summed
 * over the fits (the squared-norm error the SVD truncations introduced).  After
 * tdmps_heff_apply planning, out[0..9] describe the plan instead: algorithmic flops, executed
 * flops of the two stages, bytes of the intermediate, task and segment counts of the two
 * stages, the number of shared-environment runs (channels of one environment block with
 * their own coefficients, summed by the share pass) and the bytes of their products. */
#define TDMPS_NCOUNTERS 21
tdmps_status tdmps_ctx_counters(tdmps_ctx ctx, double* out);
tdmps_status tdmps_ctx_reset_counters(tdmps_ctx ctx);
/* Launch mode of tdmps_heff_apply (Batching row of the benchmark set): 1 = every block product
 * of a contraction stage in one grouped launch per tile shape (default); 2 = the same grouped
 * launches recorded once per (plan, input, output) into a HIP graph on the context stream and
 * replayed as one graph launch afterwards (the context stream must then be a non-default
 * stream: contexts created with a NULL stream own one); 0 = one kernel launch per block
 * product, the per-block baseline.  All three give bit-identical results.  Fits and time
 * steps take the grouped/per-block choice from tdmps_fit_params.batched instead.
 * TDMPS_ERR_ARG for other values. */
tdmps_status tdmps_ctx_set_launch_mode(tdmps_ctx ctx, int32_t batched);
/* Tile shapes of the grouped block GEMM (Batching row).  There are TDMPS_TILE_CONFIGS shapes
 * (complex rows x columns: 64x64, 32x32, 128x32, 64x48, 96x48, 128x48, 32x48, 96x64, 96x32,
 * 64x32).  By default a task's shape is chosen by a padding / throughput cost model.
 * tdmps_ctx_autotune times every shape on synthetic grouped products for each bucket of
 * (rows, columns, total reduction length) at one precision and makes plans built afterwards
 * take the fastest shape of their task's bucket.  Buckets: rows and columns by the first of
 * 16, 32, 48, 64, 96, 128, 192, 256 that is >= the size (larger sizes in the last bucket);
 * reduction length by the first of 64, 512, 4096 (same rule).  cfg_out (int32) and
 * tflops_out (measured TFLOP/s of the chosen shape), both nullable, receive
 * TDMPS_TILE_BUCKETS entries in (rows, columns, reduction) row-major order.  Takes a few
 * seconds and ~300 MiB of device memory; results do not depend on the tile shape.
 * tdmps_ctx_set_tile_config forces one shape (0..TDMPS_TILE_CONFIGS-1) for every task, -1
 * returns to the tuned table or the cost model; tdmps_ctx_clear_tuning drops tuned tables.
 * Plans made before any of these calls are rebuilt on their next use. */
#define TDMPS_TILE_CONFIGS 10
#define TDMPS_TILE_BUCKETS 192
tdmps_status tdmps_ctx_autotune(tdmps_ctx ctx, int32_t precision, int32_t* cfg_out, double* tflops_out);
tdmps_status tdmps_ctx_set_tile_config(tdmps_ctx ctx, int32_t cfg);
tdmps_status tdmps_ctx_clear_tuning(tdmps_ctx ctx);

/* ---------------------------------------------------------------- Hamiltonian MPO
 * Exact MPO of Eq. (hamil): H = sum_pq h_pq a+_{p s} a_{q s}
 *   + 1/2 sum_pqrs (pr|qs) a+_{p s} a+_{q t} a_{s t} a_{r s} + e0,
 * i.e. V_ijkl = (ik|jl) from chemists' integrals.  h: L*L row-major symmetric; eri: L^4
 * row-major (pq|rs) with 8-fold symmetry.  Returns TDMPS_ERR_NUMERIC for NaN/Inf input.
 * Channels: identity, complete, one open operator (with its complementary three-operator sum),
 * and pairs of operators named by the smaller side of the cut; at the cuts within L/6 of the
 * chain centre (environment variable TDMPS_MPO_ROUTING_WINDOW: another distance, -1 none) a
 * pair whose opposite operator sits on the site next to the cut is named by the other side, so
 * every complementary crossing of a pair happens on a site without operators of the term.
 * tdmps_mpo_bond_dims reports the channels as built; with the plain rule (-1) the bond
 * dimension at the centre is 2L^2 + 3L + 2.  Algorithmic flop counts always refer to the
 * plain rule.
 * ctx may be NULL for a host-only operator (tdmps_mpo_to_dense, tdmps_mpo_det_element). */
tdmps_status tdmps_mpo_from_integrals(tdmps_ctx ctx, int32_t L, const double* h, const double* eri,
                                      double e0, tdmps_mpo* out);
/* Orbital order by a Fiedler reduction of the band width of the orbital coupling (the
 * ordering of the molecular orbitals in the H2O section): coupling w_ij = |h_ij| + |(ij|ji)|
 * for i != j (eri nullable: hopping only), orbitals sorted by the Fiedler vector of the graph
 * Laplacian diag(sum_j w_ij) - w.  perm (L entries): position k of the new order holds old
 * orbital perm[k]; reorder the integrals as h'[k][l] = h[perm[k]][perm[l]] (and likewise all
 * four indices of eri) before building the MPO.  Host only; TDMPS_ERR_NUMERIC for NaN/Inf. */
tdmps_status tdmps_fiedler_order(int32_t L, const double* h, const double* eri, int32_t* perm);
/* One-body operator sum_pq t_pq a+_{p s} a_{q s} (e.g. the dipole operator). */
tdmps_status tdmps_mpo_one_body(tdmps_ctx ctx, int32_t L, const double* t, tdmps_mpo* out);
/* Replace the one-body integrals of an MPO in place (time-dependent H(t) = H0 + E(t) mu). */
tdmps_status tdmps_mpo_set_one_body(tdmps_mpo mpo, const double* h);
/* MPO bond dimensions at the L+1 cuts. */
tdmps_status tdmps_mpo_bond_dims(tdmps_mpo mpo, int32_t* out);
/* Host-only checks: the dense 4^L x 4^L matrix (row-major, L <= 6) and <bra|H|ket> between
 * two determinants given as occupation codes. */
tdmps_status tdmps_mpo_to_dense(tdmps_mpo mpo, double* out, int64_t len);
tdmps_status tdmps_mpo_det_element(tdmps_mpo mpo, const uint8_t* bra, const uint8_t* ket, double* out);
tdmps_status tdmps_mpo_destroy(tdmps_mpo mpo);

/* ---------------------------------------------------------------- states (Eq. (mps))
 * Product state of one determinant; occ[p] in {0,1,2,3} (bit0 = up, bit1 = down). */
tdmps_status tdmps_mps_from_determinant(tdmps_ctx ctx, int32_t L, const uint8_t* occ, tdmps_mps* out);
/* General block-sparse state.  bond_nsec[i] (i = 0..L) sectors per bond; bond_sec lists
 * (n_up, n_dn, dim) for all sectors, bond by bond (bond 0 must be (0,0,1), bond L the
 * total charge with dim 1).  data holds the site tensors one after another in the panel
 * layout described above (interleaved complex); len = number of doubles. */
tdmps_status tdmps_mps_from_blocks(tdmps_ctx ctx, int32_t L, const int32_t* bond_nsec, const int32_t* bond_sec,
                                   const double* data, int64_t len, tdmps_mps* out);
/* Sector tables: writes L+1 counts into bond_nsec and 3 ints per sector into bond_sec
 * (either may be NULL to query *total_sectors first). */
tdmps_status tdmps_mps_sectors(tdmps_mps mps, int32_t* bond_nsec, int32_t* bond_sec, int64_t* total_sectors);
/* Site tensors in the panel layout (len doubles; query with data = NULL). */
tdmps_status tdmps_mps_get_blocks(tdmps_mps mps, double* data, int64_t* len);
/* Dense 4^L coefficient vector (interleaved complex, len = 2*4^L; L <= 12). */
tdmps_status tdmps_mps_to_dense(tdmps_mps mps, double* out, int64_t len);
/* State of a dense vector (tiny L only, 2 <= L <= 12) by the sequential SVD of the MPS
 * section of Methods (Eq. (mps)): split off one site after another from the left, keeping
 * at most Dmax singular values per bond (global descending order over the charge sectors of
 * the bond) and none at or below svd_cutoff * sigma_max; nothing is renormalised.
 *   coeffs : 4^L interleaved complex coefficients in the dense order of tdmps_mps_to_dense
 *            (len = 2*4^L doubles), all zero outside the sector of N electrons with
 *            2Sz = N_up - N_dn (else TDMPS_ERR_SECTOR); copied, not retained.
 * The result has bond dimensions <= Dmax (the exact state when Dmax >= D_FCI).
 * TDMPS_ERR_NUMERIC for NaN/Inf coefficients. */
tdmps_status tdmps_mps_from_dense(tdmps_ctx ctx, int32_t L, int32_t N, int32_t twoSz, const double* coeffs,
                                  int64_t len, int32_t Dmax, double svd_cutoff, tdmps_mps* out);
/* Checkpoint files (for resuming a time evolution).  tdmps_mps_save writes the state to
 * path: an 8-byte magic "TDMPSv1\0", int32 L, N_up, N_dn, 0, then per bond int32 count and
 * count x (int32 n_up, n_dn, dim), then per site int64 n and n interleaved complex FP64 values
 * in the panel layout, then a 64-bit FNV-1a checksum of everything before it (little
 * endian).  tdmps_mps_load reads such a file into a new state on ctx: the same bonds and the
 * same bits, so a run continued from it is bitwise the run that was saved.  TDMPS_ERR_ARG for
 * unreadable, truncated, inconsistent or corrupt files (checksum), TDMPS_ERR_NUMERIC for
 * non-finite values. */
tdmps_status tdmps_mps_save(tdmps_mps mps, const char* path);
tdmps_status tdmps_mps_load(tdmps_ctx ctx, const char* path, tdmps_mps* out);
tdmps_status tdmps_mps_copy(tdmps_mps mps, tdmps_mps* out);
tdmps_status tdmps_mps_bond_dims(tdmps_mps mps, int32_t* out);
tdmps_status tdmps_mps_destroy(tdmps_mps mps);

/* ---------------------------------------------------------------- operations
 * Scaling (Operations on MPS): multiplies one site tensor by alpha (re, im), in place. */
tdmps_status tdmps_mps_scale(tdmps_mps mps, const double* alpha);
/* <a|b> (re, im). */
tdmps_status tdmps_mps_overlap(tdmps_mps a, tdmps_mps b, double* out);
/* <bra|O|ket> (re, im) for an MPO O. */
tdmps_status tdmps_mps_expect(tdmps_mpo op, tdmps_mps bra, tdmps_mps ket, double* out);
/* Variational fit (Eq. (add_min)): out ~ alpha H psi + sum_j beta_j phi_j with bonds <= Dmax.
 * alpha: (re, im); beta: 2*nterms doubles; phi: nterms states (may be 0).  The initial
 * guess is psi, right-canonicalised.  info may be NULL. */
tdmps_status tdmps_mps_apply_H(tdmps_mpo H, const double* alpha, tdmps_mps psi, int32_t nterms, const double* beta,
                               const tdmps_mps* phi, const tdmps_fit_params* prm, tdmps_mps* out,
                               tdmps_fit_info* info);
/* MPS addition by the same fit: out ~ sum_j beta_j phi_j (nterms >= 1); the initial
 * guess is phi[0], right-canonicalised. */
tdmps_status tdmps_mps_compress(int32_t nterms, const double* beta, const tdmps_mps* phi,
                                const tdmps_fit_params* prm, tdmps_mps* out, tdmps_fit_info* info);

/* One-particle reduced density matrix gamma_pq = sum_s <psi|a+_{ps} a_{qs}|psi> / <psi|psi>
 * (the accuracy measure of the time-evolved states, H2O section) for all p, q in one
 * left-to-right sweep over a right-canonical copy of psi (no truncation).  gamma: L*L
 * interleaved complex, row-major (p, q), Hermitian, trace N.  TDMPS_ERR_NUMERIC for a zero
 * state. */
tdmps_status tdmps_mps_one_rdm(tdmps_mps psi, double* gamma);

/* c_{site, spin}|psi> exactly (spin 0 = up, 1 = down), the ionisation step of the Green's
 * function of Eq. (green_time): the site tensors left of site take the Jordan-Wigner sign,
 * site takes the local annihilator, the bonds right of site lose the removed charge.  The
 * result is a new state in the sector with one electron of that spin less (no truncation).
 * TDMPS_ERR_SECTOR if psi has no electron of that spin, TDMPS_ERR_ARG for site/spin out of
 * range. */
tdmps_status tdmps_mps_annihilate(tdmps_mps psi, int32_t site, int32_t spin, tdmps_mps* out);
/* Ground state by restarted Krylov (Lanczos) iterations on the same kernels as the time step
 * (the initial state psi_0 of Eq. (green_time)): each restart builds an orthogonal Krylov
 * basis of m states from the current iterate and replaces it by the normalised lowest Ritz
 * state; energy (nullable) receives the last Ritz value.  TDMPS_ERR_ARG for restarts < 1. */
tdmps_status tdmps_krylov_ground(tdmps_mpo H, tdmps_mps psi, int32_t m, int32_t restarts,
                                 const tdmps_fit_params* prm, tdmps_mps* out, double* energy);

/* ---------------------------------------------------------------- time steps
 * Krylov step (Eqs. (kry_orth)/(kry_non), (krylov_evo)): basis of m states, the first
 * psi/|psi|; each next one fitted from H phi^k (minus the projections on all previous
 * vectors for TDMPS_KRYLOV_ORTHO) and normalised; N and H from overlaps and sandwiches;
 * out ~ |psi| sum_k [exp(-i dt N^-1 H)]_{k0} phi^k.  Nmat/Hmat (m*m interleaved complex,
 * row-major) may be NULL.  With TDMPS_KRYLOV_ORTHO the basis stops early when the space is
 * invariant (the part of H phi^k orthogonal to the basis below 1e-10 of H phi^k, e.g. psi an
 * eigenstate): the step then uses the vectors found so far and the unused rows and columns
 * of Nmat/Hmat are 0.  Returns TDMPS_ERR_SINGULAR if N is not positive definite. */
tdmps_status tdmps_krylov_step(tdmps_mpo H, tdmps_mps psi, double dt, int32_t m, int32_t flags,
                               const tdmps_fit_params* prm, tdmps_mps* out, double* Nmat, double* Hmat);
/* RK4 step (the RK4 stage definitions and Eq. (rk_add)) with k_s = -i dt H(t_s) u_s fitted, u_s compressed:
 * four H applications and four additions.  H_t, H_mid, H_t1 are the operators at t,
 * t + dt/2 and t + dt (pass the same handle three times for a static H). */
tdmps_status tdmps_rk4_step(tdmps_mpo H_t, tdmps_mpo H_mid, tdmps_mpo H_t1, tdmps_mps psi, double dt,
                            const tdmps_fit_params* prm, tdmps_mps* out, tdmps_fit_info* info);

/* ---------------------------------------------------------------- kernel-level access
 * The two-site effective Hamiltonian at bond (site, site+1) between bra and ket states
 * (the local operator of the fit): builds the left environment of sites < site and the
 * right environment of sites > site+1 once; apply() then maps a ket two-site tensor
 * theta[a, n1, n2, b] to sum L W W R theta in the bra layout.  Two-site tensors use the
 * panel layout with blocks ordered (n1, n2) = (0,0), (0,1), ..., (3,3). */
tdmps_status tdmps_heff_create(tdmps_mpo H, tdmps_mps bra, tdmps_mps ket, int32_t site, int32_t precision,
                               tdmps_heff* out);
/* Layout of the ket (which = 0) or bra (which = 1) two-site tensor: total doubles and the
 * number of blocks; blocks (may be NULL) receives per block (n_up_a, n_dn_a, n1, n2, D_a,
 * D_b, offset_in_doubles_lo, offset_hi, ld). */
tdmps_status tdmps_heff_layout(tdmps_heff op, int32_t which, int64_t* total_doubles, int64_t* nblocks,
                               int32_t* blocks);
/* theta_out = H_eff theta_in; both device pointers (FP64 interleaved complex). */
tdmps_status tdmps_heff_apply(tdmps_heff op, const void* theta_in_dev, void* theta_out_dev);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same product as tdmps_heff_apply, bit for bit, with
 * every buffer beyond theta_in / theta_out -- the H_eff intermediate, split-K partial sums,
 * products of shared environment blocks and the task tables -- placed in a fixed device
 * scratch of TDMPS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends (its address is resolved when a context is created on that GPU).  No device
 * memory is allocated or freed (host-side planning uses the C++ heap).  Returns TDMPS_ERR_ARG,
 * before any kernel runs and with theta_out untouched, when the operator needs more scratch
 * than that (the intermediate alone is ~ MPO bond dimension x the two-site tensor: e.g. fine
 * for L = 8 at D = 64, too large for L = 10 at D = 256).  Every call on a GPU reuses the same scratch
 * and lays out its plan anew: calls that overlap in time on one GPU (other threads, other
 * streams) race and must not be issued.  Returns after the context stream has finished. */
#define TDMPS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tdmps_status tdmps_heff_apply_noalloc(tdmps_heff op, const void* theta_in_dev, void* theta_out_dev);
/* Contraction precision of later applies (TDMPS_FP64, TDMPS_FP32, TDMPS_BF16X3, TDMPS_BF16X6); the
 * environments are kept.  TDMPS_ERR_ARG for other values. */
tdmps_status tdmps_heff_set_precision(tdmps_heff op, int32_t precision);
/* Algorithmic flops of one apply (8 per complex multiply-add of the block products). */
tdmps_status tdmps_heff_flops(tdmps_heff op, double* flops);
tdmps_status tdmps_heff_destroy(tdmps_heff op);

/* ---------------------------------------------------------------- differentiation
 * Field-driven dynamics: H(t) = H0 + E(t) M with E(t) = amplitude * sin(omega t) *
 * exp(-(t - t_center)^2 / (2 width^2)); the field enters through the one-body integrals of
 * Eq. (hamil), h(t) = h0 + E(t) m.  tdmps_pulse_forward propagates psi0 by nsteps RK4 steps
 * (the RK4 stage definitions and Eq. (rk_add); stage times t, t+dt/2, t+dt/2, t+dt) and returns
 * D = <psi_N|mu|psi_N> / <psi_N|psi_N>, keeping psi every checkpoint_every steps in the
 * trajectory handle.  tdmps_pulse_backward returns dD/d(amplitude) by the adjoint of the
 * discrete RK4 map: the states between checkpoints are recomputed and the adjoint stages
 * are propagated backwards with the same fit / H_eff / environment kernels (H Hermitian, so
 * the adjoint of an H application is an H application with -i dt -> +i dt).  At full bond
 * dimension (every fit exact and converged) the result is the exact derivative of the discrete
 * map.  Below it the adjoint stage maps are applied by fits of their own, each truncated to
 * Dmax: the result then approximates the derivative of the truncated forward map, with an
 * error of the order of the truncation (it does not differentiate the choice of the kept
 * singular vectors).
 *   H0       : MPO of H0 (its one-body part is replaced by h0 + E(t) m at every stage time).
 *   h0, m    : L*L row-major one-body integrals of H0 and of the field coupling.
 *   mu       : observable MPO (e.g. tdmps_mpo_one_body of the dipole integrals).
 *   The trajectory owns copies of all inputs; destroy it with tdmps_traj_destroy. */
typedef struct {
  double amplitude, omega, t_center, width;
} tdmps_pulse;
tdmps_status tdmps_pulse_forward(tdmps_mpo H0, const double* h0, const double* m, tdmps_mpo mu, tdmps_mps psi0,
                                 const tdmps_pulse* pulse, double dt, int32_t nsteps, int32_t checkpoint_every,
                                 const tdmps_fit_params* prm, tdmps_traj* out, double* value);
tdmps_status tdmps_pulse_backward(tdmps_traj traj, double* dvalue_damplitude);
tdmps_status tdmps_traj_destroy(tdmps_traj traj);

#ifdef __cplusplus
}
#endif

#endif /* TDMPS_H */
