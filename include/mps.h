/*
 * mps.h -- C ABI of libmps, the gfx950 (MI355X) two-site MPS update.
 *
 * The library implements the hot path of matrix-product-state time evolution
 * described in Jaschke, Wall, Carr, "Open source Matrix Product States"
 * (arXiv:1703.00387):
 *   theta = A_i . A_{i+1}          (Sec. "Basic concepts", Contractions)
 *   theta' = G theta or exp(-i tau H_eff) theta
 *                                  (Secs. "Sornborger-Stewart decomposition",
 *                                   "Krylov time evolution", App. "Details of
 *                                   the Krylov method")
 *   theta' = U S V^dag, cut to chi (Sec. "Basic concepts", Splitting; Eqs.
 *                                   overlap and elocal; App. "Auxiliary
 *                                   calculations")
 *
 * Conventions for every entry point
 * ---------------------------------
 * - complex64  = interleaved (re, im) float; complex128 = interleaved double.
 * - All arrays are row-major (C order).  Device pointers unless stated.
 * - Every call is asynchronous on `stream` (a hipStream_t; NULL = default
 *   stream) and returns an mps_status.  Argument and shape errors return at
 *   once, before any work is queued; the message is kept in mps_last_error().
 *   Numerical problems found on the device (non-finite values, a Jacobi or
 *   Lanczos iteration that did not converge) set bits of a device status word
 *   that mps_device_status() reads; the call still writes a best-effort
 *   result.  No C++ exception and no abort crosses this ABI.
 * - Ownership: the caller owns every input and output buffer.  A handle from
 *   mps_create owns a device workspace that it grows with hipMalloc when a
 *   call needs more (never while the stream is being captured: reserve first
 *   with mps_reserve); it is freed by mps_destroy.  A handle from
 *   mps_create_ws works in the caller's workspace instead and never
 *   allocates or frees device memory after its creation: a call that needs
 *   more than the caller gave returns MPS_ERR_CAPACITY (sizes from
 *   mps_workspace_size or mps_workspace_needed).  No pointer passed in is kept
 *   after a call returns, except that workspace.
 * - Calls that share one handle must not run concurrently on different
 *   streams: they share the workspace.
 */
#ifndef MPS_H_
#define MPS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPS_OK = 0,
  MPS_ERR_INVALID = 1,     /* bad argument (NULL pointer, bad flag, ...)      */
  MPS_ERR_SHAPE = 2,       /* inconsistent dimensions                         */
  MPS_ERR_CAPACITY = 3,    /* a size beyond a compiled or declared capacity   */
  MPS_ERR_NOCONV = 4,      /* iteration did not converge (device status bit)  */
  MPS_ERR_NONFINITE = 5,   /* NaN/Inf met on the device (device status bit)   */
  MPS_ERR_HIP = 6,         /* a HIP runtime call failed                       */
  MPS_ERR_UNSUPPORTED = 7  /* valid request the library does not implement    */
} mps_status;

/* bits of the device status word */
#define MPS_DEV_NOCONV_SVD     0x1u
#define MPS_DEV_NOCONV_LANCZOS 0x2u
#define MPS_DEV_NONFINITE      0x4u
#define MPS_DEV_SCHED_TIMEOUT  0x8u  /* a persistent kernel's bounded wait ran out */
#define MPS_DEV_CHARGE         0x10u /* a bond of a charge-carrying chain whose rows and columns share
                                        no charge (or whose bond dimension is out of range): that
                                        update was skipped, the bond keeps its tensors */

typedef struct mps_context* mps_handle;
typedef void* mps_stream; /* hipStream_t */

/* Create a handle bound to HIP device `device` (made current).  */
mps_status mps_create(mps_handle* h, int device);
/* Create a handle that works in the caller's device workspace
 * [workspace, workspace + ws_bytes) (256-byte aligned, owned by the caller,
 * kept until mps_destroy).  The handle's own small buffers (status word,
 * counters of the persistent Jacobi: about 9 MB) are allocated here; no call
 * on this handle allocates or frees device memory afterwards.  Column-split
 * Jacobi rounds keep their partial Grams behind each call's plan, and use
 * fewer column slices when the workspace leaves less room. */
mps_status mps_create_ws(mps_handle* h, int device, void* workspace, size_t ws_bytes);
/* Operations of mps_workspace_size. */
#define MPS_OP_TRUNCATE 0 /* mps_truncate of a (d chi_max) x (d chi_max) matrix              */
#define MPS_OP_TEBD     1 /* mps_tebd_step (dense chains, any order) of n_chains chains      */
#define MPS_OP_HEFF     2 /* mps_heff_apply, two sites, chi_l = chi_r = chi_max, w = w_l,m,r  */
#define MPS_OP_KRYLOV   3 /* mps_krylov_expm with those operands and n_krylov vectors       */
#define MPS_OP_TDVP     4 /* mps_tdvp2_step of a chain of L sites, MPO dimension w          */
/* Device workspace bytes that a call of `op` needs at the given capacities
 * (host only, no device work): n_chains chains of L sites, local dimension
 * d, bond capacity chi_max, element type dtype (MPS_C64 or MPS_C128), MPO
 * dimension w and Krylov vectors n_krylov where they apply.  The figure comes
 * from the entry point's own planning (run without any work) plus room for
 * the column split of one large matrix.  0 for arguments the call refuses. */
size_t mps_workspace_size(int32_t op, int32_t dtype, int32_t n_chains, int32_t L, int32_t d, int32_t chi_max,
                          int32_t w, int32_t n_krylov);
/* Largest workspace any call on this handle has planned so far. */
mps_status mps_workspace_needed(mps_handle h, size_t* bytes);
/* Free the handle and its workspace (synchronises the device first; a
 * caller-owned workspace is left to the caller). */
mps_status mps_destroy(mps_handle h);
/* Message of the last error returned on this handle ("" if none). */
const char* mps_last_error(mps_handle h);
/* Make the workspace at least `bytes` large (hipMalloc happens here; a
 * caller-owned workspace that is smaller gives MPS_ERR_CAPACITY). */
mps_status mps_reserve(mps_handle h, size_t bytes);
/* Synchronise `stream`, return and clear the device status word.  Returns
 * MPS_ERR_NONFINITE, MPS_ERR_NOCONV (NOCONV or SCHED_TIMEOUT bits) or
 * MPS_ERR_SHAPE (MPS_DEV_CHARGE) when such a bit was set, in that order. */
mps_status mps_device_status(mps_handle h, mps_stream stream, uint32_t* word);
/* Tuning knobs: 0 = Jacobi relative tolerance (default 1e-13),
 * 1 = Jacobi maximum sweeps (default 30), 2 = Jacobi absolute tolerance
 * relative to |theta|_F^2 (default 1e-15, at least 1e-30: under a purely
 * relative criterion the rows beyond the rank of a matrix with more rows
 * than columns never count as orthogonal and end as NaN rows), 3 = kernel timing on (!= 0) or
 * off (0): HIP events around every launch of the timed kernels on the call's
 * stream, plus device counters of the useful work they perform (not inside
 * captured graphs), 4 = sweeps of the 64x64 inner eigensolve per Jacobi block
 * pair (default 1), 5 = threads per Jacobi-round workgroup, 256 (four waves,
 * one per SIMD) or 512 (default: eight waves, two per SIMD; the Gram and
 * rotation column work alternates between two groups of four waves),
 * 6 = column split: a round with fewer panel pairs than this (default 32;
 * 0 = never), or with fewer than 128 pairs of matrices of at least 1024 rows,
 * gives each pair S workgroups over disjoint column ranges, which
 * form partial Grams, then each sum them, solve the same rotation and rotate
 * their own columns (one large matrix, as in the sweep or TDVP),
 * 7 = split of matrices of at most 64 rows: 0 = one-sided Jacobi SVD
 * (default), 1 = the eigendecomposition split (Sec. "Basic concepts", Eq.
 * AAD_ULLUD): the Gram theta' theta'^dag is diagonalised to convergence in LDS
 * and the rows are rotated once by its eigenvectors; a singular value s_j then
 * carries a relative error of order 1e-15 (s_1/s_j)^2,
 * 8 = persistent Jacobi (default 1): a batch whose rounds need no column
 * split runs all its sweeps in one launch of resident workgroups that take
 * (sweep, round, matrix, pair) items from a device queue, each waiting only
 * for the previous round of its own matrix, with convergence decided on the
 * device; 0 = one launch per round and a convergence read-back per sweep.
 * A wait of the persistent launch is bounded (seconds); one that runs out
 * sets MPS_DEV_SCHED_TIMEOUT and the launch ends,
 * 9 = warm start of the TEBD splits (default 0; mps_tebd_step and the other
 * stepping calls of dense chains, SVD split): for a bond of
 * 64 < d chi_l <= 512 rows the Jacobi runs on Q^dag theta' instead of theta',
 * with Q the Householder QR factor of Lambda_l B_b (the bond's left Schmidt
 * vectors before the gate, Sec. "Time evolving block decimation"), whose
 * rows are then close to orthogonal; the singular values and V^dag are those
 * of theta' either way (Q is unitary), only the number of sweeps changes.
 * Its workspace is n_bonds * (d chi_max chi_max + 256 ceil(chi_max/16))
 * complex128 per layer; 0 = the Jacobi starts from theta' itself.  The
 * Jacobi then does about a quarter less work, but a layer's time follows its
 * slowest matrix, whose sweeps the start changes little once the bonds sit
 * at chi_max,
 * 10 = polls a wait of the persistent Jacobi makes before it gives up
 * (default 1e6, a few seconds; 1 .. 1e8).  A wait that runs out sets
 * MPS_DEV_SCHED_TIMEOUT and every workgroup of the launch leaves; a tiny
 * value forces that path, to test its reporting. */
mps_status mps_set_option(mps_handle h, int option, double value);
/* Accumulated timing of one kernel class since the last reset:
 * kernel 0 = theta build + gate, 1 = Jacobi round, 2 = selection,
 * 3 = right write-back, 4 = left write-back GEMM, 5 = Jacobi preparation,
 * 6 = propagators, 7 = Krylov-TEBD propagators (identity theta build,
 * reduced matrix, local Lanczos), 8 = warm start of the Jacobi (option 9:
 * QR of Lambda_l B_b and Q^dag theta').  total_ms = summed event durations, launches = count,
 * work = flops counted on the device: for kernels 0 and 4 the products'
 * useful flops, for kernel 1 the Jacobi's own Gram and rotation flops, for
 * kernel 5 the algorithmic work of the batched TEBD splits prepared
 * (88 m n min(m, n) per m x n complex SVD, a bidiagonalisation SVD's count);
 * else 0.
 * Synchronises `stream`.  reset != 0 clears all classes afterwards. */
mps_status mps_kernel_stats(mps_handle h, mps_stream stream, int32_t kernel, double* total_ms,
                            int64_t* launches, uint64_t* work, int32_t reset);

/*
 * Autotuner of the Jacobi launch configuration for one shape bucket: n_mats
 * matrices of m x n (the split of one batched layer).  Each candidate runs the
 * whole split (preparation, sweeps, selection) on the same seeded synthetic
 * matrices with graded rows, timed with HIP events after one untimed run:
 * 256 or 512 threads per round workgroup (option 5), column split below 0, 32
 * or 128 panel pairs (option 6) and, for m <= 64, the one-sided Jacobi or the
 * eigendecomposition split (option 7).  apply != 0 leaves the fastest in the
 * handle (else the handle's settings are restored).
 *   times_ms     : HOST [*n_candidates] on entry its capacity (12 suffice);
 *                  on return the count used and the times in candidate order
 *   best         : HOST int32, index of the fastest candidate
 * mps_autotune_candidate(m, index, ...) gives candidate `index`'s settings.
 * Uses the workspace; synchronises `stream`.
 */
mps_status mps_autotune_jacobi(mps_handle h, mps_stream stream, int32_t n_mats, int32_t m, int32_t n,
                               int32_t apply, double* times_ms, int32_t* n_candidates, int32_t* best);
mps_status mps_autotune_candidate(int32_t m, int32_t index, int32_t* threads, int32_t* split_below,
                                  int32_t* method);
/*
 * Autotuner for the MFMA tile shape of the GEMMs (the contractions of the
 * effective-Hamiltonian apply, App. "Details of the Krylov method", and of
 * the Hastings write-back, Sec. "Basic concepts").  Every candidate tile,
 * (32 MI) x (32 NJ) per 256-thread workgroup of 2 x 2 waves, with
 * (MI, NJ) in {(2,2), (4,2), (2,4), (1,2), (2,1), (1,1)}, runs the product
 * on synthetic operands in `dtype` (one untimed run, then the mean of five
 * timed with HIP events on `stream`); with `apply` the fastest becomes the
 * tile of its bucket.  A bucket is (kind, precision, shape class of M x N):
 * at most 64 tiles of 64 x 64, tall (M >= 2N), wide (N >= 2M), or square.
 * The choice is process-wide (all handles and devices of the process).
 *   kind  : 0 = the strided GEMM (C = A B, A [M][K], B [K][N], batch 1);
 *           1 = the batched write-back GEMM (C_i = A_i B_i^dag, B_i [N][K],
 *               `batch` problems)
 *   times_ms, n_candidates, best : as for mps_autotune_jacobi (6 candidates)
 * Every tile shape sums each output element over K in the same order, so
 * the results do not depend on the choice.  Uses the workspace; synchronises
 * `stream`.  Errors: MPS_ERR_INVALID for a bad kind or dtype, MPS_ERR_SHAPE
 * for sizes < 1 or batch != 1 with kind 0, MPS_ERR_CAPACITY for operands
 * above 2^26 elements, batch above 4096 or a short times_ms.
 */
mps_status mps_autotune_gemm(mps_handle h, mps_stream stream, int32_t kind, int32_t dtype, int32_t batch, int32_t M,
                             int32_t N, int32_t K, int32_t apply, double* times_ms, int32_t* n_candidates,
                             int32_t* best);
/* Tile of candidate `index`: tile_m x tile_n. */
mps_status mps_gemm_candidate(int32_t index, int32_t* tile_m, int32_t* tile_n);
/* The candidate the bucket of (kind, dtype, M, N) uses now. */
mps_status mps_gemm_tile_choice(int32_t kind, int32_t dtype, int32_t M, int32_t N, int32_t* index);
/* Set the candidate of the bucket of (kind, dtype, M, N) (e.g. from a cache of earlier tuning). */
mps_status mps_set_gemm_tile(int32_t kind, int32_t dtype, int32_t M, int32_t N, int32_t index);

/*
 * Bond propagators G_n = exp(-i tau_n h_n)   (the local two-site
 * propagator, step 2 of the plain TEBD update in App. "Details of the Krylov
 * method"; built by a Hermitian
 * Jacobi eigendecomposition h = V diag(e) V^dag in FP64, G = V e^{-i tau e} V^dag).
 *   hmat  : complex128 [n][dd][dd], Hermitian (dd = d*d <= 32)
 *   tau   : FP64 [n] (real time step of each propagator)
 *   G64   : complex64 [n][dd][dd] output (may be NULL)
 *   G128  : complex128 [n][dd][dd] output (may be NULL)
 */
mps_status mps_gates(mps_handle h, mps_stream stream, int32_t n, int32_t dd,
                     const void* hmat, const double* tau, void* G64, void* G128);

/*
 * Truncated SVD of one two-site tensor (Sec. "Basic concepts",
 * Splitting, SVD case; truncation and discarded weight per Eqs. overlap and
 * elocal; renormalisation of the kept values per App. "Auxiliary calculations").  The SVD runs in FP64 (one-sided block Jacobi).
 *   theta   : complex128 [m][n] input (not modified), m = chi_l*d_l, n = d_r*chi_r
 *   chi_max : cap on the kept count k
 *   eps     : local tolerance: k = min(chi_max, min{k>=1 : sum_{j>k} s_j^2
 *             <= eps * sum_j s_j^2}); values sorted descending.  A tolerance
 *             in [0, a), a the Jacobi absolute tolerance (option 2, default
 *             1e-15), acts as a: squared values below a |theta|^2 are not
 *             resolved and their directions not orthogonalised, so they count
 *             as zero; eps < 0 keeps min(chi_max, m) values.  The same holds
 *             for eps_local of every stepping entry point.
 *   U       : complex128 [m][chi_max] (first k columns written)
 *   S       : FP64 [chi_max] kept singular values, NOT renormalised
 *   Vh      : complex128 [chi_max][n] (first k rows written)
 *   k_dev   : int32 [1] kept count; disc_dev : FP64 [1] discarded weight
 *             sum_{j>k} s_j^2; norm2_dev : FP64 [1] sum_j s_j^2
 * Limits: m, n <= 4096.
 */
mps_status mps_truncate(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n,
                        int64_t chi_max, double eps, void* U, double* S, void* Vh,
                        int32_t* k_dev, double* disc_dev, double* norm2_dev);

/*
 * mps_truncate in either precision, with the kept values renormalised on
 * request (the renormalisation of App. "Auxiliary calculations").
 *   dtype       : MPS_C128 (theta, U, Vh complex128, as mps_truncate) or
 *                 MPS_C64 (theta, U, Vh complex64; the SVD still runs in FP64
 *                 on an up-converted copy; U and Vh are written whole, zero
 *                 past the kept count)
 *   renormalize : 1: S_j <- S_j / (sum_{i<k} S_i^2)^(1/2) (the Schmidt values
 *                 of the normalised truncated state); 0: S as mps_truncate
 * Other arguments, limits and errors as mps_truncate; MPS_ERR_INVALID for
 * another dtype or renormalize flag.
 */
mps_status mps_truncate_ex(mps_handle h, mps_stream stream, int32_t dtype, const void* theta, int64_t m, int64_t n,
                           int64_t chi_max, double eps, int32_t renormalize, void* U, double* S, void* Vh,
                           int32_t* k_dev, double* disc_dev, double* norm2_dev);

/*
 * mps_truncate without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * mps_truncate (same kernels and launch shapes), but every intermediate lives
 * in a fixed device array of 9 MiB inside the library (one copy per GPU, held
 * until the process ends), so the call makes no hipMalloc, hipFree or other
 * allocating call.
 * Limits: m, n <= 512 (MPS_ERR_CAPACITY beyond).
 * Every call on one GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (two streams, two threads, two handles) race; serialise
 * them.  Nothing needs to be cleared between calls.
 */
mps_status mps_truncate_noalloc(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n,
                                int64_t chi_max, double eps, void* U, double* S, void* Vh,
                                int32_t* k_dev, double* disc_dev, double* norm2_dev);

/*
 * U(1)-symmetric truncated SVD (App. "Convenient features", symmetry
 * conservation: with a diagonal symmetry generator the tensor cut at a bond is
 * block diagonal in the bond's charge and the decomposition runs on every
 * block).  Row r of theta carries the charge row_q[r], column c the charge
 * col_q[c]; theta[r][c] must vanish unless they agree (entries that do not
 * are ignored).  Every charge present on both sides is one block; the blocks
 * go through the batched FP64 Jacobi together, and the count rule of
 * mps_truncate is applied to the union of their singular values (ties
 * ordered by ascending charge, then by row).  Rows or columns whose charge
 * has no partner are structural zeros and not part of the spectrum.
 *   theta   : complex128 [m][n] device input (not modified)
 *   row_q, col_q : int32 [m], [n] charges, HOST memory
 *   U, S, Vh, k_dev, disc_dev, norm2_dev : as for mps_truncate; U[r][j] and
 *             Vh[j][c] vanish unless the row's (column's) charge is q_out[j]
 *   q_out   : int32 [chi_max] device output: the charge of kept vector j
 * Errors: MPS_ERR_SHAPE when no charge is shared by rows and columns.
 * Limits: m, n <= 4096.
 */
mps_status mps_truncate_u1(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n,
                           const int32_t* row_q, const int32_t* col_q, int64_t chi_max, double eps, void* U,
                           double* S, void* Vh, int32_t* q_out, int32_t* k_dev, double* disc_dev,
                           double* norm2_dev);

/*
 * A chain in Vidal/Hastings form (B_i = Gamma_i Lambda_{i+1}, right-canonical):
 * |psi> = lam_0 B_0 B_1 ... B_{L-1} (Eq. mps with the Schmidt values of
 * Eq. schmidt on the bonds).  Sites 0..L-1; virtual bond j sits left of site j.
 *   dtype : MPS_C64 (B complex64, contractions on FP32 MFMA with FP32
 *           accumulation) or MPS_C128 (B complex128, FP64 MFMA); the SVD,
 *           Schmidt values and observables are FP64 either way
 *   B     : L blocks of [chi_max][d][chi_max] of dtype; site i at
 *           B + i*chi_max*d*chi_max, element (a,s,c) at (a*d+s)*chi_max+c
 *   lam   : FP64, (L+1) blocks of [chi_max]; lam_0 = lam_L = {1}
 *   chi   : int32 [L+1] current bond dimensions; chi[0] = chi[L] = 1
 *   hbond : complex128 [L-1][d*d][d*d]; bond b couples sites b, b+1, with
 *           row index (s_out*d + t_out) and column index (s_in*d + t_in)
 *   disc  : FP64 [L-1]; the discarded weight of every update of bond b is
 *           added to disc[b]
 */
#define MPS_C64 0
#define MPS_C128 1

typedef struct {
  int32_t L, d, chi_max, dtype;
  void* B;
  double* lam;
  int32_t* chi;
  const void* hbond;
  double* disc;
} mps_chain_desc;

#define MPS_FLAG_GRAPH 0x1u     /* capture one step in a hipGraph and replay it n_steps times; the handle
                                   keeps the last captured step and replays it, with no new capture, on a
                                   later call with the same chains (pointers and shapes), order, dt,
                                   eps_local, log and Jacobi options */
#define MPS_FLAG_FIXED_SWEEPS 0x2u /* no host synchronisation inside the call */
#define MPS_FLAG_PLAIN 0x4u     /* one bond per launch sequence (no batching; comparison form) */
#define MPS_FLAG_CHECKPOINT 0x8u /* mps_tebd_step_ex: keep every step's chains for mps_tebd_step_vjp */
#define MPS_FLAG_OBSERVE 0x10u   /* mps_tebd_step_ex: <op at every site> of every chain after every step */

/*
 * n_steps time steps of Trotter evolution on every chain.
 *   order 2: even/odd Strang splitting (Sec. "Sornborger-Stewart
 *            decomposition": the Suzuki-Trotter even/odd alternative the paper
 *            names): odd bonds tau/2, even bonds tau, odd bonds tau/2;
 *   order 4: five Strang steps with weights p, p, 1-4p, p, p, p = 1/(4-4^(1/3)),
 *            error O(dt^4);
 *   order 0: the paper's own second-order sweep (Eq. sornborger2): every bond
 *            from left to right with dt/2, then from right to left with dt/2,
 *            one bond at a time (the bonds of different chains together).
 * Every update: theta~ = B_b B_{b+1} and theta~' = G theta~ on MFMA (FP32 for
 * complex64 chains, FP64 for complex128), theta' = lam_b theta~' in FP64,
 * FP64 SVD, truncation by the count rule with eps_local and chi_max,
 * lam_{b+1} = s/|s_k|, B_{b+1} = V^dag_k, B_b = theta~' V_k / |s_k|.  All bonds
 * of one layer of all chains are processed together.
 *   chains : HOST array of n_chains descriptors (device pointers inside)
 *   flags  : MPS_FLAG_* bits
 * Errors: MPS_ERR_INVALID for an order other than 0, 2, 4, an unknown flag or
 * a null pointer; MPS_ERR_SHAPE / MPS_ERR_CAPACITY for chain shapes.
 */
mps_status mps_tebd_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                         int32_t n_chains, int32_t order, double dt, int32_t n_steps,
                         double eps_local, uint32_t flags);

/*
 * mps_tebd_step with the record the adjoint and the error analysis need
 * (Sec. "Time evolution methods"; the discarded weight of Sec. "Basic
 * concepts in tensor network techniques", Eq. elocal).
 *   flags       : as mps_tebd_step, plus MPS_FLAG_CHECKPOINT: before every
 *                 step and after the last, every chain (B, lam, chi) is
 *                 copied into ckpt_arena (complex64 B widened exactly to
 *                 complex128), not with MPS_FLAG_GRAPH.  mps_tebd_step_vjp
 *                 reads the arena.
 *   ckpt_arena  : device, at least mps_tebd_ckpt_bytes(chains, n_chains,
 *                 n_steps) bytes, owned by the caller (NULL without the flag)
 *   disc_log_dev: device FP64 [n_steps][n_layers][n_chains][L_max-1] or NULL,
 *                 n_layers = 3 (order 2), 15 (order 4), 2 (L_max-1) (order
 *                 0); entry (step, layer, c, b) receives the discarded weight
 *                 of the update of bond b of chain c in that layer.  Entries
 *                 of bonds a layer does not update are not written (clear the
 *                 log first).  Works with MPS_FLAG_GRAPH (the replayed step
 *                 reads its index from a device counter).
 *   obs_op      : with MPS_FLAG_OBSERVE, a single-site operator, device
 *                 complex128 [d][d] (Sec. "Observables"), else NULL
 *   obs_log_dev : with MPS_FLAG_OBSERVE, device FP64 [n_steps][n_chains][L_max]:
 *                 entry (step, c, i) receives <obs_op at site i> of chain c
 *                 after that step (sum_a lam_i[a]^2 <B_i[a]| op |B_i[a]>);
 *                 sites past a chain's L are not written.  Works with
 *                 MPS_FLAG_GRAPH (the same device step counter).
 * Errors: as mps_tebd_step; MPS_ERR_INVALID for MPS_FLAG_CHECKPOINT without
 * an arena or with MPS_FLAG_GRAPH; MPS_ERR_CAPACITY for a short arena;
 * MPS_ERR_UNSUPPORTED for MPS_FLAG_CHECKPOINT on complex64 chains.
 */
mps_status mps_tebd_step_ex(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                            int32_t order, double dt, int32_t n_steps, double eps_local, uint32_t flags,
                            void* ckpt_arena, size_t ckpt_bytes, double* disc_log_dev, const void* obs_op,
                            double* obs_log_dev);
/* Bytes of the checkpoint arena of mps_tebd_step_ex for these chains and
 * n_steps, enough for the adjoint of a TEBD2 or a TEBD4 run (the reverse
 * pass keeps one snapshot per layer of a step; host only; 0 for bad
 * arguments). */
size_t mps_tebd_ckpt_bytes(const mps_chain_desc* chains, int32_t n_chains, int32_t n_steps);

/*
 * Charges of a symmetric chain (App. "Convenient features", symmetry
 * conservation: a diagonal generator such as the particle number or 2 S^z).
 *   qbond   : int32 DEVICE [L+1][chi_max]: qbond[b][a] is the total charge of
 *             sites 0..b-1 in Schmidt state a of bond b (a < chi[b]); bond
 *             b+1 is rewritten by every update of the bond between sites b,
 *             b+1
 *   qsite   : charge of local basis state s (s < d), host values
 *   modulus : 0 for U(1) (charges compared as integers); n >= 2 for Z_n
 *             (charges compared modulo n, written in 0..n-1), e.g. n = 2 for
 *             the parity of a particle number
 * For a product of basis states q_0 = 0 and q_{b+1} = q_b + qsite[s_b].
 * Several U(1) generators pack into one charge as q_1 K + q_2 with K larger
 * than twice the range of q_2, as long as the packed values fit int32.
 */
typedef struct {
  int32_t* qbond;
  int32_t qsite[5];
  int32_t modulus;
  int32_t reserved[2];
} mps_u1_chain;

/*
 * mps_tebd_step on charge-conserving chains (App. "Convenient features",
 * symmetry conservation).  Every update cuts theta' at the new bond into its
 * charge blocks: row (a, s1) carries qbond[b][a] + qsite[s1], column
 * (s2, g) carries qbond[b+2][g] - qsite[s2]; entries between different
 * charges are not read.  The blocks of all bonds of a layer go through the
 * batched FP64 Jacobi together; the count rule (eps_local, chi_max) is applied
 * per bond to the union of its blocks' values, ties ordered by ascending
 * charge; B_{b+1} = V^dag_k (zero off its block's columns), lam_{b+1} and
 * qbond[b+1] follow, B_b = theta~' V_k / |s_k| as in mps_tebd_step.  The bond
 * Hamiltonians must commute with the charge.  The charge blocks are built on
 * the device from qbond (no host synchronisation inside a layer), so
 * MPS_FLAG_GRAPH captures and replays the step as for dense chains; an update
 * whose rows and columns share no charge (or whose bond dimension is out of
 * range) is skipped, leaving the bond as it was, and sets MPS_DEV_CHARGE.
 *   charges : HOST array of n_chains descriptors, one per chain
 * Errors: as mps_tebd_step; MPS_ERR_INVALID for a null qbond or a modulus
 * < 0 or == 1; MPS_ERR_CAPACITY when d*chi_max > 2048 or when (bonds of one
 * layer) * d * chi_max > 65536.
 */
mps_status mps_tebd_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                            const mps_u1_chain* charges, int32_t n_chains, int32_t order, double dt,
                            int32_t n_steps, double eps_local, uint32_t flags);

/*
 * n_steps Krylov-TEBD steps on every chain (Sec. "Sornborger-Stewart
 * decomposition" with the local Krylov propagation of App. "Details of the
 * Krylov method"): the sweep of order 0 above, where each update propagates
 * the two-site tensor theta' = lam_b B_b B_{b+1} (the orthogonality centre is
 * inside the two sites) with the Lanczos approximation of exp(-i dt/2 h_b),
 * h_b acting on the two physical indices, instead of the exact propagator:
 * v_1 = theta'/|theta'|, r = h_b v_j, alpha_j = Re<v_j|r>,
 * r -= alpha_j v_j + beta_{j-1} v_{j-1}, two passes of full Gram-Schmidt,
 * beta_j = |r|, u = exp(-i tau T_j) e_1, err_j = |theta'| beta_j |u_j|; stop
 * when err_j <= tol or beta_j <= 1e-14 |theta'|, else after n_max vectors
 * (then MPS_DEV_NOCONV_LANCZOS is set in the device status word).  The
 * iteration runs in FP64 on the d^2 x d^2 reduced matrix of theta' (every
 * Krylov vector is a polynomial in h_b applied to theta'); the resulting
 * polynomial propagator then takes the path of a gate (theta~ build on MFMA,
 * FP64 SVD with eps_local / chi_max, Hastings write-back).
 *   chains     : HOST array of n_chains descriptors as for mps_tebd_step
 *   n_max      : 1..32 Krylov vectors per update;  tol >= 0
 *   flags      : MPS_FLAG_GRAPH, MPS_FLAG_FIXED_SWEEPS, MPS_FLAG_PLAIN as above
 *   n_used_dev : optional device int32 [n_chains][2 (L_max - 1)]; entry
 *                [c][j] receives the vectors used by sweep position j of the
 *                last step (j < L_max - 1: bond j left to right; j >= L_max - 1:
 *                bond L_c - 2 - (j - L_max + 1) right to left); positions a
 *                shorter chain does not have are left untouched
 * Between two calls every B is right-canonical and lam_0 B_0 B_1 ... is the
 * state.  With an approximate propagator (not converged to an invariant
 * subspace) lam on a bond updated earlier in the right-to-left half differs
 * from the final Schmidt spectrum by the size of the Krylov error; the next
 * step does not read those values.
 * Errors: as mps_tebd_step; MPS_ERR_INVALID for n_max outside 1..32 or tol < 0.
 */
mps_status mps_ktebd_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                          int32_t n_chains, double dt, int32_t n_steps, double eps_local,
                          int32_t n_max, double tol, uint32_t flags, int32_t* n_used_dev);

/*
 * mps_ktebd_step on charge-carrying chains: the Krylov sweep with every cut
 * on the charge blocks of its bond, as in mps_tebd_step_u1 (App. "Convenient
 * features", symmetry conservation; App. "Details of the Krylov method").
 * The bond Hamiltonians must commute with the charge, so the Lanczos
 * propagator does.  Arguments, errors and limits as mps_ktebd_step and
 * mps_tebd_step_u1.
 */
mps_status mps_ktebd_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                             const mps_u1_chain* charges, int32_t n_chains, double dt, int32_t n_steps,
                             double eps_local, int32_t n_max, double tol, uint32_t flags, int32_t* n_used_dev);

/*
 * n_steps steps of a time-dependent Hamiltonian H(t) = sum_k f_k(t) H_k
 * (Sec. "Time evolution methods": time ordering by commutator-free Magnus
 * expansions).  Step n covers [t_n, t_n + dt] with t_n = t0 + n dt and is a
 * product of exponentials of linear combinations of H at the nodes
 * t_n + c_j dt:
 *   scheme 2 (the paper's default): one node c = 1/2, U = exp(-i dt H(t_n + dt/2));
 *   scheme 4: nodes c_{1,2} = 1/2 -+ sqrt(3)/6, weights a_1 = (3 - 2 sqrt 3)/12,
 *             a_2 = (3 + 2 sqrt 3)/12; first exp(-i dt (a_2 H_1 + a_1 H_2)), then
 *             exp(-i dt (a_1 H_1 + a_2 H_2)), H_j = H(t_n + c_j dt).
 * Every exponential exp(-i dt A), A = sum_k w_k H_k, is one Trotter step of
 * `order` as in mps_tebd_step (2, 4, or 0 for the sweep) with bond
 * Hamiltonians h_b = sum_k w_k h_b^(k), formed on the device.
 *   chains  : HOST array of descriptors as for mps_tebd_step, except that
 *             hbond holds every term: complex128 [n_terms][L-1][d*d][d*d]
 *   n_terms : 1..16;  scheme : 2 or 4 (mps_cfme_nodes gives the nodes)
 *   f_nodes : HOST FP64 [n_steps][n_nodes][n_terms], f_k(t_n + c_j dt)
 *   hwork   : DEVICE complex128 [sum_c (L_c - 1)][d*d][d*d], caller-owned
 *             scratch for the combined bond Hamiltonians
 * Errors: MPS_ERR_INVALID for a bad scheme or term count, null or
 * non-finite f_nodes, null hwork; otherwise as mps_tebd_step.
 */
mps_status mps_tebd_td_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                            int32_t n_chains, int32_t order, double dt, int32_t n_steps,
                            double eps_local, uint32_t flags, int32_t n_terms, int32_t scheme,
                            const double* f_nodes, void* hwork);

/*
 * mps_tebd_td_step on charge-carrying chains: every exponential's Trotter
 * step is a mps_tebd_step_u1 step (App. "Convenient features", symmetry
 * conservation; Sec. "Time evolution methods", time ordering).  Every term
 * set must commute with the charge.  Arguments, errors and limits as
 * mps_tebd_td_step and mps_tebd_step_u1.
 */
mps_status mps_tebd_td_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                               const mps_u1_chain* charges, int32_t n_chains, int32_t order, double dt,
                               int32_t n_steps, double eps_local, uint32_t flags, int32_t n_terms, int32_t scheme,
                               const double* f_nodes, void* hwork);
/* The nodes c_j of a scheme (host only): nodes[0..n_nodes-1]; MPS_ERR_INVALID
 * for an unknown scheme. */
mps_status mps_cfme_nodes(int32_t scheme, double* nodes, int32_t* n_nodes);

/*
 * Observables of a Hastings-form chain (Sec. "Observables",
 * reduced density matrices of Eq. reducedrho):
 *   site_out[i] = Re sum lam_i[a]^2 conj(B_i[a,s',c]) op1[s',s] B_i[a,s,c]
 *   bond_out[b] = Re <theta_b| op2_b |theta_b>, theta_b = lam_b B_b B_{b+1}
 *   entropy_out[b] = -sum_a lam_{b+1}[a]^2 ln lam_{b+1}[a]^2
 *   op1 : complex128 [d][d] (or NULL); op2 : complex128 [L-1][d*d][d*d] when
 *         op2_per_bond != 0, else [d*d][d*d] (or NULL)
 *   outputs FP64 device arrays [L], [L-1], [L-1] (any may be NULL)
 */
mps_status mps_observe(mps_handle h, mps_stream stream, const mps_chain_desc* chain,
                       const void* op1, double* site_out, const void* op2, int32_t op2_per_bond,
                       double* bond_out, double* entropy_out);

/*
 * Structured effective Hamiltonian y = H_eff x (Sec. "Fundamentals of the
 * library", Fig. LanczosMPS: the environments and the MPO matrices of the
 * active sites are contracted into x one at a time, O(chi^3), never forming the
 * chi^2 d^2 square matrix).  All operands in `dtype` (MPS_C64 on FP32 MFMA,
 * MPS_C128 on FP64 MFMA), compact row-major:
 *   Lenv : [chi_l][w_l][chi_l]  (Lenv[a_out][beta][a_in])
 *   W1   : [w_l][w_m][d1][d1]   (W[beta_l][beta_r][s_out][s_in], the MPO's |i'><i|)
 *   W2   : [w_m][w_r][d2][d2]   (NULL for the one-site H_eff; then w_m is W1's
 *          right dimension, Renv is [chi_r][w_m][chi_r] and d2, w_r are ignored)
 *   Renv : [chi_r][w_r][chi_r]  (Renv[c_out][beta][c_in])
 *   x, y : [chi_l][d1][d2][chi_r] (or [chi_l][d1][chi_r])
 * Limits: w*d <= 32 for every MPO leg.  Scratch is taken from the workspace.
 */
mps_status mps_heff_apply(mps_handle h, mps_stream stream, int32_t dtype, const void* Lenv, const void* W1,
                          const void* W2, const void* Renv, const void* x, void* y, int64_t chi_l, int32_t d1,
                          int32_t d2, int64_t chi_r, int32_t w_l, int32_t w_m, int32_t w_r);

/*
 * Lanczos exponential x <- exp(-i tau H_eff) x, tau = tau_re + i tau_im
 * (Sec. "Krylov time evolution", Eq. krylov:approx; App. "Details of the Krylov
 * method": with the orthogonality centre in the active sites every Krylov
 * vector and their weighted sum stay local).  Krylov vectors, the three-pass
 * Gram-Schmidt and the tridiagonal exponential are FP64 on the GPU; H_eff is
 * applied in `dtype`.  Stops when the a-posteriori estimate
 * |x| beta_j |(Q e^{-i tau Theta} Q^T e_1)_j| <= tol or the Krylov space is
 * invariant; else after n_max vectors (1 <= n_max <= 30) with
 * MPS_DEV_NOCONV_LANCZOS set.  Operands as for mps_heff_apply; x in `dtype`.
 * n_used (int32 [1]) and err_est (FP64 [1]) are device outputs (may be NULL).
 * Synchronises `stream` (the iteration is steered from the host).
 */
mps_status mps_krylov_expm(mps_handle h, mps_stream stream, int32_t dtype, const void* Lenv, const void* W1,
                           const void* W2, const void* Renv, void* x, int64_t chi_l, int32_t d1, int32_t d2,
                           int64_t chi_r, int32_t w_l, int32_t w_m, int32_t w_r, double tau_re, double tau_im,
                           int32_t n_max, double tol, int32_t* n_used, double* err_est);

/*
 * Environment update (Sec. "Fundamentals of the library": the fixed sites
 * are contracted with their MPO matrices into one left and one right tensor).
 *   side 0 (left):  out[a'][b'][c'] = sum conj(A[a][s'][a']) in[a][b][c] W[b][b'][s'][s] A[c][s][c']
 *                   in [chi_in][w_in][chi_in], A [chi_in][d][chi_out], W [w_in][w_out][d][d]
 *   side 1 (right): out[a'][b][c'] = sum conj(A[a'][t'][a]) W[b][b'][t'][t] in[a][b'][c] A[c'][t][c]
 *                   in [chi_in][w_in][chi_in], A [chi_out][d][chi_in], W [w_out][w_in][d][d]
 *   out [chi_out][w_out][chi_out].  dtype as above.
 */
mps_status mps_env_update(mps_handle h, mps_stream stream, int32_t dtype, int32_t side, const void* env_in,
                          const void* W, const void* A, void* env_out, int64_t chi_in, int32_t d, int64_t chi_out,
                          int32_t w_in, int32_t w_out);

/*
 * A chain in mixed-canonical form for two-site TDVP: orthogonality centre on
 * site 0, sites 1..L-1 right-canonical (Eq. oc).
 *   M   : L blocks of chi_max*d*chi_max elements of dtype; site i holds a
 *         compact row-major [chi_i][d][chi_{i+1}] tensor at the block start
 *   chi : int32 [L+1] device array, chi[0] = chi[L] = 1
 *   W   : L blocks of [w][w][d][d] (MPO matrices; the left boundary selects
 *         index w-1, the right boundary index 0, as in Eq. MPOdef)
 */
typedef struct {
  int32_t L, d, chi_max, dtype;
  int32_t w, reserved;
  void* M;
  int32_t* chi;
  const void* W;
} mps_oc_chain;

/*
 * The two-site TDVP sweep (Sec. "Time-dependent variational
 * principle"): n_steps symmetric steps; each half-sweep uses tau = dt/2, a
 * forward two-site Lanczos exponential per bond, the FP64 truncated SVD
 * (count rule with eps_local, chi_max), the environment update, and a backward
 * one-site exponential at every interior bond.  The centre returns to site 0.
 *   disc_dev : FP64 [L-1], discarded weights added per bond (may be NULL)
 *   krylov_max_dev : int32 [1], largest Krylov dimension used (may be NULL)
 * Synchronises `stream`.  Limits: w*d <= 32, d*chi_max <= 4096.
 */
mps_status mps_tdvp2_step(mps_handle h, mps_stream stream, const mps_oc_chain* chain, double dt, int32_t n_steps,
                          double eps_local, int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev);

/*
 * mps_tdvp2_step on a charge-carrying chain: every two-site split runs on the
 * charge blocks of its bond (App. "Convenient features", symmetry
 * conservation), row (a, s1) of theta carrying qbond[b][a] + qsite[s1] and
 * column (s2, g) qbond[b+2][g] - qsite[s2]; A_b = U_k (left to right) or
 * B_{b+1} = V^dag_k (right to left) vanish off each kept vector's block, and
 * qbond[b+1] takes the kept charges.  The MPO must commute with the charge.
 *   charges : one HOST descriptor (mps_u1_chain, qbond on the device)
 * Errors: as mps_tdvp2_step; MPS_ERR_INVALID for null charges or a modulus
 * < 0 or == 1; MPS_ERR_SHAPE for d > 5 or when no charge is shared across a
 * bond.
 */
mps_status mps_tdvp2_step_u1(mps_handle h, mps_stream stream, const mps_oc_chain* chain,
                             const mps_u1_chain* charges, double dt, int32_t n_steps, double eps_local,
                             int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev);

/*
 * Reverse-mode gradient of a truncated TEBD2 run (second-order Trotter-Suzuki
 * splitting of Sec. "Time evolution methods", with the truncated SVD of Sec.
 * "Basic concepts in tensor network techniques") with respect to per-bond
 * couplings J_b, where the chain's bond Hamiltonians are h_b = J_b * h0_b.
 * The paper does not differentiate its runs; this entry point is the exact
 * adjoint of the update that mps_tebd_step performs.
 *
 * Loss = <op1 on `site`> + sum_b <op2 on bond b> of the state after n_steps
 * (expectation values of Sec. "Observables", in the Hastings form).
 * The run advances `chain` from its current state exactly as mps_tebd_step
 * with order 2 and eager scheduling would, keeping one snapshot of the chain
 * per step in `arena`; the reverse pass re-runs each step layer by layer and
 * applies the adjoint of every two-site update.  The singular-value backward
 * keeps the coupling between kept and discarded singular triplets and uses a
 * Lorentzian broadening `eta` of 1/(s_j^2 - s_i^2) and of 1/s (eta >= 0; 1e-12
 * is the usual choice).  Complex64 chains: the forward and the reverse
 * pass's re-runs of each step in the chain's precision (FP32 MFMA
 * contractions, FP64 SVD), every snapshot widened exactly to complex128 and
 * the adjoint itself in FP64; the gradient then carries the FP32 rounding of
 * the forward (about 1e-5 relative against an FP64 run on the test chains).
 *   h0      : device complex128 [L-1][d^2][d^2], the unit bond terms
 *   op1     : device complex128 [d][d];  op2 : device complex128 [d^2][d^2]
 *   arena   : device memory of at least mps_tebd_grad_arena_bytes(L, d,
 *             chi_max, n_steps) bytes, owned by the caller (contents scratch)
 *   loss_dev: FP64 [1];  dJ_dev : FP64 [L-1], overwritten
 * On return the chain holds the final state; synchronises `stream`.
 * Errors: MPS_ERR_UNSUPPORTED for complex64 chains, MPS_ERR_CAPACITY for a
 * short arena or d*chi_max > 2560, MPS_ERR_NONFINITE if a kept weight vanishes.
 * The device status word carries MPS_DEV_NOCONV_SVD if a reverse-pass SVD did
 * not converge.
 */
size_t mps_tebd_grad_arena_bytes(int32_t L, int32_t d, int32_t chi_max, int32_t n_steps);
/*
 * The vector-Jacobian product of the same run: for the final observables
 * obs = (<op1 at site i>, i < L; <op2 on bond b>, b < L-1) and host weights
 * w_site [L], w_bond [L-1] (the cotangent of obs), dJ_dev receives
 * sum_i w_site[i] d<op1>_i/dJ + sum_b w_bond[b] d<op2>_b/dJ.  obs_dev (device
 * FP64 [2L-1], may be NULL) receives obs.  Other arguments, the chain's final
 * state and the errors as for mps_tebd_grad; non-finite weights are refused.
 */
mps_status mps_tebd_vjp(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* h0, double dt,
                        int32_t n_steps, double eps_local, double eta, const void* op1, const double* w_site,
                        const void* op2, const double* w_bond, void* arena, size_t arena_bytes, double* obs_dev,
                        double* dJ_dev);
mps_status mps_tebd_grad(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* h0, double dt,
                         int32_t n_steps, double eps_local, double eta, const void* op1, int32_t site,
                         const void* op2, void* arena, size_t arena_bytes, double* loss_dev, double* dJ_dev);
/*
 * The vector-Jacobian product of a batched TEBD2 or TEBD4 run recorded by
 * mps_tebd_step_ex with MPS_FLAG_CHECKPOINT (order 2 or 4), for any cotangent of
 * the final states: with dL = sum_c Re <dB_final[c], dB_c> + <dLam_final[c],
 * dlam_c> (the cotangent of a complex entry x is dL/dRe x + i dL/dIm x),
 * dJ_dev[c][b] receives dL/dJ_b of chain c, where that chain's bond terms
 * are h_b = J_b h0[c][b].  The reverse pass is the one of mps_tebd_grad
 * (truncated-SVD backward with the kept/discarded coupling and a Lorentzian
 * broadening eta), run chain by chain on the chain's arena block; for
 * TEBD4 it walks the 15 layers of every step (classes of time steps p dt/2,
 * p dt, (1-4p) dt/2, (1-4p) dt) in reverse.
 *   chains      : the chains of the forward call, holding their final states
 *                 (left so on return)
 *   h0          : HOST array of n_chains device pointers, complex128
 *                 [L-1][d^2][d^2] unit bond terms
 *   ckpt_arena  : the forward's arena (its scratch parts are overwritten)
 *   dB_final    : HOST array of device pointers, in the chain's dtype and
 *                 the layout of its B (complex64 cotangents are widened)
 *   dLam_final  : HOST array of device pointers, FP64 in the layout of lam
 *   dJ_dev      : device FP64 [n_chains][L_max-1], overwritten (entries past
 *                 a chain's L-1 are 0)
 * Synchronises `stream`.  Errors: MPS_ERR_INVALID for an arena not written by
 * an order-2 or order-4 mps_tebd_step_ex for the same chains, null pointers
 * or eta < 0;
 * MPS_ERR_CAPACITY for a short arena or d*chi_max > 2560.
 */
mps_status mps_tebd_step_vjp(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                             const void* const* h0, void* ckpt_arena, size_t ckpt_bytes,
                             const void* const* dB_final, const double* const* dLam_final, double* dJ_dev,
                             double eta);

/*
 * The vector-Jacobian products of the two pieces of one TEBD update (the
 * reverse of its steps: contraction and local propagator of the plain
 * two-site update in App. "Details of the Krylov method", truncated SVD split
 * of Sec. "Basic concepts"; the paper gives the forward steps only).
 * Cotangents follow dL = Re sum conj(Xbar) dX (the cotangent of a complex
 * entry x is dL/dRe x + i dL/dIm x); every array is complex128 row-major on
 * the device, every output is overwritten, the call is asynchronous on
 * `stream`.
 *
 * mps_theta_gate_vjp: for theta'[(a,s)][(t,c)] = lam_l[a] sum_{u,v} G[(s,t)][(u,v)]
 * sum_b Bl[a][u][b] Br[b][v][c] (theta' is [chl*d][d*chr]) and its cotangent
 * theta_bar of the same shape, writes
 *   dBl [chl][d][chm], dBr [chm][d][chr], dlam_l FP64 [chl], dG [d*d][d*d].
 * Bl [chl][d][chm], Br [chm][d][chr], lam_l FP64 [chl], G [d*d][d*d].
 * Errors: MPS_ERR_INVALID for a null pointer, MPS_ERR_SHAPE for a dimension
 * < 1 or d > 5, MPS_ERR_CAPACITY for d*chl, d*chr or chm above 4096.
 */
mps_status mps_theta_gate_vjp(mps_handle h, mps_stream stream, const void* Bl, const void* Br, const double* lam_l,
                              const void* G, const void* theta_bar, int32_t chl, int32_t d, int32_t chm, int32_t chr,
                              void* dBl, void* dBr, double* dlam_l, void* dG);
/*
 * mps_truncate_vjp: theta_bar [m][n] = dL/dtheta for the kept factors of
 * mps_truncate(theta) = (U, S, Vh) with k kept values, given
 *   S [k], Vh [k][n]      : the forward's kept values and rows of V^dag
 *   U_bar [m][ld_ubar]    : cotangent of U (first k columns), may be NULL
 *   S_bar [k], Vh_bar [k][n] : cotangents of S and Vh, each may be NULL
 *   eta                   : Lorentzian broadening (>= 0) of the inverse gaps
 *                           1/(s_j^2 - s_i^2) -> D/(D^2 + eta) and of 1/s_j
 *                           -> s_j/(s_j^2 + eta); eta = 0 is the exact
 *                           derivative where the gaps are nonzero.
 * The full reduced SVD backward is used, with the discarded triplets'
 * cotangents zero but their coupling to the kept ones retained: the
 * discarded directions are resolved by an FP64 Jacobi SVD of
 * theta (1 - V_k V_k^dag) with an absolute tolerance of 1e-30 of its weight
 * (directions of weight below 1e-26 |theta|^2 are dropped).  U_bar enters through
 * U = theta V_k S^-1.  L must not depend on the phases of the singular
 * vectors (as no quantity of the Hastings form does).
 * Errors: MPS_ERR_INVALID for a null theta, S, Vh or theta_bar or eta < 0;
 * MPS_ERR_SHAPE for k outside [1, min(m, n)] or ld_ubar < k;
 * MPS_ERR_CAPACITY for m or n above 2560.
 */
mps_status mps_truncate_vjp(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n, int32_t k,
                            const double* S, const void* Vh, const void* U_bar, int64_t ld_ubar, const double* S_bar,
                            const void* Vh_bar, double eta, void* theta_bar);

#ifdef __cplusplus
}
#endif
#endif /* MPS_H_ */
