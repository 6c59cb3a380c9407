// Internal declarations shared by the libmps translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mps.h"

#define MPS_NKERNELS 9
#define MPS_NSTATS 8
// kernel classes timed by the optional profiler (ids of mps_kernel_stats)
#define MPS_K_THETA 0
#define MPS_K_JAC_ROUND 1
#define MPS_K_SELECT 2
#define MPS_K_WB_RIGHT 3
#define MPS_K_GEMM 4
#define MPS_K_PREP 5
#define MPS_K_GATES 6
#define MPS_K_KRYLOV 7
#define MPS_K_WARM 8

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct mps_context {
  int device = 0;
  char* ws = nullptr;          // device workspace (the handle's, or the caller's)
  size_t ws_bytes = 0;
  bool ws_external = false;    // caller-owned workspace: never grown, never freed here
  size_t ws_call = 0;          // bytes the running call planned (the rest may hold split partials)
  size_t ws_needed = 0;        // largest plan seen on this handle
  bool plan_only = false;      // mps_workspace_size: entry points stop after planning
  uint32_t* status_dev = nullptr;  // device status word (MPS_DEV_* bits)
  std::string err;
  double jac_tol = 1e-13;      // relative orthogonality tolerance of the Jacobi SVD
  double jac_abs = 1e-15;      // absolute tolerance, relative to |theta|_F^2
  int jac_max_sweeps = 30;
  int jac_inner_sweeps = 1;    // sweeps of the 64x64 inner eigensolve per block pair
  int jac_threads = 512;       // threads per Jacobi-round workgroup (256 or 512)
  int jac_split_below = 32;    // split a round's pairs over columns below this many pairs (0 = never)
  int split_method = 0;        // single-panel matrices: 0 = one-sided Jacobi SVD, 1 = eigensolve of the Gram
  double2* split_part = nullptr;  // partial Grams of split rounds (grown on demand)
  size_t split_bytes = 0;
  char* scratch = nullptr;        // this device's address of the no-allocation entry's scratch array
  int jac_persistent = 1;         // batches without a column split: all sweeps in one persistent launch
  int jac_spin_limit = 1000000;   // polls of a persistent Jacobi wait before it gives up (a few seconds)
  int warm_start = 0;             // TEBD splits: Jacobi on Q^dag theta', Q from the QR of Lambda_l B_b
  int n_cu = 256;                 // compute units of the device (persistent grid size)
  char* sched = nullptr;          // counters of the persistent Jacobi (kSchedBytes)
  // pinned host scratch for small readbacks
  int32_t* host_pinned = nullptr;
  // optional per-kernel timing with HIP events on the launch stream
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;  // (kernel id, first event index)
  double k_ms[MPS_NKERNELS] = {0};
  long long k_launches[MPS_NKERNELS] = {0};
  unsigned long long* stats_dev = nullptr;  // device work counters [MPS_NSTATS]
  // extra streams (default priority) for independent per-bond work, and events to fork/join them
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_ev;
  // the last captured TEBD step (MPS_FLAG_GRAPH) and the launch parameters it
  // was captured with: a call with the same parameters replays it
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> graph_key;
};

// Make `n` auxiliary streams available on the handle (created once, kept).
mps_status mps_aux_streams(mps_handle h, int n);

// Jacobi helpers shared by the drivers (api.hip)
struct JacMat;
int jac_nb(int m);
// allow_split: rounds with few panel pairs may split each pair over columns
// split_buf (optional, split_buf_bytes long): the partial Grams of column-split
// rounds go there instead of the handle's buffer (grown on demand); the split
// then uses as many slices as it holds
mps_status run_jacobi(mps_handle h, hipStream_t s, JacMat* mats, int n, int nb_cap, int m_cap, int32_t* unconv,
                      bool fixed, bool allow_split = true, double2* split_buf = nullptr, size_t split_buf_bytes = 0);

// Local Krylov propagation of the bond terms (Krylov TEBD)
struct KryOpts {
  int n_max;            // Krylov vectors per update, 1..32
  double tol;           // stop when the a-posteriori estimate is <= tol
  int32_t* n_used_dev;  // optional [n_chains][2 (L_max - 1)] log of the vectors used
};

// The tolerance the count rule applies: squared singular values below the
// Jacobi's absolute floor (jac_abs |theta|^2) are not resolved, their
// directions are not orthogonalised, so a tail below the floor counts as zero
// (eps < 0, keep everything up to chi_max, is passed through)
// Smallest Jacobi absolute tolerance (relative to |X|_F^2).  Under a purely
// relative criterion, rows beyond the rank of a matrix with more rows than
// columns have no room to become orthogonal: they are rotated toward zero
// sweep after sweep and end as NaN rows.  The floor lets them count as
// converged once |G_pq| <= 1e-30 |X|_F^2, far below any resolved value.
constexpr double kJacAbsFloor = 1e-30;
inline double count_rule_eps(mps_handle h, double eps) { return eps >= 0.0 && eps < h->jac_abs ? h->jac_abs : eps; }

// TEBD driver with a layer window (api.hip); kry != null propagates every
// bond of the sweep (order 0) with the local Lanczos exponential of h_b
// u1 != null: charge-carrying chains, every update truncated on its charge blocks
// ckpt (MPS_FLAG_CHECKPOINT): the checkpoint arena of mps_tebd_step_ex;
// disc_log: its per-update discarded-weight log; obs_op, obs_log
// (MPS_FLAG_OBSERVE): <op at every site> of every chain after every step (all optional)
mps_status tebd_impl(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains, int32_t order,
                     double dt, int32_t n_steps, double eps_local, uint32_t flags, int lo, int hi,
                     const KryOpts* kry = nullptr, const mps_u1_chain* u1 = nullptr, void* ckpt = nullptr,
                     size_t ckpt_bytes = 0, double* disc_log = nullptr, const void* obs_op = nullptr,
                     double* obs_log = nullptr);

// Checkpoint arena of mps_tebd_step_ex: a header, then for every chain the
// block of the adjoint (mps_tebd_grad_arena_bytes of that chain), 256-byte
// aligned, whose step checkpoints grad_ckpt_save writes.
struct CkptHeader {
  uint32_t magic;          // kCkptMagic
  int32_t n_chains, n_steps, order;
  double dt, eps_local;
  int64_t shape_sum;       // sum over chains of (L, d, chi_max) mixed: a check that the chains are the same
};
constexpr uint32_t kCkptMagic = 0x4d50534bu;
constexpr size_t kCkptHeader = 256;
int64_t ckpt_shape_sum(const mps_chain_desc* chains, int n_chains);
size_t ckpt_block_offset(const mps_chain_desc* chains, int c, int n_steps);
mps_status grad_ckpt_save(mps_handle h, hipStream_t s, const mps_chain_desc& ch, char* block, int n_steps, int st);

// Charge-carrying chains (u1.hip): the truncation of one layer of n bond
// items (theta' in their X slots) on the charge blocks of every bond, in place
// of preparation, Jacobi, selection and right write-back.  ui_dev[i] holds
// the charges of item i (device); the blocks are built on the device and no
// step synchronises with the host, so a layer can be captured in a graph.
// m_cap <= 2048 and n_cap * m_cap <= kSchedCap; region holds
// u1_layer_bytes(n_cap, m_cap, chi_cap) bytes.
struct BondItem;
struct SelOut;
struct U1Item {
  int32_t* qb;         // the chain's bond charges [L+1][chi_max]
  int32_t modulus;     // 0: U(1); n >= 2: Z_n
  int32_t qsite[5];    // charges of the local states (d <= 5)
};
size_t u1_layer_bytes(int n_cap, int m_cap, int chi_cap);
mps_status u1_layer(mps_handle h, hipStream_t s, const BondItem* it_dev, const U1Item* ui_dev, int n, int n_cap,
                    int m_cap, int chi_cap, double eps, bool c128, char* region, SelOut* sel, int32_t* unconv);
// Jacobi of the slots mats[0, n_slots): empty slots are converged matrices,
// the others are found on the device (list: n_slots ints, cnt: 2 ints), so no
// launch depends on their number; when all have one panel they run in loop
// mode, else all of them on the persistent kernel.
mps_status run_jacobi_slots(mps_handle h, hipStream_t s, JacMat* mats, int n_slots, int nb_cap, int32_t* unconv,
                            int32_t* list, int32_t* cnt);

// One matrix X (complex128 [m][n], m, n <= m_cap) truncated on its charge
// blocks (row_q, col_q on the host); the kept rows, normalised, go to dst in
// the chain precision as rows [k][n] or, col_major, as columns [n][k]; k, the
// discarded weight and the kept charges (q_out, host) are returned.  region
// holds u1_layer_bytes(1, m_cap, chi_cap) bytes, sel one device SelOut.
mps_status u1_split_one(mps_handle h, hipStream_t s, const double2* X, int m, int n, const int32_t* row_q,
                        const int32_t* col_q, int kmax, double eps, char* region, int m_cap, int chi_cap,
                        SelOut* sel, void* dst, int col_major, bool c128, int* k_out, double* disc_out,
                        int32_t* q_out);

// kernel timing helpers (host)
void prof_begin(mps_handle h, hipStream_t s, int id);
void prof_end(mps_handle h, hipStream_t s, int id);
mps_status prof_harvest(mps_handle h, hipStream_t s);

#define PROF_LAUNCH(h, s, id, call)                    \
  do {                                                 \
    if ((h)->profile) prof_begin((h), (s), (id));      \
    MPS_TRY_HIP((h), (call));                          \
    if ((h)->profile) prof_end((h), (s), (id));        \
  } while (0)

mps_status mps_fail(mps_handle h, mps_status code, const std::string& msg);
// Make the workspace hold `bytes` for the running call.  A handle with a
// caller-owned workspace refuses a larger plan (MPS_ERR_CAPACITY); a
// planning handle records the size and returns MPS_ERR_UNSUPPORTED, which
// the entry points pass up before they queue any work.
mps_status mps_ensure_ws(mps_handle h, size_t bytes);

#define MPS_TRY_HIP(h, call)                                                         \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return mps_fail((h), MPS_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// Bump allocator that first measures, then carves the handle workspace.
struct WsPlan {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    size_t o = (off + 255) & ~size_t(255);
    off = o + count * sizeof(T);
    return o;
  }
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// ---------------------------------------------------------------------------
// descriptors passed to kernels (device memory)
// ---------------------------------------------------------------------------

// One two-site update of a Hastings-form chain (bond b joins sites b, b+1).
// Complex element type T of the chain (float2 = complex64 or double2 =
// complex128) applies to B, G, T and Vh.
struct BondItem {
  void* Bl;              // site b tensor, [chi_max][d][chi_max] (read, then rewritten)
  void* Br;              // site b+1 tensor
  const double* lam_l;   // Schmidt values left of site b (virtual bond b)
  double* lam_m;         // virtual bond b+1 (output)
  int32_t* chi;          // chain's chi array; chi[b], chi[b+1], chi[b+2]
  const void* G;         // gate [d*d][d*d]
  double* disc;          // chain's per-bond discarded weight accumulator (entry b)
  double2* X;            // workspace: theta' complex128 [(d chi_max)^2]
  void* T;               // workspace: theta~' [(d chi_max)^2]
  void* Vh;              // workspace: kept V^dag rows [chi_max][d chi_max]
  double2* gram;         // workspace of the eigendecomposition split of multi-panel matrices:
  double2* urows;        //   the Gram theta' theta'^dag and the rows U^dag theta' [(d chi_max)^2] (else null)
  int32_t b, d, chi_max, pad;   // pad: the item's offset in a discarded-weight log slice
};

// One Krylov-TEBD bond update's propagator job (ktebd.hip).
struct KryJob {
  const double2* h;    // bond term [D][D] complex128, D = d*d
  double2* part;       // [nblk][D][D] partial sums of the reduced matrix rho
  double2* hist;       // [2][n_max+1][D][D]: Krylov vectors Z_j, then polynomials Q_j(h)
  void* G;             // output propagator [D][D] in the chain precision
  int32_t* n_used;     // optional: Krylov vectors used
  int32_t pad[2];
};

// One propagator to build: G = exp(-i tau h).
struct GateJob {
  const double2* h;
  float2* G64;      // optional complex64 output
  double2* G128;    // optional complex128 output
  double tau;
};

// One matrix handled by the batched Jacobi SVD (rows are orthogonalised).
struct JacMat {
  double2* X;      // [m][ld] complex128, rows of length n
  int32_t* rowmap; // [m] row order used to form blocks (rows sorted by norm each sweep)
  int32_t m, n, ld, nb;  // rows, columns, leading dim, number of row blocks (even)
  int32_t conv, rot;     // converged flag, rotations applied in the running sweep
  int32_t kmax, pad;     // cap on the kept count (0 = use the launch constant)
  double fro2;           // |X|_F^2 at the start
  double* nrm2;          // [m] squared row norms by physical row, rewritten by every round
};

// Output of the selection step (sorted singular values, count rule).
struct SelOut {
  int32_t k;      // kept count
  int32_t m;      // rows considered
  double disc;    // discarded weight
  double norm2;   // sum of all s^2
  double nk;      // sqrt(sum of kept s^2)
};

// One complex GEMM problem C = alpha * A * op(B), dims may live on the device.
struct GemmProb {
  const void* A;
  const void* B;
  void* C;
  int32_t M, N, K;         // used when the matching *_dev pointer is null
  int32_t lda, ldb, ldc;
  const int32_t* M_dev;    // optional: M = M_mul * (*M_dev)
  const int32_t* N_dev;
  const int32_t* K_dev;
  int32_t M_mul, N_mul, K_mul;
  const double* inv_alpha_dev;  // optional: alpha = 1 / (*inv_alpha_dev)
  double alpha;
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
hipError_t launch_gates(hipStream_t s, const GateJob* jobs, int n, int dd);
// Workgroups of the list-walking launches (theta and batched GEMM with
// tile_offs): 8 per CU of the 256-CU device.
constexpr int kListGrid = 2048;
// Workgroups are dealt to the chip's 8 XCDs round-robin in launch order, and
// every XCD has its own L2.  For a batch of products of tiles_cap tiles each,
// launch index L goes to product xcd + 8 j (xcd = L % 8, j = (L / 8) /
// tiles_cap) and tile (L / 8) % tiles_cap: every product stays on one XCD, so
// its tiles, which read the same operand panels, meet in one L2, and the
// products of a layer (large ones in the bulk of a chain, small ones at its
// ends) are interleaved over the XCDs.  The grid is xcd_grid(n, tiles_cap);
// returns false past the last product.
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_item_tile(int L, int n_items, int tiles_cap, int& item, int& tile) {
  const int slot = L / kXcds;
  item = L % kXcds + kXcds * (slot / tiles_cap);
  tile = slot % tiles_cap;
  return item < n_items;
}
inline long long xcd_grid(long long n_items, long long tiles_cap) {
  return (n_items + kXcds - 1) / kXcds * kXcds * tiles_cap;
}
// tile_offs (optional, n_items + 1 int32 of device scratch): walk the list of
// the bonds' real tiles with a fixed grid instead of a grid sized for chi_cap
// Warm start of a layer's Jacobi (warm.hip): theta' <- Q^dag theta' with Q
// from the Householder QR of Lambda_l B_b, for the bonds of 64 < d chi_l <=
// 512 rows.  wsA: n_items * warm_a_elems(d, chi_cap) complex128, wsT:
// n_items * warm_t_elems(chi_cap).
size_t warm_a_elems(int d, int chi_cap);
size_t warm_t_elems(int chi_cap);
hipError_t launch_warm_start(hipStream_t s, const BondItem* items, int n_items, int d, int chi_cap, int chi_eff,
                             bool c128, double2* wsA, double2* wsT);
hipError_t launch_theta(hipStream_t s, const BondItem* items, int n_items, int d, int chi_cap, bool c128,
                        unsigned long long* stats, const void* G_override = nullptr, int32_t* tile_offs = nullptr);
hipError_t launch_ktebd_identity(hipStream_t s, void* G, int dd, bool c128);
hipError_t launch_ktebd_rho(hipStream_t s, const BondItem* items, const KryJob* jobs, int n_items, int d, int nblk);
hipError_t launch_ktebd_krylov(hipStream_t s, const KryJob* jobs, int n_items, int d, int nblk, int n_max, double tol,
                               double tau, bool c128, uint32_t* status);
hipError_t launch_jac_prep_bonds(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, int bs,
                                 int32_t* rowmap_ws, double* nrm_ws, int m_cap, uint32_t* status,
                                 unsigned long long* stats = nullptr);
hipError_t launch_jac_prep_plain(hipStream_t s, JacMat* mats, int n_mats, uint32_t* status);
// Eigendecomposition split of a layer (Sec. "Basic concepts": theta' theta'^dag
// = U lambda^2 U^dag, then U^dag theta' = lambda V^dag) for matrices of any
// size: the steps around the Jacobi of the Grams (probs: one GemmProb per item)
hipError_t launch_eig_gram(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, GemmProb* probs,
                           int m_cap, int32_t* tile_offs, uint32_t* status);
hipError_t launch_eig_rows(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, GemmProb* probs,
                           int m_cap, int n_cap, double floor);
// Column split of a Jacobi round (see jac_round_kernel): S workgroups per
// panel pair; part holds n_mats * pairs * S partial Grams of 64 x 64.
struct JacSplit {
  int S;          // workgroups per pair (1 = no split)
  int pairs;      // pair slots per matrix in part (nb_cap / 2)
  int phase;      // 0 = partial Grams, 1 = sum, solve, rotate; 2 = unsplit
  int eig;        // loop mode: one Gram, its eigensolve to convergence, one rotation
  double2* part;
};
// list / n_list (slot mode, optional): the round runs on the matrices
// mats[list[k]], k < n_list[0] (at most n_mats), n_grid workgroup rows taking
// them in turn (a loop-mode launch only when n_list[1], their largest block
// count, is 2); otherwise on mats[0, n_mats), one workgroup row each.
hipError_t launch_jac_round(hipStream_t s, JacMat* mats, int n_mats, int nb_cap, int round,
                            double tol, double abs_tol, int inner_sweeps, int loop_sweeps, unsigned long long* stats,
                            int threads, int split_S = 1, double2* split_part = nullptr, int eig = 0,
                            const int32_t* list = nullptr, const int32_t* n_list = nullptr, int n_grid = 0);
// Slot mode: the slots of mats[0, n) still to do (conv == 0), in slot order,
// to list; their count to cnt[0] and their largest block count (at least 2)
// to cnt[1].
hipError_t launch_jac_list(hipStream_t s, const JacMat* mats, int n, int32_t* list, int32_t* cnt);
// Capacity of the handle's persistent-Jacobi counters: matrices per launch.
constexpr int kSchedCap = 65536;
constexpr int kSchedBlkCap = 1 << 20;   // per-block round counters (matrices x blocks)
constexpr size_t kSchedBytes = 16 + 2 * sizeof(int32_t) * (size_t)kSchedCap + sizeof(int32_t) * (size_t)kSchedBlkCap;
// Counters of a persistent Jacobi launch (device memory, cleared by the launch).
struct JacSched {
  unsigned long long* head;  // next work item
  int32_t* n_conv;           // matrices converged
  int32_t* abort;            // set when a wait ran out: every workgroup leaves
  int32_t* done;             // [n] finished pair items per matrix
  int32_t* ready;            // [n] last sweep whose row order is set
  int32_t* bdone;            // [n][nb_cap] rounds each block has been through (or null)
  int32_t n, nb_cap, max_sweeps, spin_limit;
  // slot mode (or null): the launch lists the matrices still to do among
  // mats[0, n) (conv == 0) in list[], their count and largest block count in
  // act[0], act[1]; n and nb_cap are then capacities
  int32_t* list;
  int32_t* act;
};
// All sweeps of n matrices (at most max_sweeps) in one launch of `grid`
// resident workgroups (see jac_persist_kernel), then the convergence flags.
hipError_t launch_jac_persist(hipStream_t s, JacMat* mats, const JacSched& sc, double tol, double abs_tol,
                              int inner_sweeps, unsigned long long* stats, int threads, int grid,
                              uint32_t* status);
hipError_t launch_jac_sweep_end(hipStream_t s, JacMat* mats, int n_mats, int32_t* unconverged);
hipError_t launch_jac_sort(hipStream_t s, JacMat* mats, int n_mats, int m_cap);
hipError_t launch_jac_flag_noconv(hipStream_t s, const int32_t* unconverged, uint32_t* status);
hipError_t launch_jac_max_nb(hipStream_t s, const JacMat* mats, int n_mats, int32_t* out);
hipError_t launch_layer_dims(hipStream_t s, const BondItem* items, int n_items, int32_t* out);
hipError_t launch_select(hipStream_t s, JacMat* mats, int n_mats, int32_t* perm_ws, double* s2_ws,
                         int m_cap, int kmax_const, double eps, SelOut* out);
// Per-update discarded-weight log of mps_tebd_step_ex: the entry of an item
// is log[step * step_stride + layer_off + item.pad] with the step read from
// a device counter (so a captured step logs into its replay's slice).
struct DiscLog {
  double* log = nullptr;
  const int32_t* step = nullptr;
  long long step_stride = 0, layer_off = 0;
};
hipError_t launch_wb_right(hipStream_t s, const BondItem* items, int n_items, const JacMat* mats,
                           const int32_t* perm_ws, const double* s2_ws, int m_cap, const SelOut* sel,
                           int chi_cap, int d, bool c128, const DiscLog& lg = DiscLog());
hipError_t launch_set_int(hipStream_t s, int32_t* p, int v);
hipError_t launch_inc_int(hipStream_t s, int32_t* p);
hipError_t launch_wb_left_probs(hipStream_t s, const BondItem* items, int n_items, const SelOut* sel,
                                GemmProb* probs);
hipError_t launch_gemm_bt_conj(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                               unsigned long long* stats, int32_t* tile_offs = nullptr);
hipError_t launch_gemm_nn(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                          unsigned long long* stats);
hipError_t launch_truncate_out(hipStream_t s, const JacMat* mat, const int32_t* perm, const double* s2,
                               const SelOut* sel, const double2* theta, int64_t m, int64_t n,
                               int64_t chi_max, double2* U, double* S, double2* Vh, int32_t* k_dev,
                               double* disc_dev, double* norm2_dev);
// site expectation values of op1 into row *step of a log (row stride step_stride)
hipError_t launch_observe_log(hipStream_t s, const mps_chain_desc& c, const double2* op1, double* log,
                              const int32_t* step, long long step_stride);
hipError_t launch_observe(hipStream_t s, const mps_chain_desc& c, const double2* op1, double* site_out,
                          const double2* op2, int op2_per_bond, double* bond_out, double* entropy_out);

// effective Hamiltonian, environments and Lanczos kernels (heff.hip)
struct SGemm {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  long long rsA, csA, rsB, csB, rsC, csC;
  int conjA, conjB;
  double alpha;
  const double* alpha_dev = nullptr;  // when set, alpha is read from the device
};
// GEMM tile shapes: shape classes of an M x N product, the candidate a class
// uses (process-wide table per precision, set by the autotuner) and a launch
// with an explicit candidate.
constexpr int kGemmShapeClasses = 4;
int gemm_shape_class(long long M, long long N);
void set_sgemm_choice(bool c128, int shape_class, int cand);
int get_sgemm_choice(bool c128, int shape_class);
hipError_t launch_sgemm_cand(hipStream_t s, const SGemm& P, bool c128, int cand);
// complex128 products probs[0..n) (device array) in one launch; M_max, N_max
// bound every problem's M and N
hipError_t launch_sgemm_batched(hipStream_t s, const SGemm* probs, int n_probs, int M_max, int N_max);
void set_bgemm_choice(bool c128, int shape_class, int cand);
int get_bgemm_choice(bool c128, int shape_class);
hipError_t launch_gemm_bt_conj_cand(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap,
                                    bool c128, unsigned long long* stats, int32_t* tile_offs, int cand);
struct MixDesc {
  int P1, P2, R, Q1, Q2, O1, O2;
  long long is_o1, is_o2, is_q1, is_q2, is_r;
  long long os_o1, os_o2, os_q1, os_q2, os_r;
};
hipError_t launch_sgemm(hipStream_t s, const SGemm& P, bool c128);
hipError_t launch_wmix_build(hipStream_t s, const void* W, void* Wm, int O1, int O2, int Q1, int Q2, int ws_o1,
                             int ws_o2, int ws_i1, int ws_i2, bool c128);
hipError_t launch_mix(hipStream_t s, const MixDesc& D, const void* in, const void* Wm, void* out, bool c128);
hipError_t launch_zero(hipStream_t s, double* a, int n);
// Workgroups of the first stage of launch_mdot; part holds kMdotBlocks * nv
// shares, which a second launch adds to out in a fixed order.
constexpr int kMdotBlocks = 1024;
hipError_t launch_mdot(hipStream_t s, const double2* V, long long ldv, int nv, const double2* r, long long n,
                       double2* out, double2* part);
hipError_t launch_msub(hipStream_t s, const double2* V, long long ldv, int nv, const double2* c, double2* r,
                       long long n);
hipError_t launch_scale_inv_sqrt(hipStream_t s, const double2* x, double2* y, long long n, const double* norm2);
hipError_t launch_combine(hipStream_t s, const double2* V, long long ldv, int nv, const double2* u, double nrm,
                          double2* x, long long n);
hipError_t launch_convert(hipStream_t s, const void* a, void* b, long long n, bool to_c64);
hipError_t launch_tridiag_expm(hipStream_t s, const double* alpha, const double* beta, int n, double tau_re,
                               double tau_im, double nrm, double2* u, double* err);
hipError_t launch_transpose_c128(hipStream_t s, const double2* a, double2* b, int m, int n);
hipError_t launch_write_rows(hipStream_t s, const JacMat* mat, const int32_t* perm, const double* s2, const SelOut* sel,
                             void* dst, int len, int col_major, bool c128);
