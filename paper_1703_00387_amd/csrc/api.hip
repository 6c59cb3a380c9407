// Host side of libmps: handle, workspace, argument checks, and the drivers
// that queue the kernels of the two-site update on a HIP stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"

namespace {

constexpr int kJacBlock = 32;   // rows per Jacobi block
constexpr int kFixedSweeps = 20;  // sweeps queued when the host may not synchronise
constexpr int kLoopInner = 4;     // inner sweeps per outer sweep for single-panel matrices
constexpr int kEigSweeps = 40;    // eigen split: sweeps of the 64x64 Hermitian Jacobi (it stops when converged)
constexpr int kSlotGrid = 1024;      // workgroup rows of a slot-mode loop launch

}  // namespace

int jac_nb(int m) {
  int nb = (m + kJacBlock - 1) / kJacBlock;
  if (nb < 2) nb = 2;
  if (nb & 1) nb++;
  return nb;
}

namespace {

// Upload a host array into workspace memory and wait for it (descriptors only).
template <class T>
mps_status upload(mps_handle h, hipStream_t s, void* dst, const std::vector<T>& src) {
  if (src.empty()) return MPS_OK;
  MPS_TRY_HIP(h, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  return MPS_OK;
}

}  // namespace

// Run the Jacobi sweeps on mats[0..n) (already prepared on the device).
mps_status mps_aux_streams(mps_handle h, int n) {
  while ((int)h->aux.size() < n) {
    hipStream_t st;
    MPS_TRY_HIP(h, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    h->aux.push_back(st);
  }
  while ((int)h->aux_ev.size() < n + 1) {
    hipEvent_t e;
    MPS_TRY_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->aux_ev.push_back(e);
  }
  return MPS_OK;
}

mps_status run_jacobi(mps_handle h, hipStream_t s, JacMat* mats, int n, int nb_cap, int m_cap, int32_t* unconv,
                      bool fixed, bool allow_split, double2* split_buf, size_t split_buf_bytes) {
  int nb = nb_cap;
  if (!fixed) {
    // eager mode: the largest actual block count bounds the rounds of a sweep
    MPS_TRY_HIP(h, launch_jac_max_nb(s, mats, n, unconv + 1));
    MPS_TRY_HIP(h, hipMemcpyAsync(h->host_pinned + 1, unconv + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    nb = std::min(nb_cap, std::max(2, (int)h->host_pinned[1]));
  }
  const int max_sweeps = fixed ? std::min(kFixedSweeps, h->jac_max_sweeps) : h->jac_max_sweeps;
  if (nb == 2 || fixed) {
    // Matrices of one 64-row panel run all their sweeps in one launch (with a
    // few inner sweeps per outer sweep); one that converges there is done.
    // Eager mode does this only when every matrix is that small: otherwise the
    // small ones stay in the rounds, where they run beside the others.  A
    // queued schedule cannot see the sizes, so it always starts with it.
    // The eigen split (Sec. "Basic concepts": the Hermitian A A^dag = U lambda^2
    // U^dag, then U^dag A = lambda V^dag) of a single-panel matrix is one Gram,
    // its Hermitian Jacobi run to convergence and one rotation of the rows.
    const bool eig = h->split_method == 1;
    PROF_LAUNCH(h, s, MPS_K_JAC_ROUND,
                launch_jac_round(s, mats, n, 2, 0, h->jac_tol, h->jac_abs,
                                 eig ? kEigSweeps : std::max(h->jac_inner_sweeps, kLoopInner), eig ? 1 : max_sweeps,
                                 h->profile ? h->stats_dev : nullptr, h->jac_threads, 1, nullptr, eig ? 1 : 0));
    if (nb == 2) {
      MPS_TRY_HIP(h, launch_jac_sweep_end(s, mats, n, unconv));
      MPS_TRY_HIP(h, launch_jac_flag_noconv(s, unconv, h->status_dev));
      return MPS_OK;
    }
  }
  // Few panel pairs (one large matrix): split every pair over S column
  // ranges so that more CUs work; the partial Grams live in a buffer of the
  // handle (eager mode only, never inside a captured graph).
  int S = 1;
  const int pairs = n * (nb / 2);
  // Large matrices (m >= 1024) split up to half a chip's worth of pairs: a
  // 2560 x 2560 SVD (40 pairs) took 1.19 s unsplit and 0.47 s with S = 6.
  const bool few = pairs < h->jac_split_below || (pairs < 128 && m_cap >= 1024);
  double2* split_part = h->split_part;
  if (!split_buf && h->ws_external) {
    // a caller-owned workspace: the partial Grams go behind the call's plan
    const size_t off = (h->ws_call + 255) & ~size_t(255);
    split_buf = (double2*)(h->ws + std::min(off, h->ws_bytes));
    split_buf_bytes = off < h->ws_bytes ? h->ws_bytes - off : 0;
  }
  if (!fixed && allow_split && h->jac_split_below > 0 && few) {
    S = std::max(1, std::min(std::min(16, 256 / std::max(pairs, 1)), std::max(1, m_cap / 64)));
    const size_t per_slice = (size_t)n * (nb_cap / 2) * 64 * 64 * sizeof(double2);
    if (split_buf) {
      // a caller-provided buffer: as many slices as it holds, no allocation
      S = std::max(1, std::min<int>(S, (int)(split_buf_bytes / per_slice)));
      split_part = S > 1 ? split_buf : nullptr;
    }
    const size_t need = per_slice * S;
    if (!split_buf && S > 1 && need > h->split_bytes) {
      if (h->split_part) MPS_TRY_HIP(h, hipFree(h->split_part));
      h->split_part = nullptr;
      h->split_bytes = 0;
      MPS_TRY_HIP(h, hipMalloc((void**)&h->split_part, need));
      h->split_bytes = need;
      split_part = h->split_part;
    }
  }
  if (S == 1 && h->jac_persistent && n <= kSchedCap) {
    // every remaining sweep in one persistent launch: pairs from a device
    // queue, convergence decided on the device, no host round trip
    JacSched sc;
    sc.head = (unsigned long long*)h->sched;
    sc.n_conv = (int32_t*)(h->sched + 8);
    sc.abort = (int32_t*)(h->sched + 12);
    sc.done = (int32_t*)(h->sched + 16);
    sc.ready = sc.done + kSchedCap;
    sc.bdone = (size_t)n * nb <= (size_t)kSchedBlkCap ? sc.ready + kSchedCap : nullptr;
    sc.n = n;
    sc.nb_cap = nb;
    sc.max_sweeps = h->jac_max_sweeps;
    sc.spin_limit = h->jac_spin_limit;
    sc.list = nullptr;
    sc.act = nullptr;
    const int grid = std::max(1, std::min(h->n_cu, n * (nb / 2)));
    PROF_LAUNCH(h, s, MPS_K_JAC_ROUND,
                launch_jac_persist(s, mats, sc, h->jac_tol, h->jac_abs, h->jac_inner_sweeps,
                                   h->profile ? h->stats_dev : nullptr, h->jac_threads, grid, h->status_dev));
    return MPS_OK;
  }
  bool done = false;
  for (int sw = 0; sw < max_sweeps && !done; ++sw) {
    if (sw > 0) MPS_TRY_HIP(h, launch_jac_sort(s, mats, n, m_cap));
    for (int r = 0; r < nb - 1; ++r)
      PROF_LAUNCH(h, s, MPS_K_JAC_ROUND, launch_jac_round(s, mats, n, nb_cap, r, h->jac_tol, h->jac_abs, h->jac_inner_sweeps, 0,
                                                              h->profile ? h->stats_dev : nullptr, h->jac_threads, S,
                                                              split_part));
    MPS_TRY_HIP(h, launch_jac_sweep_end(s, mats, n, unconv));
    if (!fixed && sw >= 1) {
      if (h->profile) {
        mps_status ps = prof_harvest(h, s);
        if (ps != MPS_OK) return ps;
      }
      MPS_TRY_HIP(h, hipMemcpyAsync(h->host_pinned, unconv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      MPS_TRY_HIP(h, hipStreamSynchronize(s));
      if (h->host_pinned[0] == 0) done = true;
    }
  }
  if (!done) MPS_TRY_HIP(h, launch_jac_flag_noconv(s, unconv, h->status_dev));
  return MPS_OK;
}

mps_status run_jacobi_slots(mps_handle h, hipStream_t s, JacMat* mats, int n_slots, int nb_cap, int32_t* unconv,
                            int32_t* list, int32_t* cnt) {
  if (n_slots <= 0) return MPS_OK;
  if (n_slots > kSchedCap || (size_t)n_slots * nb_cap > (size_t)kSchedBlkCap)
    return mps_fail(h, MPS_ERR_CAPACITY, "too many Jacobi slots");
  const bool eig = h->split_method == 1;
  unsigned long long* stats = h->profile ? h->stats_dev : nullptr;
  // the slots to do; when every one has one panel, all their sweeps in one
  // launch (decided on the device); else the rounds take them all
  MPS_TRY_HIP(h, launch_jac_list(s, mats, n_slots, list, cnt));
  PROF_LAUNCH(h, s, MPS_K_JAC_ROUND,
              launch_jac_round(s, mats, n_slots, 2, 0, h->jac_tol, h->jac_abs,
                               eig ? kEigSweeps : std::max(h->jac_inner_sweeps, kLoopInner),
                               eig ? 1 : h->jac_max_sweeps, stats, h->jac_threads, 1, nullptr, eig ? 1 : 0, list,
                               cnt, kSlotGrid));
  if (nb_cap == 2) {
    MPS_TRY_HIP(h, launch_jac_sweep_end(s, mats, n_slots, unconv));
    MPS_TRY_HIP(h, launch_jac_flag_noconv(s, unconv, h->status_dev));
    return MPS_OK;
  }
  // the rest on the persistent kernel, which lists them again
  JacSched sc;
  sc.head = (unsigned long long*)h->sched;
  sc.n_conv = (int32_t*)(h->sched + 8);
  sc.abort = (int32_t*)(h->sched + 12);
  sc.done = (int32_t*)(h->sched + 16);
  sc.ready = sc.done + kSchedCap;
  sc.bdone = sc.ready + kSchedCap;
  sc.n = n_slots;
  sc.nb_cap = nb_cap;
  sc.max_sweeps = h->jac_max_sweeps;
  sc.spin_limit = h->jac_spin_limit;
  sc.list = list;
  sc.act = cnt;
  PROF_LAUNCH(h, s, MPS_K_JAC_ROUND,
              launch_jac_persist(s, mats, sc, h->jac_tol, h->jac_abs, h->jac_inner_sweeps, stats, h->jac_threads,
                                 h->n_cu, h->status_dev));
  return MPS_OK;
}


void prof_begin(mps_handle h, hipStream_t s, int id) {
  size_t i = h->ev_pending.size() * 2;
  while (h->ev_pool.size() < i + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    h->ev_pool.push_back(e);
  }
  hipEventRecord(h->ev_pool[i], s);
  h->ev_pending.push_back({id, (int)i});
}

void prof_end(mps_handle h, hipStream_t s, int id) {
  (void)id;
  if (h->ev_pending.empty()) return;
  hipEventRecord(h->ev_pool[h->ev_pending.back().second + 1], s);
}

mps_status prof_harvest(mps_handle h, hipStream_t s) {
  if (h->ev_pending.empty()) return MPS_OK;
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  for (auto& pr : h->ev_pending) {
    float ms = 0.f;
    MPS_TRY_HIP(h, hipEventElapsedTime(&ms, h->ev_pool[pr.second], h->ev_pool[pr.second + 1]));
    h->k_ms[pr.first] += ms;
    h->k_launches[pr.first] += 1;
  }
  h->ev_pending.clear();
  return MPS_OK;
}

mps_status mps_fail(mps_handle h, mps_status code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

mps_status mps_ensure_ws(mps_handle h, size_t bytes) {
  h->ws_needed = std::max(h->ws_needed, bytes);
  if (h->plan_only) return mps_fail(h, MPS_ERR_UNSUPPORTED, "planning only");
  h->ws_call = bytes;
  if (bytes <= h->ws_bytes) return MPS_OK;
  if (h->ws_external)
    return mps_fail(h, MPS_ERR_CAPACITY, "the caller's workspace holds " + std::to_string(h->ws_bytes) +
                                             " bytes, this call needs " + std::to_string(bytes) +
                                             " (mps_workspace_size)");
  size_t want = std::max(bytes, h->ws_bytes + h->ws_bytes / 4);
  if (h->ws) {
    MPS_TRY_HIP(h, hipDeviceSynchronize());
    MPS_TRY_HIP(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  hipError_t e = hipMalloc((void**)&h->ws, want);
  if (e != hipSuccess) {
    h->ws = nullptr;
    return mps_fail(h, MPS_ERR_CAPACITY, std::string("workspace allocation failed: ") + hipGetErrorString(e));
  }
  h->ws_bytes = want;
  return MPS_OK;
}

// ---------------------------------------------------------------------------
// truncated SVD of one matrix: shared by mps_truncate (handle workspace) and
// mps_truncate_noalloc (the fixed device scratch below)
// ---------------------------------------------------------------------------
static mps_status truncate_check(mps_handle h, const void* theta, int64_t m, int64_t n, int64_t chi_max, double eps,
                          void* U, double* S, void* Vh, int32_t* k_dev, double* disc_dev, double* norm2_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!theta || !U || !S || !Vh || !k_dev || !disc_dev || !norm2_dev)
    return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (m < 1 || n < 1 || chi_max < 1) return mps_fail(h, MPS_ERR_SHAPE, "m, n, chi_max must be >= 1");
  if (!(eps == eps)) return mps_fail(h, MPS_ERR_INVALID, "eps is NaN");
  return MPS_OK;
}

struct TruncPlan {
  size_t oX, oM, oP, oS, oSel, oU, oR, oNr, off;
};

static TruncPlan truncate_plan(int64_t m, int64_t n) {
  WsPlan p;
  TruncPlan t;
  t.oX = p.take<double2>((size_t)m * n);
  t.oM = p.take<JacMat>(1);
  t.oP = p.take<int32_t>(m);
  t.oS = p.take<double>(m);
  t.oSel = p.take<SelOut>(1);
  t.oU = p.take<int32_t>(4);
  t.oR = p.take<int32_t>(m);
  t.oNr = p.take<double>(m);
  t.off = p.off;
  return t;
}

// ws holds truncate_plan(m, n).off bytes; split_buf (optional) the partial
// Grams of column-split rounds (else the handle's buffer, grown on demand).
static mps_status truncate_run(mps_handle h, hipStream_t s, const void* theta, int64_t m, int64_t n, int64_t chi_max,
                        double eps, void* U, double* S, void* Vh, int32_t* k_dev, double* disc_dev,
                        double* norm2_dev, char* ws, double2* split_buf, size_t split_bytes) {
  const TruncPlan t = truncate_plan(m, n);
  double2* X = (double2*)(ws + t.oX);
  JacMat* mat = (JacMat*)(ws + t.oM);
  MPS_TRY_HIP(h, hipMemcpyAsync(X, theta, (size_t)m * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  JacMat hm;
  std::memset(&hm, 0, sizeof(hm));
  hm.X = X;
  hm.rowmap = (int32_t*)(ws + t.oR);
  hm.nrm2 = (double*)(ws + t.oNr);
  hm.m = (int)m;
  hm.n = (int)n;
  hm.ld = (int)n;
  hm.nb = jac_nb((int)m);
  hm.kmax = (int)std::min<int64_t>(chi_max, m);
  std::vector<JacMat> hv(1, hm);
  mps_status st = upload(h, s, mat, hv);
  if (st != MPS_OK) return st;
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, mat, 1, h->status_dev));
  st = run_jacobi(h, s, mat, 1, hm.nb, (int)m, (int32_t*)(ws + t.oU), false, true, split_buf, split_bytes);
  if (st != MPS_OK) return st;
  SelOut* sel = (SelOut*)(ws + t.oSel);
  MPS_TRY_HIP(h, launch_select(s, mat, 1, (int32_t*)(ws + t.oP), (double*)(ws + t.oS), (int)m, hm.kmax,
                                count_rule_eps(h, eps), sel));
  MPS_TRY_HIP(h, launch_truncate_out(s, mat, (int32_t*)(ws + t.oP), (double*)(ws + t.oS), sel,
                                     (const double2*)theta, m, n, chi_max, (double2*)U, S, (double2*)Vh, k_dev,
                                     disc_dev, norm2_dev));
  return MPS_OK;
}

// The scratch of mps_truncate_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes its name to
// a kernel (on the host the name is only a stand-in); mps_create takes this
// device's address of it once with hipGetSymbolAddress, and the kernels get
// that address.  Layout: the truncation's workspace (X copy of at most
// 512 x 512, descriptors, row maps), then the partial Grams of the column
// split in the rest.
constexpr int64_t kNoAllocMaxDim = 512;
constexpr size_t kNoAllocScratchBytes = size_t(9) << 20;   // 9 MiB
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch (device current), once per device.
static mps_status scratch_setup(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return MPS_ERR_CAPACITY;
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MPS_ERR_HIP;
    g_scratch_ptr[device] = (char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return MPS_OK;
}

extern "C" {

mps_status mps_create(mps_handle* out, int device) {
  if (!out) return MPS_ERR_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MPS_ERR_INVALID;
  if (hipSetDevice(device) != hipSuccess) return MPS_ERR_HIP;
  mps_context* h = new (std::nothrow) mps_context();
  if (!h) return MPS_ERR_CAPACITY;
  h->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete h;
    return MPS_ERR_HIP;
  }
  h->n_cu = std::max(1, prop.multiProcessorCount);
  if (hipMalloc((void**)&h->status_dev, 256) != hipSuccess ||
      hipMemset(h->status_dev, 0, 256) != hipSuccess ||
      hipMalloc((void**)&h->sched, kSchedBytes) != hipSuccess ||
      hipHostMalloc((void**)&h->host_pinned, 256, hipHostMallocDefault) != hipSuccess) {
    if (h->status_dev) hipFree(h->status_dev);
    if (h->sched) hipFree(h->sched);
    delete h;
    return MPS_ERR_HIP;
  }
  h->stats_dev = (unsigned long long*)((char*)h->status_dev + 64);
  if (scratch_setup(device, &h->scratch) != MPS_OK) {
    hipFree(h->status_dev);
    hipFree(h->sched);
    hipHostFree(h->host_pinned);
    delete h;
    return MPS_ERR_HIP;
  }
  *out = h;
  return MPS_OK;
}

mps_status mps_create_ws(mps_handle* out, int device, void* workspace, size_t ws_bytes) {
  if (!out) return MPS_ERR_INVALID;
  *out = nullptr;
  if (!workspace && ws_bytes > 0) return MPS_ERR_INVALID;
  mps_status st = mps_create(out, device);
  if (st != MPS_OK) return st;
  (*out)->ws = (char*)workspace;
  (*out)->ws_bytes = ws_bytes;
  (*out)->ws_external = true;
  return MPS_OK;
}

size_t mps_workspace_size(int32_t op, int32_t dtype, int32_t n_chains, int32_t L, int32_t d, int32_t chi_max,
                          int32_t w, int32_t n_krylov) {
  // A planning handle: every entry point checks its arguments and plans its
  // workspace as for a real call, then stops before any work.
  // The pointers below are never dereferenced.
  mps_context ctx;
  ctx.plan_only = true;
  void* fake = (void*)(uintptr_t)0x1000;
  double* fd = (double*)fake;
  int32_t* fi = (int32_t*)fake;
  if (dtype != MPS_C64 && dtype != MPS_C128) return 0;
  if (n_chains < 1 || L < 2 || d < 1 || chi_max < 1) return 0;
  const int64_t m = (int64_t)d * chi_max;
  switch (op) {
    case MPS_OP_TRUNCATE:
      mps_truncate(&ctx, nullptr, fake, m, m, chi_max, 0.0, fake, fd, fake, fi, fd, fd);
      break;
    case MPS_OP_TEBD: {
      std::vector<mps_chain_desc> cs((size_t)n_chains);
      for (auto& c : cs) {
        c.L = L;
        c.d = d;
        c.chi_max = chi_max;
        c.dtype = dtype;
        c.B = fake;
        c.lam = fd;
        c.chi = fi;
        c.hbond = fake;
        c.disc = fd;
      }
      mps_tebd_step(&ctx, nullptr, cs.data(), n_chains, 4, 0.05, 1, 1e-12, 0);
      break;
    }
    case MPS_OP_HEFF:
      if (w < 1) return 0;
      mps_heff_apply(&ctx, nullptr, dtype, fake, fake, fake, fake, fake, fake, chi_max, d, d, chi_max, w, w, w);
      break;
    case MPS_OP_KRYLOV:
      if (w < 1 || n_krylov < 1) return 0;
      mps_krylov_expm(&ctx, nullptr, dtype, fake, fake, fake, fake, fake, chi_max, d, d, chi_max, w, w, w, 0.01, 0.0,
                      n_krylov, 1e-10, fi, fd);
      break;
    case MPS_OP_TDVP: {
      if (w < 1 || n_krylov < 1) return 0;
      mps_oc_chain c;
      std::memset(&c, 0, sizeof(c));
      c.L = L;
      c.d = d;
      c.chi_max = chi_max;
      c.dtype = dtype;
      c.w = w;
      c.M = fake;
      c.chi = fi;
      c.W = fake;
      mps_tdvp2_step(&ctx, nullptr, &c, 0.02, 1, 1e-12, n_krylov, 1e-10, fd, fi);
      break;
    }
    default:
      return 0;
  }
  if (ctx.ws_needed == 0) return 0;   // the arguments were refused
  // room behind the plan for the partial Grams of column-split Jacobi rounds
  // (at most 256 pair slices of 64 x 64 complex128)
  return ((ctx.ws_needed + 255) & ~size_t(255)) + (size_t)256 * 64 * 64 * sizeof(double2);
}

mps_status mps_workspace_needed(mps_handle h, size_t* bytes) {
  if (!h || !bytes) return MPS_ERR_INVALID;
  *bytes = h->ws_needed;
  return MPS_OK;
}

mps_status mps_destroy(mps_handle h) {
  if (!h) return MPS_ERR_INVALID;
  hipSetDevice(h->device);
  hipDeviceSynchronize();
  for (auto e : h->ev_pool) hipEventDestroy(e);
  for (auto e : h->aux_ev) hipEventDestroy(e);
  for (auto st : h->aux) hipStreamDestroy(st);
  if (h->graph_exec) hipGraphExecDestroy(h->graph_exec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->ws && !h->ws_external) hipFree(h->ws);
  if (h->split_part) hipFree(h->split_part);
  if (h->status_dev) hipFree(h->status_dev);
  if (h->sched) hipFree(h->sched);
  if (h->host_pinned) hipHostFree(h->host_pinned);
  delete h;
  return MPS_OK;
}

const char* mps_last_error(mps_handle h) { return h ? h->err.c_str() : "null handle"; }

mps_status mps_reserve(mps_handle h, size_t bytes) {
  if (!h) return MPS_ERR_INVALID;
  return mps_ensure_ws(h, bytes);
}

mps_status mps_set_option(mps_handle h, int option, double value) {
  if (!h) return MPS_ERR_INVALID;
  switch (option) {
    case 0:
      if (!(value > 0.0 && value < 1.0)) return mps_fail(h, MPS_ERR_INVALID, "Jacobi tolerance must be in (0,1)");
      h->jac_tol = value;
      return MPS_OK;
    case 1:
      if (!(value >= 1.0 && value <= 1000.0)) return mps_fail(h, MPS_ERR_INVALID, "sweeps must be in [1,1000]");
      h->jac_max_sweeps = (int)value;
      return MPS_OK;
    case 2:
      if (!(value >= kJacAbsFloor && value < 1.0))
        return mps_fail(h, MPS_ERR_INVALID, "absolute tolerance must be in [1e-30,1)");
      h->jac_abs = value;
      return MPS_OK;
    case 3:
      h->profile = value != 0.0;
      return MPS_OK;
    case 4:
      if (!(value >= 1.0 && value <= 64.0)) return mps_fail(h, MPS_ERR_INVALID, "inner sweeps must be in [1,64]");
      h->jac_inner_sweeps = (int)value;
      return MPS_OK;
    case 5:
      if (value != 256.0 && value != 512.0) return mps_fail(h, MPS_ERR_INVALID, "Jacobi threads must be 256 or 512");
      h->jac_threads = (int)value;
      return MPS_OK;
    case 6:
      if (!(value >= 0.0 && value <= 1.0e6)) return mps_fail(h, MPS_ERR_INVALID, "split threshold must be in [0,1e6]");
      h->jac_split_below = (int)value;
      return MPS_OK;
    case 7:
      if (value != 0.0 && value != 1.0) return mps_fail(h, MPS_ERR_INVALID, "split method must be 0 or 1");
      h->split_method = (int)value;
      return MPS_OK;
    case 8:
      if (value != 0.0 && value != 1.0) return mps_fail(h, MPS_ERR_INVALID, "persistent Jacobi must be 0 or 1");
      h->jac_persistent = (int)value;
      return MPS_OK;
    case 9:
      if (value != 0.0 && value != 1.0) return mps_fail(h, MPS_ERR_INVALID, "warm start must be 0 or 1");
      h->warm_start = (int)value;
      return MPS_OK;
    case 10:
      if (!(value >= 1.0 && value <= 1.0e8)) return mps_fail(h, MPS_ERR_INVALID, "spin limit must be in [1,1e8]");
      h->jac_spin_limit = (int)value;
      return MPS_OK;
    default:
      return mps_fail(h, MPS_ERR_INVALID, "unknown option");
  }
}

mps_status mps_device_status(mps_handle h, mps_stream stream, uint32_t* word) {
  if (!h || !word) return MPS_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  uint32_t w = 0;
  MPS_TRY_HIP(h, hipMemcpy(&w, h->status_dev, sizeof(w), hipMemcpyDeviceToHost));
  MPS_TRY_HIP(h, hipMemset(h->status_dev, 0, sizeof(w)));
  *word = w;
  if (w & MPS_DEV_NONFINITE) return mps_fail(h, MPS_ERR_NONFINITE, "non-finite values met on the device");
  if (w & (MPS_DEV_NOCONV_SVD | MPS_DEV_NOCONV_LANCZOS))
    return mps_fail(h, MPS_ERR_NOCONV, "an iteration did not converge");
  if (w & MPS_DEV_SCHED_TIMEOUT)
    return mps_fail(h, MPS_ERR_NOCONV, "a persistent Jacobi wait ran out (results incomplete)");
  if (w & MPS_DEV_CHARGE)
    return mps_fail(h, MPS_ERR_SHAPE, "a bond of a charge-carrying chain shared no charge across its cut (skipped)");
  return MPS_OK;
}

mps_status mps_kernel_stats(mps_handle h, mps_stream stream, int32_t kernel, double* total_ms, int64_t* launches,
                            uint64_t* work, int32_t reset) {
  if (!h || kernel < 0 || kernel >= MPS_NKERNELS) return MPS_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  mps_status st = prof_harvest(h, s);
  if (st != MPS_OK) return st;
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  unsigned long long w[MPS_NSTATS];
  MPS_TRY_HIP(h, hipMemcpy(w, h->stats_dev, sizeof(w), hipMemcpyDeviceToHost));
  static const int work_slot[MPS_NKERNELS] = {0, 1, -1, -1, 3, 5, -1, -1, -1};
  if (total_ms) *total_ms = h->k_ms[kernel];
  if (launches) *launches = h->k_launches[kernel];
  if (work) *work = work_slot[kernel] >= 0 ? w[work_slot[kernel]] : 0;
  if (reset) {
    for (int i = 0; i < MPS_NKERNELS; ++i) {
      h->k_ms[i] = 0.0;
      h->k_launches[i] = 0;
    }
    MPS_TRY_HIP(h, hipMemset(h->stats_dev, 0, sizeof(w)));
  }
  return MPS_OK;
}

mps_status mps_gates(mps_handle h, mps_stream stream, int32_t n, int32_t dd, const void* hmat, const double* tau,
                     void* G64, void* G128) {
  if (!h) return MPS_ERR_INVALID;
  if (n < 0 || dd < 1 || dd > 32) return mps_fail(h, MPS_ERR_SHAPE, "need n >= 0 and 1 <= dd <= 32");
  if (n == 0) return MPS_OK;
  if (!hmat || !tau || (!G64 && !G128)) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> taus(n);
  MPS_TRY_HIP(h, hipMemcpyAsync(taus.data(), tau, n * sizeof(double), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  std::vector<GateJob> jobs(n);
  for (int i = 0; i < n; ++i) {
    jobs[i].h = (const double2*)hmat + (size_t)i * dd * dd;
    jobs[i].G64 = G64 ? (float2*)G64 + (size_t)i * dd * dd : nullptr;
    jobs[i].G128 = G128 ? (double2*)G128 + (size_t)i * dd * dd : nullptr;
    jobs[i].tau = taus[i];
  }
  mps_status st = mps_ensure_ws(h, n * sizeof(GateJob) + 256);
  if (st != MPS_OK) return st;
  st = upload(h, s, h->ws, jobs);
  if (st != MPS_OK) return st;
  MPS_TRY_HIP(h, launch_gates(s, (const GateJob*)h->ws, n, dd));
  return MPS_OK;
}

mps_status mps_truncate(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n, int64_t chi_max,
                        double eps, void* U, double* S, void* Vh, int32_t* k_dev, double* disc_dev,
                        double* norm2_dev) {
  mps_status st = truncate_check(h, theta, m, n, chi_max, eps, U, S, Vh, k_dev, disc_dev, norm2_dev);
  if (st != MPS_OK) return st;
  if (m > 4096 || n > 4096) return mps_fail(h, MPS_ERR_CAPACITY, "m and n are limited to 4096");
  st = mps_ensure_ws(h, truncate_plan(m, n).off);
  if (st != MPS_OK) return st;
  return truncate_run(h, (hipStream_t)stream, theta, m, n, chi_max, eps, U, S, Vh, k_dev, disc_dev, norm2_dev, h->ws,
                      nullptr, 0);
}

// S <- S / (sum_{j<k} S_j^2)^(1/2) for the kept values (one workgroup)
__global__ __launch_bounds__(256) void renorm_kept_kernel(double* S, const int32_t* k_dev) {
  __shared__ double red[256];
  const int k = *k_dev;
  double a = 0.0;
  for (int j = threadIdx.x; j < k; j += 256) a += S[j] * S[j];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double nk = sqrt(red[0]);
  const double inv = nk > 0.0 ? 1.0 / nk : 0.0;
  for (int j = threadIdx.x; j < k; j += 256) S[j] *= inv;
}

mps_status mps_truncate_ex(mps_handle h, mps_stream stream, int32_t dtype, const void* theta, int64_t m, int64_t n,
                           int64_t chi_max, double eps, int32_t renormalize, void* U, double* S, void* Vh,
                           int32_t* k_dev, double* disc_dev, double* norm2_dev) {
  mps_status st = truncate_check(h, theta, m, n, chi_max, eps, U, S, Vh, k_dev, disc_dev, norm2_dev);
  if (st != MPS_OK) return st;
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "dtype must be MPS_C64 or MPS_C128");
  if (renormalize != 0 && renormalize != 1) return mps_fail(h, MPS_ERR_INVALID, "renormalize must be 0 or 1");
  if (m > 4096 || n > 4096) return mps_fail(h, MPS_ERR_CAPACITY, "m and n are limited to 4096");
  const bool c64 = dtype == MPS_C64;
  WsPlan p;
  const size_t oT = p.take<char>(truncate_plan(m, n).off);
  size_t oX = 0, oU = 0, oV = 0;
  if (c64) {
    oX = p.take<double2>((size_t)m * n);
    oU = p.take<double2>((size_t)m * chi_max);
    oV = p.take<double2>((size_t)chi_max * n);
  }
  st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char* ws = h->ws;
  const void* th = theta;
  void* Uo = U;
  void* Vo = Vh;
  if (c64) {
    // the SVD runs in FP64: theta up-converted, the factors converted back
    MPS_TRY_HIP(h, launch_convert(s, theta, ws + oX, m * n, false));
    th = ws + oX;
    Uo = ws + oU;
    Vo = ws + oV;
    // cleared by kernels (no memset nodes if the caller captures the call)
    MPS_TRY_HIP(h, launch_zero(s, (double*)Uo, (int)(2 * m * chi_max)));
    MPS_TRY_HIP(h, launch_zero(s, (double*)Vo, (int)(2 * chi_max * n)));
  }
  st = truncate_run(h, s, th, m, n, chi_max, eps, Uo, S, Vo, k_dev, disc_dev, norm2_dev, ws + oT, nullptr, 0);
  if (st != MPS_OK) return st;
  if (c64) {
    MPS_TRY_HIP(h, launch_convert(s, Uo, U, m * chi_max, true));
    MPS_TRY_HIP(h, launch_convert(s, Vo, Vh, chi_max * n, true));
  }
  if (renormalize) {
    renorm_kept_kernel<<<1, 256, 0, s>>>(S, k_dev);
    MPS_TRY_HIP(h, hipGetLastError());
  }
  return MPS_OK;
}

mps_status mps_truncate_noalloc(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n,
                                int64_t chi_max, double eps, void* U, double* S, void* Vh, int32_t* k_dev,
                                double* disc_dev, double* norm2_dev) {
  mps_status st = truncate_check(h, theta, m, n, chi_max, eps, U, S, Vh, k_dev, disc_dev, norm2_dev);
  if (st != MPS_OK) return st;
  if (m > kNoAllocMaxDim || n > kNoAllocMaxDim)
    return mps_fail(h, MPS_ERR_CAPACITY, "mps_truncate_noalloc: m and n are limited to 512 (its fixed scratch)");
  char* base = h->scratch;   // device address of this device's copy of the scratch array
  if (!base) return mps_fail(h, MPS_ERR_HIP, "mps_truncate_noalloc: scratch address unavailable on this device");
  const size_t off = (truncate_plan(m, n).off + 255) & ~size_t(255);
  if (off > kNoAllocScratchBytes) return mps_fail(h, MPS_ERR_CAPACITY, "mps_truncate_noalloc: scratch too small");
  // no event timing here: creating events is not allowed on this path
  struct ProfGuard {
    mps_handle h;
    bool saved;
    ~ProfGuard() { h->profile = saved; }
  } guard{h, h->profile};
  h->profile = false;
  return truncate_run(h, (hipStream_t)stream, theta, m, n, chi_max, eps, U, S, Vh, k_dev, disc_dev, norm2_dev, base,
                      (double2*)(base + off), kNoAllocScratchBytes - off);
}

mps_status mps_observe(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* op1,
                       double* site_out, const void* op2, int32_t op2_per_bond, double* bond_out,
                       double* entropy_out) {
  if (!h) return MPS_ERR_INVALID;
  if (!chain) return mps_fail(h, MPS_ERR_INVALID, "null chain");
  const mps_chain_desc& c = *chain;
  if (c.L < 2 || c.d < 1 || c.d > 5 || c.chi_max < 1) return mps_fail(h, MPS_ERR_SHAPE, "bad chain shape");
  if (c.dtype != MPS_C64 && c.dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "bad dtype");
  if (c.d * c.chi_max > 2560) return mps_fail(h, MPS_ERR_CAPACITY, "observe needs d*chi_max <= 2560");
  if (!c.B || !c.lam || !c.chi) return mps_fail(h, MPS_ERR_INVALID, "null chain pointer");
  MPS_TRY_HIP(h, launch_observe((hipStream_t)stream, c, (const double2*)op1, site_out, (const double2*)op2,
                                op2_per_bond, bond_out, entropy_out));
  return MPS_OK;
}

mps_status mps_tebd_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                         int32_t order, double dt, int32_t n_steps, double eps_local, uint32_t flags) {
  return tebd_impl(h, stream, chains, n_chains, order, dt, n_steps, eps_local, flags, 0, 1 << 30);
}

mps_status mps_tebd_step_ex(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                            int32_t order, double dt, int32_t n_steps, double eps_local, uint32_t flags,
                            void* ckpt_arena, size_t ckpt_bytes, double* disc_log_dev, const void* obs_op,
                            double* obs_log_dev) {
  return tebd_impl(h, stream, chains, n_chains, order, dt, n_steps, eps_local, flags, 0, 1 << 30, nullptr, nullptr,
                   ckpt_arena, ckpt_bytes, disc_log_dev, obs_op, obs_log_dev);
}

mps_status mps_ktebd_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                          double dt, int32_t n_steps, double eps_local, int32_t n_max, double tol, uint32_t flags,
                          int32_t* n_used_dev) {
  KryOpts k;
  k.n_max = n_max;
  k.tol = tol;
  k.n_used_dev = n_used_dev;
  return tebd_impl(h, stream, chains, n_chains, 0, dt, n_steps, eps_local, flags, 0, 1 << 30, &k);
}

mps_status mps_ktebd_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                             const mps_u1_chain* charges, int32_t n_chains, double dt, int32_t n_steps,
                             double eps_local, int32_t n_max, double tol, uint32_t flags, int32_t* n_used_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!charges) return mps_fail(h, MPS_ERR_INVALID, "null charges");
  KryOpts k;
  k.n_max = n_max;
  k.tol = tol;
  k.n_used_dev = n_used_dev;
  return tebd_impl(h, stream, chains, n_chains, 0, dt, n_steps, eps_local, flags, 0, 1 << 30, &k, charges);
}

mps_status mps_tebd_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                            const mps_u1_chain* charges, int32_t n_chains, int32_t order, double dt,
                            int32_t n_steps, double eps_local, uint32_t flags) {
  if (!h) return MPS_ERR_INVALID;
  if (!charges) return mps_fail(h, MPS_ERR_INVALID, "null charges");
  return tebd_impl(h, stream, chains, n_chains, order, dt, n_steps, eps_local, flags, 0, 1 << 30, nullptr, charges);
}

}  // extern "C"

// Runs n_steps steps; only layers lo <= index < hi of each step are applied
// (all of them for the public entry point).
mps_status tebd_impl(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains, int32_t order,
                     double dt, int32_t n_steps, double eps_local, uint32_t flags, int lo, int hi,
                     const KryOpts* kry, const mps_u1_chain* u1, void* ckpt, size_t ckpt_bytes, double* disc_log,
                     const void* obs_op, double* obs_log) {
  if (!h) return MPS_ERR_INVALID;
  if (!chains || n_chains < 1) return mps_fail(h, MPS_ERR_INVALID, "need at least one chain");
  if (order != 0 && order != 2 && order != 4) return mps_fail(h, MPS_ERR_INVALID, "order must be 0, 2 or 4");
  if (kry) {
    if (order != 0) return mps_fail(h, MPS_ERR_INVALID, "Krylov propagation runs on the sweep (order 0)");
    if (kry->n_max < 1 || kry->n_max > 32) return mps_fail(h, MPS_ERR_INVALID, "n_max must be in 1..32");
    if (!(kry->tol >= 0.0)) return mps_fail(h, MPS_ERR_INVALID, "tol must be >= 0");
  }
  if (n_steps < 0) return mps_fail(h, MPS_ERR_INVALID, "n_steps < 0");
  if (!(dt == dt) || !(eps_local == eps_local)) return mps_fail(h, MPS_ERR_INVALID, "NaN argument");
  if (flags & ~(MPS_FLAG_GRAPH | MPS_FLAG_FIXED_SWEEPS | MPS_FLAG_PLAIN | MPS_FLAG_CHECKPOINT | MPS_FLAG_OBSERVE))
    return mps_fail(h, MPS_ERR_INVALID, "unknown flag");
  if ((flags & MPS_FLAG_OBSERVE) && (!obs_op || !obs_log))
    return mps_fail(h, MPS_ERR_INVALID, "MPS_FLAG_OBSERVE needs an operator and a log");
  if (!(flags & MPS_FLAG_OBSERVE)) {
    obs_op = nullptr;
    obs_log = nullptr;
  }
  const bool plain = flags & MPS_FLAG_PLAIN;
  const bool checkpoint = flags & MPS_FLAG_CHECKPOINT;
  if (checkpoint) {
    if (!ckpt) return mps_fail(h, MPS_ERR_INVALID, "MPS_FLAG_CHECKPOINT needs an arena");
    if (flags & MPS_FLAG_GRAPH) return mps_fail(h, MPS_ERR_INVALID, "MPS_FLAG_CHECKPOINT excludes MPS_FLAG_GRAPH");
    if (u1 || kry) return mps_fail(h, MPS_ERR_INVALID, "MPS_FLAG_CHECKPOINT is for dense gate TEBD");
    if (n_steps > 0 && ckpt_bytes < mps_tebd_ckpt_bytes(chains, n_chains, n_steps))
      return mps_fail(h, MPS_ERR_CAPACITY, "arena smaller than mps_tebd_ckpt_bytes()");
  }
  if (disc_log && (u1 || kry)) return mps_fail(h, MPS_ERR_INVALID, "the discarded-weight log is for dense gate TEBD");
  if (u1) {
    for (int c = 0; c < n_chains; ++c)
      if (!u1[c].qbond) return mps_fail(h, MPS_ERR_INVALID, "null qbond");
      else if (u1[c].modulus < 0 || u1[c].modulus == 1)
        return mps_fail(h, MPS_ERR_INVALID, "modulus must be 0 (U(1)) or at least 2 (Z_n)");
  }
  if (plain && (flags & MPS_FLAG_GRAPH)) return mps_fail(h, MPS_ERR_INVALID, "MPS_FLAG_PLAIN excludes MPS_FLAG_GRAPH");
  hipStream_t s = (hipStream_t)stream;
  const bool graph = flags & MPS_FLAG_GRAPH;
  // no event timing inside a captured graph
  struct ProfGuard {
    mps_handle h;
    bool saved;
    ~ProfGuard() { h->profile = saved; }
  } guard{h, h->profile};
  if (graph) h->profile = false;
  const bool fixed = graph || (flags & MPS_FLAG_FIXED_SWEEPS);
  if (graph && s == nullptr) return mps_fail(h, MPS_ERR_INVALID, "graph capture needs a non-default stream");
  const int d = chains[0].d;
  const int dtype = chains[0].dtype;
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "dtype must be MPS_C64 or MPS_C128");
  const bool c128 = dtype == MPS_C128;
  const size_t esz = c128 ? sizeof(double2) : sizeof(float2);
  int chi_cap = 0;
  for (int c = 0; c < n_chains; ++c) {
    const mps_chain_desc& ch = chains[c];
    if (ch.d != d) return mps_fail(h, MPS_ERR_SHAPE, "all chains must share d");
    if (ch.dtype != dtype) return mps_fail(h, MPS_ERR_INVALID, "all chains must share dtype");
    if (ch.L < 2 || ch.d < 1 || ch.d > 5 || ch.chi_max < 1)
      return mps_fail(h, MPS_ERR_SHAPE, "bad chain shape (need L >= 2, 1 <= d <= 5, chi_max >= 1)");
    if ((int64_t)ch.d * ch.chi_max > 4096) return mps_fail(h, MPS_ERR_CAPACITY, "d*chi_max is limited to 4096");
    if (!ch.B || !ch.lam || !ch.chi || !ch.hbond || !ch.disc) return mps_fail(h, MPS_ERR_INVALID, "null chain pointer");
    chi_cap = std::max(chi_cap, ch.chi_max);
  }
  if (n_steps == 0) return MPS_OK;
  const int dd = d * d;

  // time-step classes and the layer sequence of one step
  std::vector<double> taus;
  std::vector<std::pair<int, int>> layers;  // (parity 0 = odd bonds b=0,2,..., class)
  int l_max = 0;
  for (int c = 0; c < n_chains; ++c) l_max = std::max(l_max, (int)chains[c].L);
  if (order == 0) {
    // the sweep: one bond per layer (in every chain), left to right then back,
    // all with dt/2; layer j < l_max-1 is bond j, layer l_max-1+j is bond L-2-j
    taus = {0.5 * dt};
    for (int j = 0; j < 2 * (l_max - 1); ++j) layers.push_back({j, 0});
  } else if (order == 2) {
    taus = {0.5 * dt, dt};
    layers = {{0, 0}, {1, 1}, {0, 0}};
  } else {
    const double p = 1.0 / (4.0 - std::cbrt(4.0));
    taus = {0.5 * p * dt, p * dt, 0.5 * (1.0 - 4.0 * p) * dt, (1.0 - 4.0 * p) * dt};
    const int cls[5] = {0, 0, 2, 0, 0};
    for (int st = 0; st < 5; ++st) {
      layers.push_back({0, cls[st]});
      layers.push_back({1, cls[st] + 1});
      layers.push_back({0, cls[st]});
    }
  }
  const int n_cls = (int)taus.size();

  // workspace plan
  WsPlan p;
  size_t gate_elems = 0;
  for (int c = 0; c < n_chains; ++c) gate_elems += (size_t)n_cls * (chains[c].L - 1) * dd * dd;
  size_t oG = p.take<double2>(gate_elems);
  size_t n_jobs = 0;
  for (int c = 0; c < n_chains; ++c) n_jobs += (size_t)n_cls * (chains[c].L - 1);
  size_t oJobs = p.take<GateJob>(n_jobs);
  // multi-panel matrices under the eigendecomposition split take two more
  // slots per item (the Gram and the rows U^dag theta')
  const bool eig_slots = h->split_method == 1 && !u1 && d * chi_cap > 64;
  // per parity: items and their workspace slots
  size_t n_par[2] = {0, 0}, slot_bytes[2] = {0, 0};
  for (int c = 0; c < n_chains; ++c) {
    const mps_chain_desc& ch = chains[c];
    size_t sq = (size_t)ch.d * ch.chi_max * ch.d * ch.chi_max;
    for (int b = 0; b < ch.L - 1; ++b) {
      int par = b & 1;
      n_par[par]++;
      slot_bytes[par] += ((sq * sizeof(double2) + 255) & ~size_t(255)) + ((sq * esz + 255) & ~size_t(255)) +
                         (((size_t)ch.chi_max * ch.d * ch.chi_max * esz + 255) & ~size_t(255)) +
                         (eig_slots ? 2 * ((sq * sizeof(double2) + 255) & ~size_t(255)) : 0);
    }
  }
  const size_t max_items = std::max(n_par[0], n_par[1]);
  size_t oSlots = p.take<char>(std::max(slot_bytes[0], slot_bytes[1]) + 256);
  size_t oItems = p.take<BondItem>((n_par[0] + n_par[1]) * (order == 0 ? 2 : n_cls));
  size_t oMats = p.take<JacMat>(max_items);
  size_t oSel = p.take<SelOut>(max_items);
  size_t oProbs = p.take<GemmProb>(max_items);
  const int m_cap = d * chi_cap;
  size_t oPerm = p.take<int32_t>(max_items * m_cap);
  size_t oS2 = p.take<double>(max_items * m_cap);
  size_t oUnc = p.take<int32_t>(8);
  size_t oRow = p.take<int32_t>(max_items * m_cap);
  size_t oNrm = p.take<double>(max_items * m_cap);
  size_t oTiles = p.take<int32_t>(max_items + 1);   // tile lists of the fixed-grid launches
  // warm start of the Jacobi: per item A = Lambda_l B_b and its panels' T
  const bool warm = h->warm_start && !u1 && !eig_slots && d * chi_cap > 64;
  size_t oWarmA = 0, oWarmT = 0;
  if (warm) {
    oWarmA = p.take<double2>(max_items * warm_a_elems(d, chi_cap));
    oWarmT = p.take<double2>(max_items * warm_t_elems(chi_cap));
  }
  // Krylov propagation: identity propagator, one propagator per chain, a job
  // per item, rho partials and Krylov histories per item of a layer
  const int kt_nblk = 32;
  const size_t kt_hist = kry ? (size_t)2 * (kry->n_max + 1) * dd * dd : 0;
  size_t oKId = 0, oKG = 0, oKJobs = 0, oKPart = 0, oKHist = 0;
  if (kry) {
    oKId = p.take<double2>((size_t)dd * dd);
    oKG = p.take<double2>((size_t)n_chains * dd * dd);
    oKJobs = p.take<KryJob>((n_par[0] + n_par[1]) * 2);
    oKPart = p.take<double2>((size_t)n_chains * kt_nblk * dd * dd);
    oKHist = p.take<double2>((size_t)n_chains * kt_hist);
  }
  size_t oU1 = 0, oU1Items = 0;
  if (u1) {
    // the device block plan holds a bond's row and column charges in LDS and
    // lists every charge block of a layer among n_items * d chi_max slots
    if (d * chi_cap > 2048)
      return mps_fail(h, MPS_ERR_CAPACITY, "charge-carrying chains need d*chi_max <= 2048");
    if ((int64_t)max_items * d * chi_cap > kSchedCap)
      return mps_fail(h, MPS_ERR_CAPACITY, "charge-carrying layers need bonds * d*chi_max <= 65536");
    oU1 = p.take<char>(u1_layer_bytes((int)max_items, d * chi_cap, chi_cap));
    oU1Items = p.take<U1Item>((n_par[0] + n_par[1]) * (order == 0 ? 2 : n_cls));
  }
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;

  // gates: G[chain][class][bond]
  std::vector<GateJob> jobs;
  jobs.reserve(n_jobs);
  std::vector<size_t> gate_base(n_chains);
  size_t goff = 0;
  for (int c = 0; c < n_chains; ++c) {
    gate_base[c] = goff;
    for (int k = 0; k < n_cls; ++k)
      for (int b = 0; b < chains[c].L - 1; ++b) {
        GateJob j;
        j.h = (const double2*)chains[c].hbond + (size_t)b * dd * dd;
        j.G64 = c128 ? nullptr : (float2*)(ws + oG) + goff;
        j.G128 = c128 ? (double2*)(ws + oG) + goff : nullptr;
        j.tau = taus[k];
        jobs.push_back(j);
        goff += (size_t)dd * dd;
      }
  }
  st = upload(h, s, ws + oJobs, jobs);
  if (st != MPS_OK) return st;
  PROF_LAUNCH(h, s, MPS_K_GATES, launch_gates(s, (const GateJob*)(ws + oJobs), (int)jobs.size(), dd));

  // bond items: for every group a contiguous array.  Groups are (parity,
  // class) for the even/odd orders and single sweep layers for order 0.
  const int n_groups = order == 0 ? (int)layers.size() : 2 * n_cls;
  std::vector<BondItem> items;
  std::vector<int> item_chain;
  std::vector<KryJob> kjobs;
  std::vector<size_t> start(n_groups), count(n_groups);
  for (int gi = 0; gi < n_groups; ++gi) {
    {
      const int par = order == 0 ? 0 : gi / n_cls, k = order == 0 ? 0 : gi % n_cls;
      start[gi] = items.size();
      char* slot = ws + oSlots;
      for (int c = 0; c < n_chains; ++c) {
        const mps_chain_desc& ch = chains[c];
        const size_t site = (size_t)ch.chi_max * ch.d * ch.chi_max;
        const size_t sq = (size_t)ch.d * ch.chi_max * ch.d * ch.chi_max;
        std::vector<int> bl;
        if (order == 0) {
          const int j = gi < l_max - 1 ? gi : gi - (l_max - 1);
          if (j < ch.L - 1) bl.push_back(gi < l_max - 1 ? j : ch.L - 2 - j);
        } else {
          for (int b = par; b < ch.L - 1; b += 2) bl.push_back(b);
        }
        for (int b : bl) {
          BondItem it;
          it.Bl = (char*)ch.B + (size_t)b * site * esz;
          it.Br = (char*)ch.B + (size_t)(b + 1) * site * esz;
          it.lam_l = ch.lam + (size_t)b * ch.chi_max;
          it.lam_m = ch.lam + (size_t)(b + 1) * ch.chi_max;
          it.chi = ch.chi;
          it.G = (const char*)(ws + oG) + (gate_base[c] + ((size_t)k * (ch.L - 1) + b) * dd * dd) * esz;
          if (kry) {
            const size_t li = items.size() - start[gi];   // position inside the layer
            KryJob kj;
            std::memset(&kj, 0, sizeof(kj));
            kj.h = (const double2*)ch.hbond + (size_t)b * dd * dd;
            kj.part = (double2*)(ws + oKPart) + li * kt_nblk * dd * dd;
            kj.hist = (double2*)(ws + oKHist) + li * kt_hist;
            kj.G = ws + oKG + (size_t)c * dd * dd * esz;
            kj.n_used = kry->n_used_dev ? kry->n_used_dev + (size_t)c * 2 * (l_max - 1) + gi : nullptr;
            kjobs.push_back(kj);
            it.G = kj.G;
          }
          it.disc = ch.disc;
          it.X = (double2*)slot;
          slot += (sq * sizeof(double2) + 255) & ~size_t(255);
          it.T = slot;
          slot += (sq * esz + 255) & ~size_t(255);
          it.Vh = slot;
          slot += ((size_t)ch.chi_max * ch.d * ch.chi_max * esz + 255) & ~size_t(255);
          it.gram = nullptr;
          it.urows = nullptr;
          if (eig_slots) {
            it.gram = (double2*)slot;
            slot += (sq * sizeof(double2) + 255) & ~size_t(255);
            it.urows = (double2*)slot;
            slot += (sq * sizeof(double2) + 255) & ~size_t(255);
          }
          it.b = b;
          it.d = ch.d;
          it.chi_max = ch.chi_max;
          it.pad = c * (l_max - 1) + b;   // the update's offset in a layer's log slice
          items.push_back(it);
          item_chain.push_back(c);
        }
      }
      count[gi] = items.size() - start[gi];
    }
  }
  st = upload(h, s, ws + oItems, items);
  if (st != MPS_OK) return st;
  if (u1) {
    // the charges of every item, beside the items
    std::vector<U1Item> uitems(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
      const mps_u1_chain& q = u1[item_chain[i]];
      uitems[i].qb = q.qbond;
      uitems[i].modulus = q.modulus;
      for (int t = 0; t < 5; ++t) uitems[i].qsite[t] = t < d ? q.qsite[t] : 0;
    }
    st = upload(h, s, ws + oU1Items, uitems);
    if (st != MPS_OK) return st;
  }
  if (kry) {
    st = upload(h, s, ws + oKJobs, kjobs);
    if (st != MPS_OK) return st;
    MPS_TRY_HIP(h, launch_ktebd_identity(s, ws + oKId, dd, c128));
  }
  KryJob* dJobs = (KryJob*)(ws + oKJobs);

  BondItem* dItems = (BondItem*)(ws + oItems);
  JacMat* mats = (JacMat*)(ws + oMats);
  SelOut* sel = (SelOut*)(ws + oSel);
  GemmProb* probs = (GemmProb*)(ws + oProbs);
  int32_t* perm = (int32_t*)(ws + oPerm);
  double* s2 = (double*)(ws + oS2);
  int32_t* unconv = (int32_t*)(ws + oUnc);
  const int nb_cap = jac_nb(m_cap);
  // device step counter of the discarded-weight log (bytes 192.. of the status block)
  int32_t* log_step = (int32_t*)((char*)h->status_dev + 192);
  if (disc_log || obs_log) MPS_TRY_HIP(h, launch_set_int(s, log_step, 0));
  if (checkpoint) {
    CkptHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    hd.magic = kCkptMagic;
    hd.n_chains = n_chains;
    hd.n_steps = n_steps;
    hd.order = order;
    hd.dt = dt;
    hd.eps_local = eps_local;
    hd.shape_sum = ckpt_shape_sum(chains, n_chains);
    MPS_TRY_HIP(h, hipMemcpyAsync(ckpt, &hd, sizeof(hd), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
  }
  auto save_all = [&](int stp) -> mps_status {
    for (int c = 0; c < n_chains; ++c) {
      mps_status r = grad_ckpt_save(h, s, chains[c], (char*)ckpt + ckpt_block_offset(chains, c, n_steps), n_steps,
                                    stp);
      if (r != MPS_OK) return r;
    }
    return MPS_OK;
  };

  auto run_step = [&]() -> mps_status {
    for (int li = 0; li < (int)layers.size(); ++li) {
      if (li < lo || li >= hi) continue;
      const auto& ly = layers[li];
      const int idx = order == 0 ? ly.first : ly.first * n_cls + ly.second;
      const int n_layer = (int)count[idx];
      if (n_layer == 0) continue;
      // plain form: one bond per launch sequence; else the whole layer at once
      for (int i0 = 0; i0 < n_layer; i0 += plain ? 1 : n_layer) {
      const int n = plain ? 1 : n_layer;
      BondItem* it = dItems + start[idx] + i0;
      const bool prof = h->profile;
      unsigned long long* stats = prof ? h->stats_dev : nullptr;
      // grid bounds: the capacity when the host may not synchronise, else the
      // layer's actual largest bond dimensions (one small readback)
      int chi_eff = chi_cap, chl_eff = chi_cap;
      if (!fixed) {
        MPS_TRY_HIP(h, launch_layer_dims(s, it, n, unconv + 2));
        MPS_TRY_HIP(h, hipMemcpyAsync(h->host_pinned + 2, unconv + 2, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MPS_TRY_HIP(h, hipStreamSynchronize(s));
        chl_eff = std::min(chi_cap, (int)h->host_pinned[2]);
        chi_eff = std::min(chi_cap, std::max(h->host_pinned[2], h->host_pinned[3]));
      }
      const int k_cap = std::min(chi_cap, d * chi_eff);  // kept count <= min(d chi_l, d chi_r)
      if (kry) {
        // theta' with the identity, its reduced matrix, the local Lanczos
        // propagator of the bond term into the item's gate
        KryJob* kj = dJobs + start[idx] + i0;
        if (prof) prof_begin(h, s, MPS_K_KRYLOV);
        MPS_TRY_HIP(h, launch_theta(s, it, n, d, chi_eff, c128, nullptr, ws + oKId));
        MPS_TRY_HIP(h, launch_ktebd_rho(s, it, kj, n, d, kt_nblk));
        MPS_TRY_HIP(h, launch_ktebd_krylov(s, kj, n, d, kt_nblk, kry->n_max, kry->tol, taus[0], c128, h->status_dev));
        if (prof) prof_end(h, s, MPS_K_KRYLOV);
      }
      if (prof) prof_begin(h, s, MPS_K_THETA);
      // without host synchronisation the bond dimensions are only known on the
      // device: the theta and write-back GEMM launches walk lists of real tiles
      int32_t* tiles = fixed ? (int32_t*)(ws + oTiles) : nullptr;
      MPS_TRY_HIP(h, launch_theta(s, it, n, d, chi_eff, c128, stats, nullptr, tiles));
      if (prof) prof_end(h, s, MPS_K_THETA);
      if (u1) {
        const size_t first = start[idx] + i0;
        mps_status r = u1_layer(h, s, it, (const U1Item*)(ws + oU1Items) + first, n, (int)max_items, m_cap, chi_cap,
                                eps_local, c128, ws + oU1, sel, unconv);
        if (r != MPS_OK) return r;
      } else {
      if (warm) {
        if (prof) prof_begin(h, s, MPS_K_WARM);
        MPS_TRY_HIP(h, launch_warm_start(s, it, n, d, chi_cap, chi_eff, c128, (double2*)(ws + oWarmA),
                                         (double2*)(ws + oWarmT)));
        if (prof) prof_end(h, s, MPS_K_WARM);
      }
      if (prof) prof_begin(h, s, MPS_K_PREP);
      MPS_TRY_HIP(h, launch_jac_prep_bonds(s, it, mats, n, kJacBlock, (int32_t*)(ws + oRow), (double*)(ws + oNrm), m_cap,
                                           h->status_dev, stats));
      if (prof) prof_end(h, s, MPS_K_PREP);
      mps_status r = MPS_OK;
      if (eig_slots && nb_cap > 2) {
        // the eigendecomposition split at any size: Gram on MFMA, the
        // one-sided Jacobi on its rows with the smallest absolute tolerance,
        // rows normalised, W = U^dag theta' on MFMA
        MPS_TRY_HIP(h, launch_eig_gram(s, it, mats, n, probs, m_cap, tiles, h->status_dev));
        const double abs_saved = h->jac_abs;
        const int meth_saved = h->split_method;
        h->jac_abs = kJacAbsFloor;
        h->split_method = 0;
        r = run_jacobi(h, s, mats, n, nb_cap, m_cap, unconv, fixed);
        h->jac_abs = abs_saved;
        h->split_method = meth_saved;
        if (r != MPS_OK) return r;
        MPS_TRY_HIP(h, launch_eig_rows(s, it, mats, n, probs, m_cap, m_cap, kJacAbsFloor));
      } else {
        r = run_jacobi(h, s, mats, n, nb_cap, m_cap, unconv, fixed);
        if (r != MPS_OK) return r;
      }
      if (prof) prof_begin(h, s, MPS_K_SELECT);
      MPS_TRY_HIP(h, launch_select(s, mats, n, perm, s2, m_cap, chi_cap, count_rule_eps(h, eps_local), sel));
      if (prof) prof_end(h, s, MPS_K_SELECT);
      if (prof) prof_begin(h, s, MPS_K_WB_RIGHT);
      DiscLog lg;
      if (disc_log) {
        lg.log = disc_log;
        lg.step = log_step;
        lg.step_stride = (long long)layers.size() * n_chains * (l_max - 1);
        lg.layer_off = (long long)li * n_chains * (l_max - 1);
      }
      MPS_TRY_HIP(h, launch_wb_right(s, it, n, mats, perm, s2, m_cap, sel, chi_eff, d, c128, lg));
      if (prof) prof_end(h, s, MPS_K_WB_RIGHT);
      }
      MPS_TRY_HIP(h, launch_wb_left_probs(s, it, n, sel, probs));
      if (prof) prof_begin(h, s, MPS_K_GEMM);
      MPS_TRY_HIP(h, launch_gemm_bt_conj(s, probs, n, d * chl_eff, k_cap, c128, stats, tiles));
      if (prof) prof_end(h, s, MPS_K_GEMM);
      if (prof) {
        mps_status ps = prof_harvest(h, s);
        if (ps != MPS_OK) return ps;
      }
      }
    }
    if (obs_log)
      for (int c = 0; c < n_chains; ++c)
        MPS_TRY_HIP(h, launch_observe_log(s, chains[c], (const double2*)obs_op, obs_log + (size_t)c * l_max, log_step,
                                          (long long)n_chains * l_max));
    if (disc_log || obs_log) MPS_TRY_HIP(h, launch_inc_int(s, log_step));
    return MPS_OK;
  };

  if (!graph) {
    for (int stp = 0; stp < n_steps; ++stp) {
      if (checkpoint && (st = save_all(stp)) != MPS_OK) return st;
      st = run_step();
      if (st != MPS_OK) return st;
    }
    if (checkpoint && (st = save_all(n_steps)) != MPS_OK) return st;
    return MPS_OK;
  }
  // Everything one step's launches depend on: the workspace and its plan, the
  // chains, the schedule, the count rule and the solver options.  The gates
  // and the bond items were rewritten into the workspace above, so a step
  // captured with the same key replays unchanged.
  std::vector<uint64_t> key;
  auto put = [&](uint64_t v) { key.push_back(v); };
  auto bits = [](double x) {
    uint64_t u;
    std::memcpy(&u, &x, sizeof(u));
    return u;
  };
  put((uint64_t)(uintptr_t)ws);
  put(p.off);
  put((uint64_t)n_chains);
  put((uint64_t)order);
  put(flags);
  put(bits(dt));
  put(bits(eps_local));
  put((uint64_t)(uintptr_t)disc_log);
  put((uint64_t)(uintptr_t)obs_op);
  put((uint64_t)(uintptr_t)obs_log);
  put(kry ? (uint64_t)kry->n_max : 0);
  put(kry ? bits(kry->tol) : 0);
  put(kry ? (uint64_t)(uintptr_t)kry->n_used_dev : 0);
  put(bits(h->jac_tol));
  put(bits(h->jac_abs));
  put((uint64_t)h->jac_max_sweeps);
  put((uint64_t)h->jac_inner_sweeps);
  put((uint64_t)h->jac_threads);
  put((uint64_t)h->jac_split_below);
  put((uint64_t)h->split_method);
  put((uint64_t)h->jac_persistent);
  put((uint64_t)h->warm_start);
  put((uint64_t)h->jac_spin_limit);
  put(u1 ? 1 : 0);
  for (int c = 0; c < n_chains; ++c) {
    const mps_chain_desc& ch = chains[c];
    put(((uint64_t)(uint32_t)ch.L << 32) | (uint32_t)ch.d);
    put(((uint64_t)(uint32_t)ch.chi_max << 32) | (uint32_t)ch.dtype);
    put((uint64_t)(uintptr_t)ch.B);
    put((uint64_t)(uintptr_t)ch.lam);
    put((uint64_t)(uintptr_t)ch.chi);
    put((uint64_t)(uintptr_t)ch.hbond);
    put((uint64_t)(uintptr_t)ch.disc);
  }
  if (!h->graph_exec || key != h->graph_key) {
    if (h->graph_exec) {
      MPS_TRY_HIP(h, hipStreamSynchronize(s));
      hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
    if (h->graph) {
      hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
    h->graph_key.clear();
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    MPS_TRY_HIP(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = run_step();
    hipError_t ec = hipStreamEndCapture(s, &g);
    if (st != MPS_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) return mps_fail(h, MPS_ERR_HIP, std::string("capture: ") + hipGetErrorString(ec));
    hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      hipGraphDestroy(g);
      return mps_fail(h, MPS_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(ei));
    }
    h->graph = g;
    h->graph_exec = ge;
    h->graph_key = key;
  }
  for (int stp = 0; stp < n_steps; ++stp) {
    hipError_t el = hipGraphLaunch(h->graph_exec, s);
    if (el != hipSuccess) return mps_fail(h, MPS_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(el));
  }
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  return MPS_OK;
}


