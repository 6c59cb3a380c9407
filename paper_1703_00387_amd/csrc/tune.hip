// Autotuner for the launch configuration of the FP64 Jacobi split.
//
// For a shape bucket (n_mats matrices of m x n, the layer of a batched step)
// every candidate configuration runs the whole split (preparation, Jacobi
// sweeps, selection) on the same synthetic matrices, timed with HIP events on
// the call's stream after one untimed run.  Candidates: 256 or 512 threads per
// round workgroup, the column split off / default / extended (pairs below 0,
// 32, 128), and, for single-panel matrices (m <= 64), the one-sided Jacobi or
// the eigendecomposition split.  The synthetic matrices have graded rows
// (scale exp(-4 r / m)) and pseudo-random entries from a counter hash, so the
// sweep counts resemble those of TEBD matrices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "mfma_tile.h"

namespace {

__device__ __forceinline__ double tune_hash(unsigned long long x) {
  // SplitMix64 finaliser, mapped to [-1, 1)
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void tune_fill_kernel(double2* X, long long per_mat, int m, int n, int n_mats) {
  const long long total = per_mat * n_mats;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long within = e % per_mat;
    const int r = (int)(within / n);
    const double sc = exp(-4.0 * r / m);
    X[e] = make_double2(sc * tune_hash(2 * (unsigned long long)e), sc * tune_hash(2 * (unsigned long long)e + 1));
  }
}

struct Candidate {
  int threads, split_below, method;
};

}  // namespace

extern "C" mps_status mps_autotune_jacobi(mps_handle h, mps_stream stream, int32_t n_mats, int32_t m, int32_t n,
                                          int32_t apply, double* times_ms, int32_t* n_candidates, int32_t* best) {
  if (!h) return MPS_ERR_INVALID;
  if (!times_ms || !n_candidates || !best) return mps_fail(h, MPS_ERR_INVALID, "null output");
  if (n_mats < 1 || m < 1 || n < 1) return mps_fail(h, MPS_ERR_SHAPE, "bad shape");
  if (m > 4096 || n > 4096 || n_mats > 1024) return mps_fail(h, MPS_ERR_CAPACITY, "m, n <= 4096, n_mats <= 1024");
  std::vector<Candidate> cands;
  for (int t : {256, 512})
    for (int sb : {0, 32, 128})
      for (int meth = 0; meth < (m <= 64 ? 2 : 1); ++meth) cands.push_back({t, sb, meth});
  if ((int)cands.size() > *n_candidates) return mps_fail(h, MPS_ERR_CAPACITY, "times_ms too short");
  hipStream_t s = (hipStream_t)stream;
  const long long per_mat = (long long)m * n;
  WsPlan p;
  size_t oX = p.take<double2>((size_t)per_mat * n_mats);
  size_t oM = p.take<JacMat>(n_mats);
  size_t oR = p.take<int32_t>((size_t)n_mats * m);
  size_t oN = p.take<double>((size_t)n_mats * m);
  size_t oP = p.take<int32_t>((size_t)n_mats * m);
  size_t oS = p.take<double>((size_t)n_mats * m);
  size_t oSel = p.take<SelOut>(n_mats);
  size_t oU = p.take<int32_t>(8);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  std::vector<JacMat> hm(n_mats);
  for (int i = 0; i < n_mats; ++i) {
    std::memset(&hm[i], 0, sizeof(JacMat));
    hm[i].X = (double2*)(ws + oX) + (size_t)i * per_mat;
    hm[i].rowmap = (int32_t*)(ws + oR) + (size_t)i * m;
    hm[i].nrm2 = (double*)(ws + oN) + (size_t)i * m;
    hm[i].m = m;
    hm[i].n = n;
    hm[i].ld = n;
    hm[i].nb = jac_nb(m);
    hm[i].kmax = std::min(m, n);
  }
  const Candidate saved{h->jac_threads, h->jac_split_below, h->split_method};
  hipEvent_t e0, e1;
  MPS_TRY_HIP(h, hipEventCreate(&e0));
  MPS_TRY_HIP(h, hipEventCreate(&e1));
  int best_i = -1;
  double best_ms = 1e300;
  st = MPS_OK;
  for (size_t c = 0; c < cands.size() && st == MPS_OK; ++c) {
    h->jac_threads = cands[c].threads;
    h->jac_split_below = cands[c].split_below;
    h->split_method = cands[c].method;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == MPS_OK; ++rep) {
      const int grid = (int)std::min<long long>((per_mat * n_mats + 255) / 256, 4096);
      tune_fill_kernel<<<grid, 256, 0, s>>>((double2*)(ws + oX), per_mat, m, n, n_mats);
      if (hipGetLastError() != hipSuccess) { st = mps_fail(h, MPS_ERR_HIP, "fill launch"); break; }
      if (hipMemcpyAsync(ws + oM, hm.data(), n_mats * sizeof(JacMat), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) { st = mps_fail(h, MPS_ERR_HIP, "descriptor upload"); break; }
      if (hipEventRecord(e0, s) != hipSuccess) { st = mps_fail(h, MPS_ERR_HIP, "event"); break; }
      if (launch_jac_prep_plain(s, (JacMat*)(ws + oM), n_mats, h->status_dev) != hipSuccess) {
        st = mps_fail(h, MPS_ERR_HIP, "prep launch");
        break;
      }
      st = run_jacobi(h, s, (JacMat*)(ws + oM), n_mats, jac_nb(m), m, (int32_t*)(ws + oU), false);
      if (st != MPS_OK) break;
      if (launch_select(s, (JacMat*)(ws + oM), n_mats, (int32_t*)(ws + oP), (double*)(ws + oS), m,
                        std::min(m, n), 1e-12, (SelOut*)(ws + oSel)) != hipSuccess) {
        st = mps_fail(h, MPS_ERR_HIP, "select launch");
        break;
      }
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = mps_fail(h, MPS_ERR_HIP, "timing"); break; }
    }
    times_ms[c] = ms;
    if (st == MPS_OK && ms < best_ms) {
      best_ms = ms;
      best_i = (int)c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != MPS_OK || best_i < 0 || !apply) {
    h->jac_threads = saved.threads;
    h->jac_split_below = saved.split_below;
    h->split_method = saved.method;
  } else {
    h->jac_threads = cands[best_i].threads;
    h->jac_split_below = cands[best_i].split_below;
    h->split_method = cands[best_i].method;
  }
  if (st != MPS_OK) return st;
  *n_candidates = (int)cands.size();
  *best = best_i;
  return MPS_OK;
}

extern "C" mps_status mps_autotune_candidate(int32_t m, int32_t index, int32_t* threads, int32_t* split_below,
                                             int32_t* method) {
  if (!threads || !split_below || !method || m < 1) return MPS_ERR_INVALID;
  int i = 0;
  for (int t : {256, 512})
    for (int sb : {0, 32, 128})
      for (int meth = 0; meth < (m <= 64 ? 2 : 1); ++meth, ++i)
        if (i == index) {
          *threads = t;
          *split_below = sb;
          *method = meth;
          return MPS_OK;
        }
  return MPS_ERR_INVALID;
}

// ---------------------------------------------------------------------------
// Tile shapes of the MFMA GEMMs
// ---------------------------------------------------------------------------
namespace {

template <class T>
__global__ void tune_fill_c_kernel(T* X, long long n, unsigned long long seed) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    T v;
    v.x = tune_hash(seed + 2 * (unsigned long long)e);
    v.y = tune_hash(seed + 2 * (unsigned long long)e + 1);
    X[e] = v;
  }
}

}  // namespace

extern "C" mps_status mps_autotune_gemm(mps_handle h, mps_stream stream, int32_t kind, int32_t dtype, int32_t batch,
                                        int32_t M, int32_t N, int32_t K, int32_t apply, double* times_ms,
                                        int32_t* n_candidates, int32_t* best) {
  if (!h) return MPS_ERR_INVALID;
  if (!times_ms || !n_candidates || !best) return mps_fail(h, MPS_ERR_INVALID, "null output");
  if (kind != 0 && kind != 1) return mps_fail(h, MPS_ERR_INVALID, "kind must be 0 (strided) or 1 (batched)");
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "dtype must be MPS_C64 or MPS_C128");
  if (M < 1 || N < 1 || K < 1 || batch < 1 || (kind == 0 && batch != 1))
    return mps_fail(h, MPS_ERR_SHAPE, "bad shape (the strided kind takes batch = 1)");
  if ((long long)M * K > (1LL << 26) || (long long)N * K > (1LL << 26) || (long long)M * N > (1LL << 26) ||
      batch > 4096)
    return mps_fail(h, MPS_ERR_CAPACITY, "operands are limited to 2^26 elements, batch to 4096");
  if (*n_candidates < kGemmCands) return mps_fail(h, MPS_ERR_CAPACITY, "times_ms too short");
  const bool c128 = dtype == MPS_C128;
  const size_t es = c128 ? sizeof(double2) : sizeof(float2);
  hipStream_t s = (hipStream_t)stream;
  WsPlan p;
  const size_t oA = p.take<char>((size_t)batch * M * K * es), oB = p.take<char>((size_t)batch * N * K * es),
               oC = p.take<char>((size_t)batch * M * N * es), oP = p.take<GemmProb>(batch);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  const int g = 1024;
  if (c128) {
    tune_fill_c_kernel<double2><<<g, 256, 0, s>>>((double2*)(ws + oA), (long long)batch * M * K, 11);
    tune_fill_c_kernel<double2><<<g, 256, 0, s>>>((double2*)(ws + oB), (long long)batch * N * K, 1u << 30);
  } else {
    tune_fill_c_kernel<float2><<<g, 256, 0, s>>>((float2*)(ws + oA), (long long)batch * M * K, 11);
    tune_fill_c_kernel<float2><<<g, 256, 0, s>>>((float2*)(ws + oB), (long long)batch * N * K, 1u << 30);
  }
  MPS_TRY_HIP(h, hipGetLastError());
  SGemm sg;
  std::memset(&sg, 0, sizeof(sg));
  if (kind == 0) {
    // C = A B with A [M][K], B [K][N] row-major (the H_eff stage form)
    sg.A = ws + oA; sg.rsA = K; sg.csA = 1;
    sg.B = ws + oB; sg.rsB = N; sg.csB = 1;
    sg.C = ws + oC; sg.rsC = N; sg.csC = 1;
    sg.M = M; sg.N = N; sg.K = K; sg.alpha = 1.0;
  } else {
    // C_i = A_i B_i^dag, the write-back form, batch problems
    std::vector<GemmProb> pr(batch);
    for (int i = 0; i < batch; ++i) {
      GemmProb& q = pr[i];
      std::memset(&q, 0, sizeof(q));
      q.A = ws + oA + (size_t)i * M * K * es;
      q.B = ws + oB + (size_t)i * N * K * es;
      q.C = ws + oC + (size_t)i * M * N * es;
      q.M = M; q.N = N; q.K = K;
      q.lda = K; q.ldb = K; q.ldc = N;
      q.alpha = 1.0;
    }
    MPS_TRY_HIP(h, hipMemcpyAsync(ws + oP, pr.data(), batch * sizeof(GemmProb), hipMemcpyHostToDevice, s));
  }
  hipEvent_t e0, e1;
  MPS_TRY_HIP(h, hipEventCreate(&e0));
  MPS_TRY_HIP(h, hipEventCreate(&e1));
  auto run = [&](int c) -> hipError_t {
    return kind == 0 ? launch_sgemm_cand(s, sg, c128, c)
                     : launch_gemm_bt_conj_cand(s, (const GemmProb*)(ws + oP), batch, M, N, c128, nullptr, nullptr, c);
  };
  int best_i = -1;
  double best_ms = 1e300;
  hipError_t he = hipSuccess;
  for (int c = 0; c < kGemmCands && he == hipSuccess; ++c) {
    he = run(c);   // untimed
    const int reps = 5;
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int r = 0; r < reps && he == hipSuccess; ++r) he = run(c);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    times_ms[c] = ms / reps;
    if (he == hipSuccess && times_ms[c] < best_ms) {
      best_ms = times_ms[c];
      best_i = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (he != hipSuccess) return mps_fail(h, MPS_ERR_HIP, std::string("gemm tuning: ") + hipGetErrorString(he));
  if (apply) {
    const int cls = gemm_shape_class(M, N);
    if (kind == 0) set_sgemm_choice(c128, cls, best_i);
    else set_bgemm_choice(c128, cls, best_i);
  }
  *n_candidates = kGemmCands;
  *best = best_i;
  return MPS_OK;
}

extern "C" mps_status mps_gemm_candidate(int32_t index, int32_t* tile_m, int32_t* tile_n) {
  if (!tile_m || !tile_n || index < 0 || index >= kGemmCands) return MPS_ERR_INVALID;
  *tile_m = 32 * gemm_cand_mi(index);
  *tile_n = 32 * gemm_cand_nj(index);
  return MPS_OK;
}

extern "C" mps_status mps_gemm_tile_choice(int32_t kind, int32_t dtype, int32_t M, int32_t N, int32_t* index) {
  if (!index || (kind != 0 && kind != 1) || (dtype != MPS_C64 && dtype != MPS_C128) || M < 1 || N < 1)
    return MPS_ERR_INVALID;
  const int cls = gemm_shape_class(M, N);
  *index = kind == 0 ? get_sgemm_choice(dtype == MPS_C128, cls) : get_bgemm_choice(dtype == MPS_C128, cls);
  return MPS_OK;
}

extern "C" mps_status mps_set_gemm_tile(int32_t kind, int32_t dtype, int32_t M, int32_t N, int32_t index) {
  if ((kind != 0 && kind != 1) || (dtype != MPS_C64 && dtype != MPS_C128) || M < 1 || N < 1 || index < 0 ||
      index >= kGemmCands)
    return MPS_ERR_INVALID;
  const int cls = gemm_shape_class(M, N);
  if (kind == 0) set_sgemm_choice(dtype == MPS_C128, cls, index);
  else set_bgemm_choice(dtype == MPS_C128, cls, index);
  return MPS_OK;
}
