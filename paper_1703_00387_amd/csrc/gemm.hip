// Batched complex GEMM on MFMA (complex64: FP32 MFMA with FP32 accumulation;
// complex128: FP64 MFMA with FP64 accumulation):
//   C = alpha * A * op(B),  A row-major [M][lda],
//   op(B) = B (row-major [K][ldb])            for the NN variant,
//   op(B) = B^dag (B row-major [N][ldb])      for the BT-conj variant.
// Used for the Hastings write-back B_b = theta~' V_k / |s_k| (Sec. "Basic
// concepts", Splitting).  Each problem of the batch reads its own dimensions
// (possibly written by an earlier kernel on the device); either the grid is
// sized for the capacity and tiles beyond a problem's dimensions return at
// once, or a fixed grid walks a device-built list of the real tiles.  The
// workgroup tile is (32 MI) x (32 NJ), chosen per precision and shape class
// from the table the autotuner fills (64 x 64 until then); a complex product
// is three real MFMA products (mfma_3m.h).
#include <algorithm>

#include "mfma_3m.h"

__device__ __forceinline__ int gemm_dim_m(const GemmProb& P) { return P.M_dev ? P.M_mul * *P.M_dev : P.M; }
__device__ __forceinline__ int gemm_dim_n(const GemmProb& P) { return P.N_dev ? P.N_mul * *P.N_dev : P.N; }

template <class T, int MI, int NJ>
struct BGemmLds {
  static constexpr int BM = 32 * MI, BN = 32 * NJ, LDA = BM + 4, LDB = BN + 4;
  static constexpr int kElems = TBK * (LDA + LDB);
};

// One output tile (tm, tn) of problem P; a tile past its dimensions returns.
template <class T, bool BT, int MI, int NJ>
__device__ __forceinline__ void gemm_tile(const GemmProb& P, int tm, int tn, unsigned long long* stats, T* stage) {
  typedef BGemmLds<T, MI, NJ> Ly;
  constexpr int BM = Ly::BM, BN = Ly::BN, LDA = Ly::LDA, LDB = Ly::LDB;
  constexpr int PA = BM >= 64 ? BM / 64 : 1, PB = BN >= 64 ? BN / 64 : 1;
  const int M = gemm_dim_m(P);
  const int N = gemm_dim_n(P);
  const int K = P.K_dev ? P.K_mul * *P.K_dev : P.K;
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * MI * 16, wn = (wave & 1) * NJ * 16;
  if (tid == 0 && stats)
    atomicAdd(&stats[3], 8ull * (unsigned long long)min(BM, M - m0) * min(BN, N - n0) * K);
  const T* PA_ = (const T*)P.A;
  const T* PB_ = (const T*)P.B;
  T* PC = (T*)P.C;
  T* As = stage;
  T* Bs = stage + TBK * LDA;
  Acc3<T, MI, NJ> acc;
  acc3_zero<T, MI, NJ>(acc);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    {
      const int i0 = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < PA; ++q) {
        const int i = i0 + 64 * q;
        if (i < BM) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int k = k0 + kq + e;
            T v = Cx<T>::make(0.0, 0.0);
            if (m0 + i < M && k < K) v = PA_[(size_t)(m0 + i) * P.lda + k];
            As[(kq + e) * LDA + i] = v;
          }
        }
      }
    }
    if (BT) {
      // element (k, j) = conj(B[n0+j][k0+k]); a thread loads 4 consecutive k of one j
      const int j0 = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int j = j0 + 64 * q;
        if (j < BN) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int k = k0 + kq + e;
            T v = Cx<T>::make(0.0, 0.0);
            if (n0 + j < N && k < K) {
              v = PB_[(size_t)(n0 + j) * P.ldb + k];
              v.y = -v.y;
            }
            Bs[(kq + e) * LDB + j] = v;
          }
        }
      }
    } else {
      const int k = tid >> 4, jq = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < PB; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = jq + 64 * q + e;
          if (j < BN) {
            T v = Cx<T>::make(0.0, 0.0);
            if (n0 + j < N && k0 + k < K) v = PB_[(size_t)(k0 + k) * P.ldb + n0 + j];
            Bs[k * LDB + j] = v;
          }
        }
      }
    }
    __syncthreads();
    mma3_chunk<T, MI, NJ>(As, LDA, Bs, LDB, acc, wm, wn, lane);
    __syncthreads();
  }
  typedef typename Cx<T>::R R;
  const R alpha = (R)(P.inv_alpha_dev ? 1.0 / *P.inv_alpha_dev : P.alpha);
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm + i * 16 + Cx<T>::acc_row(lane, r);
        int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          T v = acc3_get<T, MI, NJ>(acc, i, j, r);
          v.x *= alpha;
          v.y *= alpha;
          PC[(size_t)row * P.ldc + col] = v;
        }
      }
}

// 1-D grid over the capacity tiles of all problems, each problem on one XCD
// (tile row-major within it).
template <class T, bool BT, int MI, int NJ>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmProb* __restrict__ probs, int n_probs, int ntn_cap,
                                                   int tiles_cap, unsigned long long* stats) {
  __shared__ T stage[BGemmLds<T, MI, NJ>::kElems];
  int item, tile;
  if (!xcd_item_tile(blockIdx.x, n_probs, tiles_cap, item, tile)) return;
  const GemmProb P = probs[item];
  gemm_tile<T, BT, MI, NJ>(P, tile / ntn_cap, tile % ntn_cap, stats, stage);
}

// offs[i] = output tiles (BM x BN) of the problems before i (dimensions read on
// the device), offs[n] = total; one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void gemm_tile_offsets_kernel(const GemmProb* __restrict__ probs, int n, int BM,
                                                                 int BN, int32_t* offs) {
  __shared__ int part[1024];
  const int per = (n + 1023) / 1024;
  const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
  auto count = [&](int i) {
    const GemmProb& P = probs[i];
    return ((gemm_dim_m(P) + BM - 1) / BM) * ((gemm_dim_n(P) + BN - 1) / BN);
  };
  int sum = 0;
  for (int i = i0; i < i1; ++i) sum += count(i);
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int i = i0; i < i1; ++i) {
    offs[i] = run;
    run += count(i);
  }
  if (threadIdx.x == 1023) offs[n] = part[1023];
}

// A fixed grid walking the list of real tiles.
template <class T, bool BT, int MI, int NJ>
__global__ __launch_bounds__(256) void gemm_list_kernel(const GemmProb* __restrict__ probs, int n,
                                                        const int32_t* __restrict__ offs,
                                                        unsigned long long* stats) {
  __shared__ T stage[BGemmLds<T, MI, NJ>::kElems];
  const int total = offs[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n - 1;   // the last problem whose first tile is <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const GemmProb P = probs[lo];
    const int ntn = (gemm_dim_n(P) + 32 * NJ - 1) / (32 * NJ);
    const int l = t - offs[lo];
    gemm_tile<T, BT, MI, NJ>(P, l / ntn, l % ntn, stats, stage);
    __syncthreads();
  }
}

// Tile shape of the batched GEMM per (precision, shape class of the
// capacity), candidate indices of gemm_cand_mi / gemm_cand_nj.
static int g_bgemm_choice[2][kGemmShapeClasses] = {};

void set_bgemm_choice(bool c128, int shape_class, int cand) { g_bgemm_choice[c128 ? 1 : 0][shape_class] = cand; }
int get_bgemm_choice(bool c128, int shape_class) { return g_bgemm_choice[c128 ? 1 : 0][shape_class]; }

template <class T, bool BT, int MI, int NJ>
static hipError_t bgemm_go(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap,
                           unsigned long long* stats, int32_t* tile_offs) {
  constexpr int BM = 32 * MI, BN = 32 * NJ;
  const int ntm = (M_cap + BM - 1) / BM, ntn = (N_cap + BN - 1) / BN;
  if (tile_offs) {
    gemm_tile_offsets_kernel<<<1, 1024, 0, s>>>(probs, n_probs, BM, BN, tile_offs);
    const int grid = (int)std::min<long long>((long long)ntm * ntn * n_probs, kListGrid);
    gemm_list_kernel<T, BT, MI, NJ><<<grid, 256, 0, s>>>(probs, n_probs, tile_offs, stats);
    return hipGetLastError();
  }
  const int grid = (int)xcd_grid(n_probs, (long long)ntm * ntn);
  gemm_kernel<T, BT, MI, NJ><<<grid, 256, 0, s>>>(probs, n_probs, ntn, ntm * ntn, stats);
  return hipGetLastError();
}

template <class T, bool BT>
static hipError_t bgemm_cand(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap,
                             unsigned long long* stats, int32_t* tile_offs, int cand) {
  switch (cand) {
    case 1: return bgemm_go<T, BT, 4, 2>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
    case 2: return bgemm_go<T, BT, 2, 4>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
    case 3: return bgemm_go<T, BT, 1, 2>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
    case 4: return bgemm_go<T, BT, 2, 1>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
    case 5: return bgemm_go<T, BT, 1, 1>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
    default: return bgemm_go<T, BT, 2, 2>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs);
  }
}

hipError_t launch_gemm_bt_conj_cand(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap,
                                    bool c128, unsigned long long* stats, int32_t* tile_offs, int cand) {
  if (n_probs <= 0) return hipSuccess;
  return c128 ? bgemm_cand<double2, true>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs, cand)
              : bgemm_cand<float2, true>(s, probs, n_probs, M_cap, N_cap, stats, tile_offs, cand);
}

hipError_t launch_gemm_bt_conj(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                               unsigned long long* stats, int32_t* tile_offs) {
  return launch_gemm_bt_conj_cand(s, probs, n_probs, M_cap, N_cap, c128, stats, tile_offs,
                                  get_bgemm_choice(c128, gemm_shape_class(M_cap, N_cap)));
}

hipError_t launch_gemm_nn(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                          unsigned long long* stats) {
  if (n_probs <= 0) return hipSuccess;
  return c128 ? bgemm_cand<double2, false>(s, probs, n_probs, M_cap, N_cap, stats, nullptr, 0)
              : bgemm_cand<float2, false>(s, probs, n_probs, M_cap, N_cap, stats, nullptr, 0);
}
