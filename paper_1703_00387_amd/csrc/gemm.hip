// Batched complex GEMM on MFMA (complex64: FP32 MFMA with FP32 accumulation;
// complex128: FP64 MFMA with FP64 accumulation):
//   C = alpha * A * op(B),  A row-major [M][lda],
//   op(B) = B (row-major [K][ldb])            for the NN variant,
//   op(B) = B^dag (B row-major [N][ldb])      for the BT-conj variant.
// Used for the Hastings write-back B_b = theta~' V_k / |s_k| (Sec. "Basic
// concepts", Splitting) and the stages of the effective-Hamiltonian apply.
// Each problem of the batch reads its own dimensions (possibly written by an
// earlier kernel on the device); the grid is sized for the capacity and tiles
// beyond a problem's dimensions return at once.
#include <algorithm>

#include "mfma_tile.h"

__device__ __forceinline__ int gemm_dim_m(const GemmProb& P) { return P.M_dev ? P.M_mul * *P.M_dev : P.M; }
__device__ __forceinline__ int gemm_dim_n(const GemmProb& P) { return P.N_dev ? P.N_mul * *P.N_dev : P.N; }

// One output tile (tm, tn) of problem P; a tile past its dimensions returns.
template <class T, bool BT>
__device__ __forceinline__ void gemm_tile(const GemmProb& P, int tm, int tn, unsigned long long* stats, T* As,
                                          T* Bs) {
  const int M = gemm_dim_m(P);
  const int N = gemm_dim_n(P);
  const int K = P.K_dev ? P.K_mul * *P.K_dev : P.K;
  const int m0 = tm * TBM, n0 = tn * TBN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  if (tid == 0 && stats)
    atomicAdd(&stats[3], 8ull * (unsigned long long)min(TBM, M - m0) * min(TBN, N - n0) * K);
  const T* PA = (const T*)P.A;
  const T* PB = (const T*)P.B;
  T* PC = (T*)P.C;
  AccTile<T> acc;
  acc_zero<T>(acc);
  for (int k0 = 0; k0 < K; k0 += TBK) {
    {
      int i = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int k = k0 + kq + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (m0 + i < M && k < K) v = PA[(size_t)(m0 + i) * P.lda + k];
        As[(kq + e) * TLD + i] = v;
      }
    }
    if (BT) {
      // element (k, j) = conj(B[n0+j][k0+k]); thread loads 4 consecutive k of one j
      int j = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int k = k0 + kq + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (n0 + j < N && k < K) {
          v = PB[(size_t)(n0 + j) * P.ldb + k];
          v.y = -v.y;
        }
        Bs[(kq + e) * TLD + j] = v;
      }
    } else {
      int k = tid >> 4, jq = (tid & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int j = jq + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (n0 + j < N && k0 + k < K) v = PB[(size_t)(k0 + k) * P.ldb + n0 + j];
        Bs[k * TLD + j] = v;
      }
    }
    __syncthreads();
    mma_chunk<T>(As, Bs, acc, wm, wn, lane);
    __syncthreads();
  }
  typedef typename Cx<T>::R R;
  const R alpha = (R)(P.inv_alpha_dev ? 1.0 / *P.inv_alpha_dev : P.alpha);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm + i * 16 + Cx<T>::acc_row(lane, r);
        int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          T v;
          v.x = alpha * acc.re[i][j][r];
          v.y = alpha * acc.im[i][j][r];
          PC[(size_t)row * P.ldc + col] = v;
        }
      }
}

// Grid over (capacity tiles, problems).
template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmProb* __restrict__ probs, int ntn_cap,
                                                   unsigned long long* stats) {
  __shared__ T As[TBK * TLD];
  __shared__ T Bs[TBK * TLD];
  const GemmProb P = probs[blockIdx.y];
  gemm_tile<T, BT>(P, blockIdx.x / ntn_cap, blockIdx.x % ntn_cap, stats, As, Bs);
}

// offs[i] = output tiles of the problems before i (dimensions read on the
// device), offs[n] = total; one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void gemm_tile_offsets_kernel(const GemmProb* __restrict__ probs, int n,
                                                                 int32_t* offs) {
  __shared__ int part[1024];
  const int per = (n + 1023) / 1024;
  const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
  auto count = [&](int i) {
    const GemmProb& P = probs[i];
    return ((gemm_dim_m(P) + TBM - 1) / TBM) * ((gemm_dim_n(P) + TBN - 1) / TBN);
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
template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_list_kernel(const GemmProb* __restrict__ probs, int n,
                                                        const int32_t* __restrict__ offs,
                                                        unsigned long long* stats) {
  __shared__ T As[TBK * TLD];
  __shared__ T Bs[TBK * TLD];
  const int total = offs[n];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n - 1;   // the last problem whose first tile is <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const GemmProb P = probs[lo];
    const int ntn = (gemm_dim_n(P) + TBN - 1) / TBN;
    const int l = t - offs[lo];
    gemm_tile<T, BT>(P, l / ntn, l % ntn, stats, As, Bs);
    __syncthreads();
  }
}

hipError_t launch_gemm_bt_conj(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                               unsigned long long* stats, int32_t* tile_offs) {
  if (n_probs <= 0) return hipSuccess;
  int ntm = (M_cap + TBM - 1) / TBM, ntn = (N_cap + TBN - 1) / TBN;
  if (tile_offs) {
    gemm_tile_offsets_kernel<<<1, 1024, 0, s>>>(probs, n_probs, tile_offs);
    const int grid = (int)std::min<long long>((long long)ntm * ntn * n_probs, kListGrid);
    if (c128)
      gemm_list_kernel<double2, true><<<grid, 256, 0, s>>>(probs, n_probs, tile_offs, stats);
    else
      gemm_list_kernel<float2, true><<<grid, 256, 0, s>>>(probs, n_probs, tile_offs, stats);
    return hipGetLastError();
  }
  dim3 grid(ntm * ntn, n_probs);
  if (c128)
    gemm_kernel<double2, true><<<grid, 256, 0, s>>>(probs, ntn, stats);
  else
    gemm_kernel<float2, true><<<grid, 256, 0, s>>>(probs, ntn, stats);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                          unsigned long long* stats) {
  if (n_probs <= 0) return hipSuccess;
  int ntm = (M_cap + TBM - 1) / TBM, ntn = (N_cap + TBN - 1) / TBN;
  dim3 grid(ntm * ntn, n_probs);
  if (c128)
    gemm_kernel<double2, false><<<grid, 256, 0, s>>>(probs, ntn, stats);
  else
    gemm_kernel<float2, false><<<grid, 256, 0, s>>>(probs, ntn, stats);
  return hipGetLastError();
}
