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
#include "mfma_tile.h"

template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmProb* __restrict__ probs, int ntn_cap,
                                                   unsigned long long* stats) {
  __shared__ T As[TBK * TLD];
  __shared__ T Bs[TBK * TLD];
  const GemmProb P = probs[blockIdx.y];
  const int M = P.M_dev ? P.M_mul * *P.M_dev : P.M;
  const int N = P.N_dev ? P.N_mul * *P.N_dev : P.N;
  const int K = P.K_dev ? P.K_mul * *P.K_dev : P.K;
  const int tm = blockIdx.x / ntn_cap, tn = blockIdx.x % ntn_cap;
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

hipError_t launch_gemm_bt_conj(hipStream_t s, const GemmProb* probs, int n_probs, int M_cap, int N_cap, bool c128,
                               unsigned long long* stats) {
  if (n_probs <= 0) return hipSuccess;
  int ntm = (M_cap + TBM - 1) / TBM, ntn = (N_cap + TBN - 1) / TBN;
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
