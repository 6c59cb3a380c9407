// fused two-site tensor build, gate and left Schmidt scaling.
//
// For bond b of a Hastings-form chain (Sec. "Basic concepts": contraction of
// two neighbouring tensors into Theta; App. "Details of the Krylov method":
// steps 1 and 3 of the plain TEBD update):
//   theta~[a,s,t,c]  = sum_beta B_b[a,s,beta] B_{b+1}[beta,t,c]    (FP32 MFMA)
//   theta~'[a,u,v,c] = sum_{s,t} G[(u v),(s t)] theta~[a,s,t,c]    (epilogue)
//   theta'[a,u,v,c]  = lam_b[a] theta~'[a,u,v,c]                   (FP64 out)
// The workgroup tile covers a block of TA left indices a, every s, every t and
// a block of TC right indices c, so all d^2 (s,t) slices of each (a,c) pair
// are in the tile and the gate is applied before anything leaves the chip.
// Outputs (row (a*d+u), column (v*chi_r+c), row length n = d*chi_r):
//   T : theta~' in the chain's precision (kept for the write-back GEMM)
//   X : theta'  complex128 (input of the FP64 SVD)
// The chain precision T is complex64 (FP32 MFMA) or complex128 (FP64 MFMA).
#include "mfma_tile.h"

template <class T>
__global__ __launch_bounds__(256) void theta_gate_kernel(const BondItem* __restrict__ items, int d, int TA,
                                                         int TC, int ntc_cap, unsigned long long* stats) {
  __shared__ T smem[TBM * (TBN + 1) > 2 * TBK * TLD ? TBM * (TBN + 1) : 2 * TBK * TLD];
  __shared__ T Gs[32 * 32];
  T* As = smem;
  T* Bs = smem + TBK * TLD;
  T* Cs = smem;  // reused after the K loop
  typedef typename Cx<T>::R R;

  const BondItem it = items[blockIdx.y];
  const int chi_max = it.chi_max;
  const int chl = it.chi[it.b], chm = it.chi[it.b + 1], chr = it.chi[it.b + 2];
  const int ta = blockIdx.x / ntc_cap, tc = blockIdx.x % ntc_cap;
  const int a0 = ta * TA, c0 = tc * TC;
  if (a0 >= chl || c0 >= chr) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int dd = d * d;
  for (int i = tid; i < dd * dd; i += 256) Gs[i] = ((const T*)it.G)[i];

  AccTile<T> acc;
  acc_zero<T>(acc);
  const int rows_valid = min(TA, chl - a0) * d;    // tile rows i < rows_valid are real
  const int K = chm;
  const T* Abase = (const T*)it.Bl + (size_t)a0 * d * chi_max;
  const T* Br = (const T*)it.Br;
  for (int k0 = 0; k0 < K; k0 += TBK) {
    // A tile: rows i (a = a0 + i/d, s = i%d), k = k0..k0+15; As[k][i]
    {
      int i = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int k = k0 + kq + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (i < rows_valid && k < K) v = Abase[(size_t)i * chi_max + k];
        As[(kq + e) * TLD + i] = v;
      }
    }
    // B tile: k, columns j (t = j/TC, c = c0 + j%TC); Bs[k][j]
    {
      int k = tid >> 4, jq = (tid & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int j = jq + e;
        int t = j / TC, c = c0 + j % TC;
        T v = Cx<T>::make(0.0, 0.0);
        if (t < d && c < chr && k0 + k < K) v = Br[((size_t)(k0 + k) * d + t) * chi_max + c];
        Bs[k * TLD + j] = v;
      }
    }
    __syncthreads();
    mma_chunk<T>(As, Bs, acc, wm, wn, lane);
    __syncthreads();
  }
  acc_to_lds<T>(acc, Cs, TBN + 1, wm, wn, lane);
  __syncthreads();

  // epilogue: gate on the (s,t) slices of every (a, c) pair, then lam scaling
  const int n = d * chr;
  double2* X = it.X;
  T* Tt = (T*)it.T;
  const int na = min(TA, chl - a0), nc = min(TC, chr - c0);
  if (tid == 0 && stats)  // useful flops: theta GEMM 8*rows*cols*K, gate 8*(d^2)^2 per (a,c)
    atomicAdd(&stats[0], (unsigned long long)(8ull * (na * d) * (nc * d) * K + 8ull * dd * dd * na * nc));
  for (int p = tid; p < na * TC; p += 256) {
    int al = p / TC, cl = p % TC;
    if (cl >= nc) continue;
    int a = a0 + al, c = c0 + cl;
    T th[25];
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) th[s * d + t] = Cs[(al * d + s) * (TBN + 1) + t * TC + cl];
    double la = it.lam_l[a];
    for (int u = 0; u < d; ++u)
      for (int v = 0; v < d; ++v) {
        R ar = 0, ai = 0;
        const T* g = Gs + (u * d + v) * dd;
        for (int q = 0; q < dd; ++q) {
          ar += g[q].x * th[q].x - g[q].y * th[q].y;
          ai += g[q].x * th[q].y + g[q].y * th[q].x;
        }
        T acc2;
        acc2.x = ar;
        acc2.y = ai;
        size_t off = (size_t)(a * d + u) * n + v * chr + c;
        Tt[off] = acc2;
        X[off] = make_double2(la * (double)acc2.x, la * (double)acc2.y);
      }
  }
}

hipError_t launch_theta(hipStream_t s, const BondItem* items, int n_items, int d, int chi_cap, bool c128,
                        unsigned long long* stats) {
  if (n_items <= 0) return hipSuccess;
  if (d < 1 || d > 5) return hipErrorInvalidValue;
  const int TA = TBM / d, TC = TBN / d;
  const int nta = (chi_cap + TA - 1) / TA, ntc = (chi_cap + TC - 1) / TC;
  dim3 grid(nta * ntc, n_items);
  if (c128)
    theta_gate_kernel<double2><<<grid, 256, 0, s>>>(items, d, TA, TC, ntc, stats);
  else
    theta_gate_kernel<float2><<<grid, 256, 0, s>>>(items, d, TA, TC, ntc, stats);
  return hipGetLastError();
}
