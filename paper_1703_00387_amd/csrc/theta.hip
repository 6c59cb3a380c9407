// fused two-site tensor build, gate and left Schmidt scaling.
//
// For bond b of a Hastings-form chain (Sec. "Basic concepts": contraction of
// two neighbouring tensors into Theta; App. "Details of the Krylov method":
// steps 1 and 3 of the plain TEBD update):
//   theta~[a,s,t,c]  = sum_beta B_b[a,s,beta] B_{b+1}[beta,t,c]    (MFMA, three real
//                      products per complex one)
//   theta~'[a,u,v,c] = sum_{s,t} G[(u v),(s t)] theta~[a,s,t,c]    (epilogue)
//   theta'[a,u,v,c]  = lam_b[a] theta~'[a,u,v,c]                   (FP64 out)
// The workgroup tile covers a block of TA left indices a, every s, every t and
// a block of TC right indices c, so all d^2 (s,t) slices of each (a,c) pair
// are in the tile and the gate is applied before anything leaves the chip.
// Outputs (row (a*d+u), column (v*chi_r+c), row length n = d*chi_r):
//   T : theta~' in the chain's precision (kept for the write-back GEMM)
//   X : theta'  complex128 (input of the FP64 SVD)
// The chain precision T is complex64 (FP32 MFMA) or complex128 (FP64 MFMA).
#include <algorithm>

#include "mfma_3m.h"

// two staging buffers (A and B tiles each), reused for the output tile
template <class T>
struct ThetaLds {
  static constexpr int kElems = TBM * (TBN + 1) > 4 * TBK * TLD ? TBM * (TBN + 1) : 4 * TBK * TLD;
};

// Epilogue of one tile for local dimension D: for every (a, c) pair of the
// tile, the D^2 (s, t) slices from the LDS tile Cs, the gate applied,
// theta~' to Tt and lam_b[a] theta~' to X.
template <class T, int D>
__device__ __forceinline__ void theta_epilogue(const BondItem& it, const T* Cs, const T* Gs, int a0, int c0, int na,
                                               int nc, int TC, int chr, int n, T* Tt, double2* X) {
  typedef typename Cx<T>::R R;
  constexpr int DD = D * D;
  for (int p = threadIdx.x; p < na * TC; p += 256) {
    const int al = p / TC, cl = p % TC;
    if (cl >= nc) continue;
    const int a = a0 + al, c = c0 + cl;
    // slice q = s D + t of the pair; held in registers for D <= 3, read from
    // the LDS tile for larger D (25 complex128 would crowd the registers)
    constexpr int DR = D <= 3 ? DD : 1, UQ = D <= 3 ? DD : 1;
    T th[DR];
    if (D <= 3) {
#pragma unroll
      for (int q = 0; q < DR; ++q) th[q] = Cs[(al * D + q / D) * (TBN + 1) + (q % D) * TC + cl];
    }
    auto slice = [&](int q) -> T { return D <= 3 ? th[q % DR] : Cs[(al * D + q / D) * (TBN + 1) + (q % D) * TC + cl]; };
    const double la = it.lam_l[a];
#pragma unroll 1
    for (int u = 0; u < D; ++u)
#pragma unroll 1
      for (int v = 0; v < D; ++v) {
        R ar = 0, ai = 0;
        const T* g = Gs + (u * D + v) * DD;
#pragma unroll UQ
        for (int q = 0; q < DD; ++q) {
          const T x = slice(q);
          ar += g[q].x * x.x - g[q].y * x.y;
          ai += g[q].x * x.y + g[q].y * x.x;
        }
        T acc2;
        acc2.x = ar;
        acc2.y = ai;
        const size_t off = (size_t)(a * D + u) * n + v * chr + c;
        Tt[off] = acc2;
        X[off] = make_double2(la * (double)acc2.x, la * (double)acc2.y);
      }
  }
}

// One output tile (left block ta, right block tc) of item `it`; a tile past
// the bond's dimensions returns at once.  smem holds ThetaLds<T>::kElems
// elements, Gs 25 * 25 (the gate, d <= 5).
template <class T>
__device__ __forceinline__ void theta_tile(const BondItem& it, int d, int TA, int TC, int ta, int tc,
                                           unsigned long long* stats, const void* __restrict__ G_override,
                                           T* smem, T* Gs) {
  T* Cs = smem;  // reused after the K loop
  typedef typename Cx<T>::R R;

  const int chi_max = it.chi_max;
  const int chl = it.chi[it.b], chm = it.chi[it.b + 1], chr = it.chi[it.b + 2];
  const int a0 = ta * TA, c0 = tc * TC;
  if (a0 >= chl || c0 >= chr) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int dd = d * d;
  const T* Gsrc = G_override ? (const T*)G_override : (const T*)it.G;
  for (int i = tid; i < dd * dd; i += 256) Gs[i] = Gsrc[i];

  Acc3<T, 2, 2> acc;
  acc3_zero<T, 2, 2>(acc);
  const int rows_valid = min(TA, chl - a0) * d;    // tile rows i < rows_valid are real
  const int K = chm;
  const T* Abase = (const T*)it.Bl + (size_t)a0 * d * chi_max;
  const T* Br = (const T*)it.Br;
  // A tile: rows i (a = a0 + i/d, s = i%d), k = k0..k0+15, staged as As[k][i];
  // B tile: k, columns j (t = j/TC, c = c0 + j%TC), staged as Bs[k][j].
  // kPf chunks are in flight in registers ahead of the one being multiplied.
  // One, in both precisions: it leaves the registers to the three
  // accumulators, and it is the depth at which the complex64 build keeps them
  // in AGPRs throughout.  With three in flight that build moves part of them
  // through VGPR copies at the joins of the unrolled slots, and on the path
  // that skips the last staging store a copy reads an accumulator three
  // instructions after the MFMA writing it, well inside the instruction's
  // result latency (the compiler pads such reads to ten elsewhere); its
  // imaginary parts then came out wrong.  One in flight also measured faster.
  constexpr int kPf = 1;
  const int ia = tid >> 2, kqa = (tid & 3) * 4;
  const int kb = tid >> 4, jqb = (tid & 15) * 4;
  T va[kPf][4], vb[kPf][4];
  auto load = [&](int ci, T* da, T* db) {
    const int k0 = ci * TBK;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int k = k0 + kqa + e;
      T v = Cx<T>::make(0.0, 0.0);
      if (ia < rows_valid && k < K) v = Abase[(size_t)ia * chi_max + k];
      da[e] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int j = jqb + e;
      int t = j / TC, c = c0 + j % TC;
      T v = Cx<T>::make(0.0, 0.0);
      if (t < d && c < chr && k0 + kb < K) v = Br[((size_t)(k0 + kb) * d + t) * chi_max + c];
      db[e] = v;
    }
  };
  auto store = [&](int buf, const T* da, const T* db) {
    T* As = smem + buf * 2 * TBK * TLD;
    T* Bs = As + TBK * TLD;
#pragma unroll
    for (int e = 0; e < 4; ++e) As[(kqa + e) * TLD + ia] = da[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) Bs[kb * TLD + jqb + e] = db[e];
  };
  const int nch = (K + TBK - 1) / TBK;
#pragma unroll
  for (int u = 0; u < kPf; ++u)
    if (u < nch) load(u, va[u], vb[u]);
  store(0, va[0], vb[0]);
  __syncthreads();
  for (int base = 0; base < nch; base += kPf) {
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
      const int ci = base + u;
      if (ci < nch) {
        if (ci + kPf < nch) load(ci + kPf, va[u], vb[u]);  // chunk ci's registers were staged already
        const T* As = smem + (ci & 1) * 2 * TBK * TLD;
        mma3_chunk<T, 2, 2>(As, TLD, As + TBK * TLD, TLD, acc, wm, wn, lane);
        if (ci + 1 < nch) store((ci + 1) & 1, va[(u + 1) % kPf], vb[(u + 1) % kPf]);
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Cs[(wm + i * 16 + Cx<T>::acc_row(lane, r)) * (TBN + 1) + wn + j * 16 + (lane & 15)] =
            acc3_get<T, 2, 2>(acc, i, j, r);
  __syncthreads();

  // epilogue: gate on the (s,t) slices of every (a, c) pair, then lam scaling
  const int n = d * chr;
  double2* X = it.X;
  T* Tt = (T*)it.T;
  const int na = min(TA, chl - a0), nc = min(TC, chr - c0);
  if (tid == 0 && stats)  // useful flops: theta GEMM 8*rows*cols*K, gate 8*(d^2)^2 per (a,c)
    atomicAdd(&stats[0], (unsigned long long)(8ull * (na * d) * (nc * d) * K + 8ull * dd * dd * na * nc));
  switch (d) {  // the slices of a pair in registers: the local dimension fixed at compile time
    case 1: theta_epilogue<T, 1>(it, Cs, Gs, a0, c0, na, nc, TC, chr, n, Tt, X); break;
    case 2: theta_epilogue<T, 2>(it, Cs, Gs, a0, c0, na, nc, TC, chr, n, Tt, X); break;
    case 3: theta_epilogue<T, 3>(it, Cs, Gs, a0, c0, na, nc, TC, chr, n, Tt, X); break;
    case 4: theta_epilogue<T, 4>(it, Cs, Gs, a0, c0, na, nc, TC, chr, n, Tt, X); break;
    default: theta_epilogue<T, 5>(it, Cs, Gs, a0, c0, na, nc, TC, chr, n, Tt, X); break;
  }
}

// 1-D grid over the capacity tiles of all items, each item on one XCD (tile
// row-major within it); tiles past an item's dimensions return.
template <class T>
__global__ __launch_bounds__(256) void theta_gate_kernel(const BondItem* __restrict__ items, int n_items, int d,
                                                         int TA, int TC, int ntc_cap, int tiles_cap,
                                                         unsigned long long* stats,
                                                         const void* __restrict__ G_override) {
  __shared__ T smem[ThetaLds<T>::kElems];
  __shared__ T Gs[25 * 25];
  int item, tile;
  if (!xcd_item_tile(blockIdx.x, n_items, tiles_cap, item, tile)) return;
  const BondItem it = items[item];
  theta_tile<T>(it, d, TA, TC, tile / ntc_cap, tile % ntc_cap, stats, G_override, smem, Gs);
}

// Number of output tiles of item i: ceil(chi_l / TA) * ceil(chi_r / TC) from
// the bond dimensions on the device; offs[i] = sum of the counts before i,
// offs[n] = total (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void theta_tile_offsets_kernel(const BondItem* __restrict__ items, int n, int TA,
                                                                  int TC, int32_t* offs) {
  __shared__ int part[1024];
  const int per = (n + 1023) / 1024;
  const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
  auto count = [&](int i) {
    const BondItem& it = items[i];
    return ((it.chi[it.b] + TA - 1) / TA) * ((it.chi[it.b + 2] + TC - 1) / TC);
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

// A fixed grid walking the list of real tiles (offs from the kernel above):
// no workgroup is spent on capacity that the bonds do not use, so the grid
// can be sized without knowing the bond dimensions on the host.
template <class T>
__global__ __launch_bounds__(256) void theta_gate_list_kernel(const BondItem* __restrict__ items, int n_items,
                                                              const int32_t* __restrict__ offs, int d, int TA,
                                                              int TC, unsigned long long* stats,
                                                              const void* __restrict__ G_override) {
  __shared__ T smem[ThetaLds<T>::kElems];
  __shared__ T Gs[25 * 25];
  const int total = offs[n_items];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n_items - 1;   // the last item whose first tile is <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const BondItem it = items[lo];
    const int ntc = (it.chi[it.b + 2] + TC - 1) / TC;
    const int l = t - offs[lo];
    theta_tile<T>(it, d, TA, TC, l / ntc, l % ntc, stats, G_override, smem, Gs);
    __syncthreads();   // the next tile restages the gate and the staging buffers
  }
}

// G_override (optional): one propagator used for every item instead of its own.
hipError_t launch_theta(hipStream_t s, const BondItem* items, int n_items, int d, int chi_cap, bool c128,
                        unsigned long long* stats, const void* G_override, int32_t* tile_offs) {
  if (n_items <= 0) return hipSuccess;
  if (d < 1 || d > 5) return hipErrorInvalidValue;
  const int TA = TBM / d, TC = TBN / d;
  const int nta = (chi_cap + TA - 1) / TA, ntc = (chi_cap + TC - 1) / TC;
  if (tile_offs) {
    theta_tile_offsets_kernel<<<1, 1024, 0, s>>>(items, n_items, TA, TC, tile_offs);
    const long long cap_tiles = (long long)nta * ntc * n_items;
    const int grid = (int)std::min<long long>(cap_tiles, kListGrid);
    if (c128)
      theta_gate_list_kernel<double2><<<grid, 256, 0, s>>>(items, n_items, tile_offs, d, TA, TC, stats, G_override);
    else
      theta_gate_list_kernel<float2><<<grid, 256, 0, s>>>(items, n_items, tile_offs, d, TA, TC, stats, G_override);
    return hipGetLastError();
  }
  const int grid = (int)xcd_grid(n_items, (long long)nta * ntc);
  if (c128)
    theta_gate_kernel<double2><<<grid, 256, 0, s>>>(items, n_items, d, TA, TC, ntc, nta * ntc, stats, G_override);
  else
    theta_gate_kernel<float2><<<grid, 256, 0, s>>>(items, n_items, d, TA, TC, ntc, nta * ntc, stats, G_override);
  return hipGetLastError();
}
