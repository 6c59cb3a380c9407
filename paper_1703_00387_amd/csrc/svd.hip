// batched truncated SVD in FP64 by one-sided block Jacobi.
//
// The SVD split with truncation of Sec. "Basic concepts" (Splitting; Eqs.
// overlap and elocal).  For theta' (m x n) the rows are orthogonalised by
// unitary combinations: Z theta' has orthogonal rows s_j v_j^dag, so each
// converged row divided by its norm is a row of V^dag and its norm is a
// singular value.  U is never formed on the TEBD path (the Hastings
// write-back needs V only).
//
// Rows are grouped in blocks of 32 (after sorting them by norm at the start of
// every sweep).  A round pairs every block with another by the circle method;
// one workgroup per pair forms the 64x64 Gram matrix of its two blocks on FP64
// MFMA, partly diagonalises it with the LDS Jacobi solver (G ~= Q D Q^dag, a
// few sweeps) and replaces the 64 rows x_p by y_j = sum_p Q[p][j] x_p (FP64
// MFMA again).
// A sweep is nb-1 rounds; sweeps repeat until a whole sweep applies no
// rotation (a pair is left alone when every |G_pq| <= max(abs_tol*|X|_F^2,
// tol*sqrt(G_pp G_qq))).
// Selection sorts the row norms descending and applies the count rule
//   k = min(k_max, min{k >= 1 : sum_{j>k} s_j^2 <= eps sum_j s_j^2}).
#include <algorithm>

#include "common.h"
#include "jacobi_small.h"
#include "mfma_tile.h"

#define JB 32   // rows per block
#define JP 64   // rows per block pair (panel)
constexpr int kPf = 3;  // staged chunks in flight per thread in the Gram and rotation loops

// Block pairs of round r by the circle method over nb blocks (nb even):
// nb - 1 rounds pair every block with every other once.  Every round keeps
// all nb/2 pairs busy, which sets the round time (one workgroup per pair).
__device__ __forceinline__ void jac_pair(int nb, int r, int p, int& I, int& J) {
  if (p == 0) {
    I = nb - 1;
    J = r;
  } else {
    I = (r + p) % (nb - 1);
    J = (r - p + nb - 1) % (nb - 1);
  }
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Preparation of the Jacobi, in three short launches so that reading X is
// spread over many workgroups: the descriptors (batched TEBD: from the bond
// items), the squared row norms (kRowSlices workgroups per matrix, one wave
// per row), then |X|_F^2 as the sum of the row norms in a fixed order, the
// natural row order, and the converged/non-finite flags.  The row norms also
// stand in nrm2 until the first round rewrites them (a matrix that never
// reaches a round, with non-finite input, keeps them for the selection).
constexpr int kRowSlices = 16;

// stats (optional) slot 5 accumulates the algorithmic work of the splits:
// 88 m n min(m, n) real flops per m x n complex SVD, the count of a
// bidiagonalisation SVD that the Jacobi's own Gram and rotation flops exceed.
__global__ void jac_desc_bonds_kernel(const BondItem* __restrict__ items, JacMat* __restrict__ mats, int n_items,
                                      int bs, int32_t* rowmap_ws, double* nrm_ws, int m_cap,
                                      unsigned long long* stats) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondItem it = items[i];
  const int d = it.d;
  JacMat M;
  M.X = it.X;
  M.rowmap = rowmap_ws + (size_t)i * m_cap;
  M.nrm2 = nrm_ws + (size_t)i * m_cap;
  M.m = it.chi[it.b] * d;
  M.n = d * it.chi[it.b + 2];
  M.ld = M.n;
  int nb = (M.m + bs - 1) / bs;
  if (nb < 2) nb = 2;
  if (nb & 1) nb++;
  M.nb = nb;
  M.rot = 0;
  M.kmax = it.chi_max;
  M.pad = 0;
  M.fro2 = 0.0;
  M.conv = 0;
  mats[i] = M;
  if (stats) {
    const unsigned long long mm = M.m, nn = M.n;
    atomicAdd(&stats[5], 88ull * mm * nn * (mm < nn ? mm : nn));
  }
}

// grid (n_mats, kRowSlices), 256 threads: wave w of slice s takes the rows
// r = 4 s + w (mod 4 kRowSlices)
__global__ __launch_bounds__(256) void jac_row_norms_kernel(const JacMat* __restrict__ mats) {
  const JacMat& M = mats[blockIdx.x];
  const int m = M.m, n = M.n, ld = M.ld, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = blockIdx.y * 4 + wave; r < m; r += 4 * kRowSlices) {
    const double2* xr = M.X + (size_t)r * ld;
    double a = 0.0;
    for (int c = lane; c < n; c += 64) {
      const double2 v = xr[c];
      a += v.x * v.x + v.y * v.y;
    }
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) M.nrm2[r] = a;
  }
}

__global__ __launch_bounds__(256) void jac_fro_kernel(JacMat* __restrict__ mats, uint32_t* status) {
  __shared__ double red[256];
  JacMat* M = mats + blockIdx.x;
  const int m = M->m;
  double a = 0.0;
  for (int r = threadIdx.x; r < m; r += blockDim.x) a += M->nrm2[r];
  const double f2 = block_sum(a, red);
  for (int g = threadIdx.x; g < m; g += blockDim.x) M->rowmap[g] = g;  // the first sweep keeps the natural order
  if (threadIdx.x == 0) {
    M->fro2 = f2;
    M->rot = 0;
    M->conv = (f2 == f2 && f2 < 1e300) ? 0 : 1;
    if (M->conv) atomicOr(status, MPS_DEV_NONFINITE);
  }
}

// Hermitian 64x64 Gram on FP64 MFMA: the 10 upper 16x16 tiles (ti <= tj)
// shared out 3, 3, 2, 2 over the four waves.
// Gram accumulators of a wave's (up to) three tiles, three real products per
// complex one: for conj(a) b, t1 = ar br, t2 = ai bi, t3 = (ar - ai)(br + bi),
// Re = t1 + t2, Im = t3 - t1 + t2.
struct HermAcc {
  doublex4 t1[3], t2[3], t3[3];
};

__device__ __forceinline__ void gram_tiles(int wave, int* ti, int* tj, int& nt) {
  // wave 0: (0,0) (0,1) (0,2); wave 1: (0,3) (1,1) (1,2); wave 2: (1,3) (2,2); wave 3: (2,3) (3,3)
  const int TI[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 2, 0}, {2, 3, 0}};
  const int TJ[4][3] = {{0, 1, 2}, {3, 1, 2}, {3, 2, 0}, {3, 3, 0}};
  nt = wave < 2 ? 3 : 2;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    ti[u] = TI[wave][u];
    tj[u] = TJ[wave][u];
  }
}

__device__ __forceinline__ void herm_acc_zero(HermAcc& a) {
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a.t1[u][r] = 0.0;
      a.t2[u][r] = 0.0;
      a.t3[u][r] = 0.0;
    }
}

// One staged K-chunk Bs[TBK][TLD] of the 64 rows: G_ij += sum_k conj(x_ik) x_jk.
__device__ __forceinline__ void herm_mma_chunk(const double2* __restrict__ Bs, HermAcc& acc, const int* ti,
                                               const int* tj, int nt, int lane) {
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      if (u < nt) {
        const double2 a = Bs[kr * TLD + ti[u] * 16 + (lane & 15)];
        const double2 b = Bs[kr * TLD + tj[u] * 16 + (lane & 15)];
        acc.t1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc.t1[u], 0, 0, 0);
        acc.t2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc.t2[u], 0, 0, 0);
        acc.t3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x - a.y, b.x + b.y, acc.t3[u], 0, 0, 0);
      }
    }
  }
}

__device__ __forceinline__ void herm_acc_to_lds(const HermAcc& acc, double2* Gs, int ldg, const int* ti,
                                                const int* tj, int nt, int lane) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (u >= nt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ti[u] * 16 + Cx<double2>::acc_row(lane, r);
      const int col = tj[u] * 16 + (lane & 15);
      const double t1 = acc.t1[u][r], t2 = acc.t2[u][r];
      const double re = t1 + t2, im = acc.t3[u][r] - t1 + t2;
      Gs[row * ldg + col] = make_double2(re, im);
      if (ti[u] != tj[u]) Gs[col * ldg + row] = make_double2(re, -im);
    }
  }
}

// Add a Hermitian partial Gram (same tile split) into the LDS matrix.
__device__ __forceinline__ void herm_acc_add_lds(const HermAcc& acc, double2* Gs, int ldg, const int* ti,
                                                 const int* tj, int nt, int lane) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (u >= nt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ti[u] * 16 + Cx<double2>::acc_row(lane, r);
      const int col = tj[u] * 16 + (lane & 15);
      const double t1 = acc.t1[u][r], t2 = acc.t2[u][r];
      const double re = t1 + t2, im = acc.t3[u][r] - t1 + t2;
      double2 g = Gs[row * ldg + col];
      Gs[row * ldg + col] = make_double2(g.x + re, g.y + im);
      if (ti[u] != tj[u]) {
        g = Gs[col * ldg + row];
        Gs[col * ldg + row] = make_double2(g.x + re, g.y - im);
      }
    }
  }
}

// The rotation's complex products with three real MFMAs instead of four
// (Gauss): for a = ar + i ai and b = br + i bi, t1 = ar br, t2 = ai bi,
// t3 = (ar + ai)(br + bi), then Re ab = t1 - t2 and Im ab = t3 - t1 - t2.
struct RotAcc {
  doublex4 t1[2][2], t2[2][2], t3[2][2];
};

__device__ __forceinline__ void rot_acc_zero(RotAcc& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a.t1[i][j][r] = 0.0;
        a.t2[i][j][r] = 0.0;
        a.t3[i][j][r] = 0.0;
      }
}

// One staged K-chunk: C(m, n) += sum_k A(k, m) B(k, n), A(k, m) = Al[k * lda + m].
__device__ __forceinline__ void rot_mma_chunk(const double2* __restrict__ Al, int lda,
                                              const double2* __restrict__ Bs, RotAcc& acc, int wm, int wn,
                                              int lane) {
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    double2 a[2], b[2];
    double as[2], bs[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = Al[kr * lda + wm + i * 16 + (lane & 15)];
      as[i] = a[i].x + a[i].y;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      b[j] = Bs[kr * TLD + wn + j * 16 + (lane & 15)];
      bs[j] = b[j].x + b[j].y;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc.t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.t1[i][j], 0, 0, 0);
        acc.t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc.t2[i][j], 0, 0, 0);
        acc.t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], bs[j], acc.t3[i][j], 0, 0, 0);
      }
  }
}

// One round of the block Jacobi (loop_sweeps == 0), or, for matrices of one
// 64-row panel (nb == 2), up to loop_sweeps complete sweeps in one launch
// (loop_sweeps > 0): the panel's only pair is re-formed, solved and rotated
// until it is orthogonal, with no launch or host round trip per sweep.
// NT = 256 (four waves) or 512 threads.  With 512 the waves form two groups
// of four: the Gram's 16-column chunks and the rotation's 64-column blocks
// alternate between the groups (each with its own two staging buffers), the
// two partial Grams are summed in LDS, and the LDS eigensolve uses all eight
// waves, so every SIMD holds two waves.
// Column split (split.S > 1, round mode only): S workgroups share a panel
// pair, slice s taking the 64-column blocks [ncb s / S, ncb (s+1) / S).
// Phase 0 writes each slice's partial Gram to split.part; phase 1 sums the S
// partials in a fixed order (so every slice holds the same G and computes the
// same rotation), runs the LDS solve and rotates its own columns.  Matrices
// whose rounds have few panel pairs (one large matrix) then use more CUs.
// Both LDS arrays of a round hold a [JP][JP+1] matrix (4160 elements) or four
// staging buffers of [TBK][TLD] (4352 elements); sized for the larger.
constexpr int kLdsElems = (JP * (JP + 1) > 4 * TBK * TLD) ? JP * (JP + 1) : 4 * TBK * TLD;

// The LDS a workgroup works in while it handles one panel pair, at module
// scope so that every kernel using the pair body addresses it directly.
__shared__ double2 jl_G[kLdsElems];         // Gram matrix; staging of the update afterwards
__shared__ double2 jl_Q[kLdsElems];         // staging of the Gram; then the panel rotation
__shared__ double2 jl_rotw[kJac64Scratch];  // rotations, index pairs and lists of the inner solve
__shared__ int jl_rows[JP];                 // physical rows of the pair
__shared__ int jl_flag;
__shared__ int jl_need;

// One panel pair (blocks I and J of matrix M, pair slot p of matrix index mat)
// handled by one workgroup: Gram, orthogonality test, LDS solve, rotation of
// the rows (or, column split, this slice's share; loop mode, several sweeps).
template <int NT>
__device__ __forceinline__ void jac_pair_body(JacMat* __restrict__ M, int I, int J, int mat, int p, int slice,
                                              double tol, double abs_tol, int inner_sweeps, int loop_sweeps,
                                              unsigned long long* stats, const JacSplit& split);

// Matrix k of the launch is mats[list[k]] for k < *n_list (slot mode) or
// mats[k] for k < n_mats; workgroup row y takes k = y, y + gridDim.y, ...
template <int NT>
__global__ __launch_bounds__(NT) void jac_round_kernel(JacMat* __restrict__ mats, int n_mats,
                                                       const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ n_list, int round, double tol,
                                                       double abs_tol, int inner_sweeps, int loop_sweeps,
                                                       unsigned long long* stats, JacSplit split) {
  // slot mode, loop mode: only when every listed matrix has one panel (as
  // the eager schedule does: otherwise the small ones run in the rounds
  // beside the others)
  if (list && loop_sweeps > 0 && n_list[1] > 2) return;
  const int nk = list ? min(*n_list, n_mats) : n_mats;
  for (int k = blockIdx.y; k < nk; k += gridDim.y) {
    const int mi = list ? list[k] : k;
    JacMat* M = mats + mi;
    if (M->conv) continue;
    const int S = split.S, slice = blockIdx.x % S;
    const int nb = M->nb, p = blockIdx.x / S;
    if (2 * p >= nb || round >= nb - 1) continue;
    if (loop_sweeps > 0 && nb != 2) continue;  // larger matrices take the round-based sweeps
    int I, J;
    jac_pair(nb, round, p, I, J);
    if (loop_sweeps > 0) {  // one panel: keep the real rows first
      I = 0;
      J = 1;
    }
    jac_pair_body<NT>(M, I, J, mi, p, slice, tol, abs_tol, inner_sweeps, loop_sweeps, stats, split);
  }
}

template <int NT>
__device__ __forceinline__ void jac_pair_body(JacMat* __restrict__ M, int I, int J, int mat, int p, int slice,
                                              double tol, double abs_tol, int inner_sweeps, int loop_sweeps,
                                              unsigned long long* stats, const JacSplit& split) {
  constexpr int NG = NT / 256;  // wave groups
  // chunks in flight per thread in the Gram and rotation loops: with two
  // waves per SIMD one is enough (measured: 233 us against 250 us for three
  // at chi = 256), and it leaves more registers
  constexpr int kPf = NG > 1 ? 1 : ::kPf;
  double2* const G = jl_G;
  double2* const Q = jl_Q;
  double2* const rotw = jl_rotw;
  int* const rows_s = jl_rows;
  int& flag = jl_flag;
  int& need = jl_need;
  const int S = split.S;
  const int m = M->m, n = M->n, ld = M->ld;
  double2* X = M->X;
  // this workgroup's 64-column blocks [cb0, cb1) and 16-column chunks [ch0, ch1)
  const int ncb_all = (n + TBN - 1) / TBN;
  const int cb0 = (int)((long long)ncb_all * slice / S), cb1 = (int)((long long)ncb_all * (slice + 1) / S);
  const int ch0 = cb0 * (TBN / TBK), ch1 = min(cb1 * (TBN / TBK), (n + TBK - 1) / TBK);
  // partial Gram of (matrix, pair, slice): [JP][JP]
  double2* part = S > 1 ? split.part + (((size_t)mat * split.pairs + p) * S + slice) * (JP * JP) : nullptr;
  const int tid = threadIdx.x, lane = tid & 63;
  // group, thread and wave inside the group (constants for one group)
  const int grp = NG > 1 ? tid >> 8 : 0, gtid = NG > 1 ? tid & 255 : tid, wave = gtid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  if (tid < JP) {
    int g = (tid < JB) ? I * JB + tid : J * JB + (tid - JB);
    rows_s[tid] = g < m ? M->rowmap[g] : -1;
  }
  const int iters = loop_sweeps > 0 ? loop_sweeps : 1;
  bool rotated = false;
  for (int it = 0; it < iters; ++it) {
  if (tid == 0) need = 0;
  __syncthreads();

  // ---- Gram matrix of the 64 rows on FP64 MFMA: G[i][j] = <x_i, x_j> --------
  // 16-column chunks are staged in LDS (two buffers); the next kPf chunks are
  // already in flight in registers, so the loads of one panel overlap its
  // multiplies.  (Phase 1 of a split round reads the partials instead.)
  if (split.phase != 1) {
    // group grp takes the chunks ci = lc * NG + grp, lc = 0 .. nloc-1
    double2* Bs0 = Q + grp * 2 * TBK * TLD;
    double2* Bs1 = Bs0 + TBK * TLD;
    const int i = gtid >> 2, kq = (gtid & 3) * 4;
    const int gi = rows_s[i];
    const double2* xr = X + (size_t)(gi >= 0 ? gi : 0) * ld;
    const int nch = max(ch1 - ch0, 0);
    const int nloc = (nch - grp + NG - 1) / NG, nloc_max = (nch + NG - 1) / NG;
    double2 v[kPf][4];
    auto load = [&](int lc, double2* dst) {
      const int ci = ch0 + lc * NG + grp;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int c = ci * TBK + kq + e;
        dst[e] = (gi >= 0 && c < n) ? xr[c] : make_double2(0.0, 0.0);
      }
    };
    auto store = [&](double2* Bs, const double2* src) {
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[(kq + e) * TLD + i] = src[e];
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u)
      if (u < nloc) load(u, v[u]);
    if (nloc > 0) store(Bs0, v[0]);
    __syncthreads();
    // G is Hermitian: only its 10 upper 16x16 tiles are formed (3, 3, 2 and 2
    // per wave of a group) and the lower ones are written as their conjugate
    // transposes.
    // The second group takes the tile sets in the order 2, 3, 0, 1, so that
    // the two waves sharing a SIMD (waves w and w + 4) hold 3 + 2 tiles
    // between them and every SIMD issues the same number of MFMAs.
    int ti[3], tj[3], nt;
    gram_tiles(grp ? (wave + 2) & 3 : wave, ti, tj, nt);
    HermAcc hacc;
    herm_acc_zero(hacc);
    // every thread passes the same barriers: nloc_max iterations for both groups
    for (int base = 0; base < nloc_max; base += kPf) {
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int lc = base + u;
        if (lc < nloc_max) {
          if (lc < nloc) {
            if (lc + kPf < nloc) load(lc + kPf, v[u]);  // chunk lc's registers were staged already
            herm_mma_chunk((lc & 1) ? Bs1 : Bs0, hacc, ti, tj, nt, lane);
            if (lc + 1 < nloc) store((lc & 1) ? Bs0 : Bs1, v[(u + 1) % kPf]);
          }
          __syncthreads();
        }
      }
    }
    if (grp == 0) herm_acc_to_lds(hacc, G, JP + 1, ti, tj, nt, lane);
    if (NG > 1) {
      __syncthreads();
      if (grp == 1) herm_acc_add_lds(hacc, G, JP + 1, ti, tj, nt, lane);
    }
  }
  __syncthreads();
  if (S > 1 && split.phase == 0) {
    // phase 0: leave this slice's partial Gram and stop
    for (int e = tid; e < JP * JP; e += NT) part[e] = G[(e / JP) * (JP + 1) + e % JP];
    return;
  }
  if (S > 1) {
    // phase 1: the pair's Gram is the sum of the S partials, added in slice order
    const double2* pp0 = split.part + ((size_t)mat * split.pairs + p) * S * (JP * JP);
    for (int e = tid; e < JP * JP; e += NT) {
      double2 a = make_double2(0.0, 0.0);
      for (int t = 0; t < S; ++t) {
        const double2 b = pp0[(size_t)t * (JP * JP) + e];
        a.x += b.x;
        a.y += b.y;
      }
      G[(e / JP) * (JP + 1) + e % JP] = a;
    }
    __syncthreads();
  }

  // ---- is any pair of the 64 rows still not orthogonal? --------------------
  // A pair counts as orthogonal when |G_pq| <= max(tol sqrt(G_pp G_qq),
  // abs_tol |X|_F^2): the absolute floor bounds the error of every squared
  // singular value by about abs_tol |X|_F^2 and guarantees termination.
  const double abs_thr = abs_tol * M->fro2;
  for (int e = tid; e < JP * JP; e += NT) {
    int r = e / JP, c = e % JP;
    if (r < c) {
      double2 g = G[r * (JP + 1) + c];
      double ag = sqrt(g.x * g.x + g.y * g.y);
      double thr = fmax(abs_thr, tol * sqrt(fabs(G[r * (JP + 1) + r].x * G[c * (JP + 1) + c].x)));
      if (ag > thr) need = 1;
    }
  }
  __syncthreads();
  // work counter (real flops): the Hermitian Gram needs 64*65/2 complex MACs
  // per column (16640 n), the rotation 64*64 (32768 n)
  if (tid == 0 && stats && slice == 0)
    atomicAdd(&stats[1], (16640ull + (need ? 32768ull : 0ull)) * (unsigned long long)n);
  if (!need) {
    if (tid < JP && rows_s[tid] >= 0 && slice == 0) M->nrm2[rows_s[tid]] = G[tid * (JP + 1) + tid].x;
    rotated = false;
    break;
  }
  rotated = true;

  if (loop_sweeps > 0 && m <= JB) {
    // a matrix of at most 32 rows: the 32x32 solve on the leading block (the
    // other rows are zero), Q the identity elsewhere
    herm_jacobi<JB, JP + 1, NT>(G, Q, JB, 0.25 * abs_thr, tol, inner_sweeps, reinterpret_cast<double4*>(rotw), &flag);
    for (int e = tid; e < JP * JP; e += NT) {
      const int i = e / JP, j = e % JP;
      if (i >= JB || j >= JB) Q[i * (JP + 1) + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
  } else {
    herm_jacobi64<NT, JP + 1>(G, Q, 0.25 * abs_thr, tol, inner_sweeps, rotw, &flag);
  }
  // the rotated rows have squared norms diag(Q^dag G Q), left on G's diagonal
  if (tid < JP && rows_s[tid] >= 0 && slice == 0) M->nrm2[rows_s[tid]] = G[tid * (JP + 1) + tid].x;
  __syncthreads();

  // ---- rotate the rows: y_j = sum_p Q[p][j] x_p, 64 columns at a time -------
  // The A operand Q[p0+k][j] is read in place from LDS; the B operand
  // X[row_{p0+k}][c0+c] is staged (two LDS buffers) with kPf steps in flight.
  {
    // group grp takes the column blocks cb = lb * NG + grp, lb = 0 .. nlb-1
    double2* Bs0 = G + grp * 2 * TBK * TLD;
    double2* Bs1 = Bs0 + TBK * TLD;
    const int k = gtid >> 4, q4 = (gtid & 15) * 4;
    constexpr int PCH = JP / TBK;  // p-chunks per column block
    const int ncb = max(cb1 - cb0, 0);
    const int nsteps = ((ncb - grp + NG - 1) / NG) * PCH, nsteps_max = ((ncb + NG - 1) / NG) * PCH;
    double2 v[kPf][4];
    auto load = [&](int st, double2* dst) {
      const int c0 = (cb0 + (st / PCH) * NG + grp) * TBN, p0 = (st % PCH) * TBK;
      const int g = rows_s[p0 + k];
      const double2* xr = X + (size_t)(g >= 0 ? g : 0) * ld;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int c = c0 + q4 + e;
        dst[e] = (g >= 0 && c < n) ? xr[c] : make_double2(0.0, 0.0);
      }
    };
    auto store = [&](double2* Bs, const double2* src) {
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[k * TLD + q4 + e] = src[e];
    };
#pragma unroll
    for (int u = 0; u < kPf; ++u)
      if (u < nsteps) load(u, v[u]);
    if (nsteps > 0) store(Bs0, v[0]);
    __syncthreads();
    RotAcc acc;
    rot_acc_zero(acc);
    // every thread passes the same barriers: nsteps_max iterations for both groups
    for (int base = 0; base < nsteps_max; base += kPf) {
#pragma unroll
      for (int u = 0; u < kPf; ++u) {
        const int st = base + u;
        if (st < nsteps_max) {
          if (st < nsteps) {
          const int c0 = (cb0 + (st / PCH) * NG + grp) * TBN, p0 = (st % PCH) * TBK;
          if (st + kPf < nsteps) load(st + kPf, v[u]);
          rot_mma_chunk(Q + p0 * (JP + 1), JP + 1, (st & 1) ? Bs1 : Bs0, acc, wm, wn, lane);
          if (p0 + TBK == JP) {
            // the column block is complete: write its 64 rows (every load of
            // these columns was issued earlier), then start the next block
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                  int row = wm + i * 16 + Cx<double2>::acc_row(lane, r);
                  int col = c0 + wn + j * 16 + (lane & 15);
                  int g = rows_s[row];
                  if (g >= 0 && col < n) {
                    const double t1 = acc.t1[i][j][r], t2 = acc.t2[i][j][r];
                    X[(size_t)g * ld + col] = make_double2(t1 - t2, acc.t3[i][j][r] - t1 - t2);
                  }
                }
            rot_acc_zero(acc);
          }
          if (st + 1 < nsteps) store((st & 1) ? Bs0 : Bs1, v[(u + 1) % kPf]);
          }
          __syncthreads();
        }
      }
    }
  }
  if (loop_sweeps == 0 && tid == 0 && slice == 0) atomicAdd(&M->rot, 1);
  __syncthreads();
  }
  // loop mode: a converged matrix is done; one whose pair still rotated in
  // the last sweep is left to the round-based sweeps (and counted as not
  // converged by the next sweep end)
  if (loop_sweeps > 0 && tid == 0) {
    if (rotated && !split.eig) {
      M->rot = 1;
    } else {
      // converged, or the eigen split: its one rotation by the eigenvectors of
      // the Gram is the split (the rows' norms are the eigenvalues s^2)
      M->rot = 0;
      M->conv = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent sweeps: one launch runs every round of every sweep of a batch.
// The work items are (sweep s, round r, matrix i, pair slot p), numbered
//   g = ((s * (nb_cap - 1) + r) * n + i) * (nb_cap / 2) + p
// and taken in increasing g from a device counter by workgroups that stay
// resident.  Inside a sweep an item needs only the two pairs of the previous
// round that held its blocks I and J (bdone[i][b] counts the rounds block b
// of matrix i has been through; without that array, the whole previous round
// of its matrix: done[i] counts its finished pair items);
// the first item of a sweep after the first (p = 0, r = 0) waits for the
// whole previous sweep, decides convergence (no rotation in it) and sorts the
// rows by norm, and the other items of that round wait for the sort
// (ready[i] = s).  Every dependency has a smaller g, so the item with the
// smallest g not yet finished can always run: the queue cannot deadlock.
// A workgroup that finishes a pair early (an orthogonal pair stops after its
// Gram) takes the next item at once instead of idling until the slowest pair
// of a round launch ends, and there is no launch or host round trip between
// rounds or sweeps.  Waits are bounded: past spin_limit polls the workgroup
// sets MPS_DEV_SCHED_TIMEOUT and leaves, and so do those waiting on it.
// Cross-workgroup visibility: the rows, norms and counters are published with
// agent-scope release fences and read after agent-scope acquires.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ld_acq(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_rlx(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *ctr >= target or the matrix is converged; false on timeout or
// when another workgroup has aborted the launch.  The polls are relaxed (no
// cache invalidation per poll); one acquire fence follows the poll that
// succeeds.
__device__ bool jac_wait(const int32_t* ctr, int target, const int32_t* conv, const int32_t* abort_flag,
                         int spin_limit) {
  for (int it = 0; it < spin_limit; ++it) {
    if (ld_rlx(ctr) >= target || ld_rlx(conv) != 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (ld_rlx(abort_flag) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

constexpr int kActExit = 0, kActSkip = 1, kActPair = 2, kActSortPair = 3;

template <int NT>
__global__ __launch_bounds__(NT) void jac_persist_kernel(JacMat* __restrict__ mats, JacSched sc, double tol,
                                                         double abs_tol, int inner_sweeps,
                                                         unsigned long long* stats, uint32_t* status) {
  __shared__ int act_s, mat_s, I_s, J_s, p_s, sweep_s, rg_s;
  const int tid = threadIdx.x, lane = tid & 63;
  // Wave 0 decides, with all its lanes active: the leader test is uniform over
  // a wave (readfirstlane), so the decision is a scalar branch around whole
  // waves.  A per-thread test (tid == 0) around the waits let the compiler
  // restructure the item loop so that the other lanes re-entered it without
  // the decision; every loop inside the decision is free of barriers.
  const bool leader = __builtin_amdgcn_readfirstlane(tid) == 0;
  // slot mode: the listed matrices (count and largest block count from the
  // list launch before this one); else all of mats[0, n)
  const int n = sc.list ? sc.act[0] : sc.n;
  const int nbl = sc.list ? sc.act[1] : sc.nb_cap;
  const int R = nbl - 1, P = nbl / 2;
  const unsigned long long total = (unsigned long long)sc.max_sweeps * R * n * P;
  JacSplit unsplit;
  unsplit.S = 1;
  unsplit.pairs = P;
  unsplit.phase = 2;
  unsplit.eig = 0;
  unsplit.part = nullptr;
  for (;;) {
    if (leader) {
      // one atomic for the wave (lane 0 adds 1, the others 0); every lane
      // takes lane 0's value
      const unsigned long long inc = lane == 0 ? 1ull : 0ull;
      const unsigned long long got =
          __hip_atomic_fetch_add(sc.head, inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long g = __shfl(got, 0);
      int act = kActExit, mi = 0, I = 0, J = 0, p = 0, sw = 0, rg = 0;
      if (g < total && ld_rlx(sc.n_conv) < n && ld_rlx(sc.abort) == 0) {
        p = (int)(g % P);
        unsigned long long q = g / P;
        mi = (int)(q % n);
        q /= n;
        const int r = (int)(q % R);
        sw = (int)(q / R);
        JacMat* M = mats + (sc.list ? sc.list[mi] : mi);
        const int nb = M->nb;
        act = kActSkip;
        if (r < nb - 1 && 2 * p < nb && ld_rlx(&M->conv) == 0) {
          const int per_round = nb / 2, rounds = nb - 1;
          rg = sw * rounds + r;   // rounds of this matrix before this one
          jac_pair(nb, r, p, I, J);
          bool ok = true;
          if (sw > 0 && r == 0 && p == 0) {
            // the whole previous sweep, then convergence and the row order
            ok = jac_wait(sc.done + mi, sw * rounds * per_round, &M->conv, sc.abort, sc.spin_limit);
            if (ok && ld_rlx(&M->conv) == 0) {
              if (__hip_atomic_load(&M->rot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                // converged: the wave's lanes store the same flag; one count
                __hip_atomic_store(&M->conv, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(sc.n_conv, lane == 0 ? 1 : 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
              } else {
                act = kActSortPair;
              }
            }
          } else if (sw > 0 && r == 0) {
            ok = jac_wait(sc.ready + mi, sw, &M->conv, sc.abort, sc.spin_limit);
            if (ok && ld_rlx(&M->conv) == 0) act = kActPair;
          } else if (r > 0) {
            if (sc.bdone) {
              // only the two pairs of the previous round that held blocks I and J
              const int32_t* bd = sc.bdone + (size_t)mi * sc.nb_cap;
              ok = jac_wait(bd + I, rg, &M->conv, sc.abort, sc.spin_limit) &&
                   jac_wait(bd + J, rg, &M->conv, sc.abort, sc.spin_limit);
            } else {
              ok = jac_wait(sc.done + mi, rg * per_round, &M->conv, sc.abort, sc.spin_limit);
            }
            if (ok && ld_rlx(&M->conv) == 0) act = kActPair;
          } else {
            act = kActPair;   // round 0 of the first sweep: the rows as prepared
          }
          if (!ok) {
            // out of time (or another workgroup gave up): every workgroup leaves
            atomicOr(status, MPS_DEV_SCHED_TIMEOUT);
            __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            act = kActExit;
          }
        }
      }
      // the lanes agree (same loads of the same words); lane 0's decision is
      // the workgroup's
      act = __shfl(act, 0);
      if (lane == 0) {
        act_s = act;
        mat_s = __shfl(mi, 0);
        I_s = I;
        J_s = J;
        p_s = p;
        sweep_s = sw;
        rg_s = rg;
      }
    }
    // the leader's acquire (in jac_wait) came after the waited-for workgroups'
    // releases; the barrier orders the rest of the workgroup after it
    __syncthreads();
    const int act = __builtin_amdgcn_readfirstlane(act_s);
    const int mi = __builtin_amdgcn_readfirstlane(mat_s);
    const int I = __builtin_amdgcn_readfirstlane(I_s), J = __builtin_amdgcn_readfirstlane(J_s);
    const int p = __builtin_amdgcn_readfirstlane(p_s), sw = __builtin_amdgcn_readfirstlane(sweep_s);
    const int rg = __builtin_amdgcn_readfirstlane(rg_s);
    __syncthreads();
    if (act == kActExit) break;
    if (act == kActSkip) continue;
    JacMat* M = mats + (sc.list ? sc.list[mi] : mi);
    if (act == kActSortPair) {
      // rows by decreasing norm (the norms the last rounds left), NaN last;
      // the ranks of all rows are computed from the norms in global memory
      const int m = M->m;
      for (int j = tid; j < m; j += NT) {
        double v = M->nrm2[j];
        if (!(v >= 0.0 && v <= 1.0e300)) v = -1.0;
        int rank = 0;
        for (int i = 0; i < m; ++i) {
          double w = M->nrm2[i];
          if (!(w >= 0.0 && w <= 1.0e300)) w = -1.0;
          rank += (w > v) || (w == v && i < j);
        }
        M->rowmap[rank] = j;
      }
      if (leader) __hip_atomic_store(&M->rot, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // every wave's stores complete (in L2), then one release by the leader
      // (its write-back of L2 covers the whole workgroup's rows)
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (leader) __hip_atomic_store(sc.ready + mi, sw, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    jac_pair_body<NT>(M, I, J, mi, p, 0, tol, abs_tol, inner_sweeps, 0, stats, unsplit);
    // publish the rotated rows and their norms, then count the item: every
    // wave waits for its stores to complete (they are in L2 then), and the
    // leader's release (one write-back of L2 to memory) precedes the count
    // (one add per workgroup: lane 0 of wave 0 adds 1, the other lanes 0)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (leader) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (sc.bdone) {
        int32_t* bd = sc.bdone + (size_t)mi * sc.nb_cap;
        __hip_atomic_store(bd + I, rg + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bd + J, rg + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_fetch_add(sc.done + mi, lane == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Slot mode: the slots of mats[0, n) with conv == 0 in slot order, their
// count and their largest block count.  One workgroup of 256.
__global__ __launch_bounds__(256) void jac_list_kernel(const JacMat* __restrict__ mats, int n, int32_t* list,
                                                       int32_t* cnt) {
  __shared__ int part[256];
  __shared__ int nbmax;
  const int tid = threadIdx.x;
  if (tid == 0) nbmax = 2;
  const int per = (n + 255) / 256, lo = min(n, tid * per), hi = min(n, lo + per);
  int c = 0, nbm = 2;
  for (int i = lo; i < hi; ++i)
    if (mats[i].conv == 0) {
      ++c;
      nbm = max(nbm, mats[i].nb);
    }
  part[tid] = c;
  __syncthreads();
  atomicMax(&nbmax, nbm);
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int v = part[t];
      part[t] = acc;
      acc += v;
    }
    cnt[0] = acc;
  }
  __syncthreads();
  int pos = part[tid];
  for (int i = lo; i < hi; ++i)
    if (mats[i].conv == 0) list[pos++] = i;
  if (tid == 0) cnt[1] = nbmax;
}

// Before a persistent launch: counters cleared, matrices already converged
// (non-finite input) counted.  One workgroup.
__global__ void jac_persist_init_kernel(JacMat* __restrict__ mats, JacSched sc) {
  __shared__ int cnt;
  if (threadIdx.x == 0) {
    cnt = 0;
    *sc.head = 0ull;
    *sc.abort = 0;
  }
  __syncthreads();
  // slot mode: the listed matrices (none of them converged)
  const int n = sc.list ? sc.act[0] : sc.n;
  int local = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    JacMat* M = mats + (sc.list ? sc.list[i] : i);
    sc.done[i] = 0;
    sc.ready[i] = 0;
    M->rot = 0;
    local += M->conv != 0;
  }
  if (sc.bdone)
    for (int i = threadIdx.x; i < n * sc.nb_cap; i += blockDim.x) sc.bdone[i] = 0;
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) *sc.n_conv = cnt;
}

// After it: a matrix whose last sweep rotated nothing is converged; one that
// still rotated after max_sweeps is flagged.
__global__ void jac_persist_finish_kernel(JacMat* __restrict__ mats, int n, uint32_t* status) {
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    JacMat* M = mats + i;
    if (!M->conv) {
      if (M->rot == 0) M->conv = 1;
      else bad = 1;
    }
  }
  if (bad) atomicOr(status, MPS_DEV_NOCONV_SVD);
}

__global__ void jac_sweep_end_kernel(JacMat* __restrict__ mats, int n_mats, int32_t* unconverged) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int i = threadIdx.x; i < n_mats; i += blockDim.x) {
    JacMat* M = mats + i;
    if (!M->conv) {
      if (M->rot == 0) M->conv = 1;
      else local++;
      M->rot = 0;
    }
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) *unconverged = cnt;
}

// Order the rows by decreasing norm before every sweep after the first, so that
// blocks hold rows of similar magnitude (the Gram-based inner solve resolves
// small rows accurately only in blocks without much larger ones; de Rijk's
// sorting idea for one-sided Jacobi).  The norms are those the last round
// wrote; the first sweep keeps the natural order, which the descending Schmidt
// values of the left bond already make nearly sorted.  One workgroup per matrix.
__global__ __launch_bounds__(256) void jac_sort_kernel(JacMat* __restrict__ mats, int m_cap) {
  extern __shared__ double dyn2[];
  double* s2 = dyn2;
  JacMat* M = mats + blockIdx.x;
  if (M->conv) return;
  const int m = M->m, tid = threadIdx.x;
  for (int r = tid; r < m; r += 256) {
    double a = M->nrm2[r];
    s2[r] = (a >= 0.0 && a <= 1.0e300) ? a : -1.0;
  }
  __syncthreads();
  for (int j = tid; j < m; j += 256) {
    double v = s2[j];
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      double w = s2[i];
      rank += (w > v) || (w == v && i < j);
    }
    M->rowmap[rank] = j;
  }
}

// Largest left and right bond dimensions over the items of a layer.
__global__ void layer_dims_kernel(const BondItem* __restrict__ items, int n_items, int32_t* out) {
  __shared__ int ml, mr;
  if (threadIdx.x == 0) {
    ml = 1;
    mr = 1;
  }
  __syncthreads();
  int a = 1, c = 1;
  for (int i = threadIdx.x; i < n_items; i += blockDim.x) {
    a = max(a, items[i].chi[items[i].b]);
    c = max(c, items[i].chi[items[i].b + 2]);
  }
  atomicMax(&ml, a);
  atomicMax(&mr, c);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = ml;
    out[1] = mr;
  }
}

// Largest block count over the batch (bounds the useful rounds of a sweep).
__global__ void jac_max_nb_kernel(const JacMat* __restrict__ mats, int n_mats, int32_t* out) {
  __shared__ int mx;
  if (threadIdx.x == 0) mx = 2;
  __syncthreads();
  int local = 2;
  for (int i = threadIdx.x; i < n_mats; i += blockDim.x)
    if (!mats[i].conv) local = max(local, mats[i].nb);
  atomicMax(&mx, local);
  __syncthreads();
  if (threadIdx.x == 0) *out = mx;
}

__global__ void jac_flag_noconv_kernel(const int32_t* unconverged, uint32_t* status) {
  if (*unconverged > 0) atomicOr(status, MPS_DEV_NOCONV_SVD);
}

// ---------------------------------------------------------------------------
// selection: row norms, descending order, count rule
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void select_kernel(const JacMat* __restrict__ mats, int32_t* perm_ws,
                                                     double* s2_ws, int m_cap, int kmax_const, double eps,
                                                     SelOut* out) {
  extern __shared__ double dyn[];
  double* s2 = dyn;                       // [m_cap]
  int* perm = (int*)(dyn + m_cap);        // [m_cap]
  const JacMat M = mats[blockIdx.x];
  const int m = M.m, tid = threadIdx.x;
  // the squared row norms of the orthogonalised rows: the diagonal of the
  // Gram that the last round formed from them (the converging sweep rotates
  // nothing, so every row's entry comes from a Gram of its final values)
  for (int r = tid; r < m; r += 256) s2[r] = M.nrm2[r];
  __syncthreads();
  // NaN or negative entries (only possible from non-finite input, already
  // flagged by the preparation) sort last as -1, so the ranks below form a
  // permutation of 0..m-1 under any input.
  for (int j = tid; j < m; j += 256) {
    double v = s2[j];
    if (!(v >= 0.0) || !(v <= 1.0e300)) s2[j] = -1.0;
  }
  __syncthreads();
  for (int j = tid; j < m; j += 256) {
    double v = s2[j];
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      double w = s2[i];
      rank += (w > v) || (w == v && i < j);
    }
    perm[rank] = j;
  }
  __syncthreads();
  int32_t* P = perm_ws + (size_t)blockIdx.x * m_cap;
  double* S = s2_ws + (size_t)blockIdx.x * m_cap;
  for (int r = tid; r < m; r += 256) {
    P[r] = perm[r];
    S[r] = fmax(s2[perm[r]], 0.0);
  }
  if (tid == 0) {
    int kmax = M.kmax > 0 ? M.kmax : kmax_const;
    double total = 0.0;
    for (int r = m - 1; r >= 0; --r) total += fmax(s2[perm[r]], 0.0);
    int k = m;
    double tail = 0.0;
    if (eps >= 0.0) {
      for (int kk = m - 1; kk >= 1; --kk) {
        double t2 = tail + fmax(s2[perm[kk]], 0.0);
        if (t2 <= eps * total) {
          tail = t2;
          k = kk;
        } else {
          break;
        }
      }
    }
    if (k > kmax) k = kmax;
    if (k < 1) k = 1;
    double disc = 0.0, kept = 0.0;
    for (int r = m - 1; r >= k; --r) disc += fmax(s2[perm[r]], 0.0);
    for (int r = k - 1; r >= 0; --r) kept += fmax(s2[perm[r]], 0.0);
    SelOut o;
    o.k = k;
    o.m = m;
    o.disc = disc;
    o.norm2 = total;
    o.nk = kept > 0.0 ? sqrt(kept) : 1.0;
    out[blockIdx.x] = o;
  }
}

// ---------------------------------------------------------------------------
// write-back of the right site and the Schmidt values (Hastings form)
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void wb_right_kernel(const BondItem* __restrict__ items,
                                                       const JacMat* __restrict__ mats,
                                                       const int32_t* __restrict__ perm_ws,
                                                       const double* __restrict__ s2_ws, int m_cap,
                                                       const SelOut* __restrict__ sel, int d, DiscLog lg) {
  const BondItem it = items[blockIdx.y];
  const JacMat M = mats[blockIdx.y];
  const SelOut so = sel[blockIdx.y];
  const int k = so.k, n = M.n, chr = n / d;
  const int32_t* P = perm_ws + (size_t)blockIdx.y * m_cap;
  const double* S2 = s2_ws + (size_t)blockIdx.y * m_cap;
  T* Vh = (T*)it.Vh;
  T* Br = (T*)it.Br;
  const int chi_max = it.chi_max;
  const size_t total = (size_t)k * n;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    int j = (int)(idx / n), col = (int)(idx % n);
    double s = sqrt(S2[j]);
    double inv = s > 0.0 ? 1.0 / s : 0.0;
    int pj = P[j];
    pj = (pj >= 0 && pj < M.m) ? pj : 0;
    double2 x = M.X[(size_t)pj * M.ld + col];
    T v;
    v.x = x.x * inv;
    v.y = x.y * inv;
    int vv = col / chr, c = col % chr;
    Br[((size_t)j * d + vv) * chi_max + c] = v;
    Vh[idx] = v;
  }
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j < k; j += 256) it.lam_m[j] = sqrt(S2[j]) / so.nk;
    if (threadIdx.x == 0) {
      it.chi[it.b + 1] = k;
      it.disc[it.b] += so.disc;
      // the update's own entry of the discarded-weight log (step from the device counter)
      if (lg.log) lg.log[(long long)(*lg.step) * lg.step_stride + lg.layer_off + it.pad] = so.disc;
    }
  }
}

__global__ void set_int_kernel(int32_t* p, int v) { *p = v; }
__global__ void inc_int_kernel(int32_t* p) { *p += 1; }

// Fill the write-back GEMM problems B_b = theta~' Vh^dag / n_k on the device.
__global__ void wb_left_probs_kernel(const BondItem* __restrict__ items, int n_items,
                                     const SelOut* __restrict__ sel, GemmProb* probs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const BondItem it = items[i];
  const int m = it.chi[it.b] * it.d;
  GemmProb p;
  const int ncols = it.d * it.chi[it.b + 2];
  p.A = it.T;
  p.B = it.Vh;
  p.C = it.Bl;
  p.M = m;
  p.N = sel[i].k;
  p.K = ncols;
  p.lda = ncols;
  p.ldb = ncols;
  p.ldc = it.chi_max;
  p.M_dev = p.N_dev = p.K_dev = nullptr;
  p.M_mul = p.N_mul = p.K_mul = 1;
  p.inv_alpha_dev = &sel[i].nk;
  p.alpha = 1.0;
  probs[i] = p;
}

// ---------------------------------------------------------------------------
// outputs of the stand-alone truncation entry point (complex128 U, S, Vh)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trunc_vh_kernel(const JacMat* mat, const int32_t* P, const double* S2,
                                                       const SelOut* sel, int64_t n, int64_t chi_max,
                                                       double2* Vh, double* S, int32_t* k_dev,
                                                       double* disc_dev, double* norm2_dev) {
  const SelOut so = *sel;
  const int k = so.k;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < (size_t)k * n;
       idx += (size_t)gridDim.x * 256) {
    int j = (int)(idx / n), col = (int)(idx % n);
    double s = sqrt(S2[j]);
    double inv = s > 0.0 ? 1.0 / s : 0.0;
    int pj = P[j];
    pj = (pj >= 0 && pj < mat->m) ? pj : 0;
    double2 x = mat->X[(size_t)pj * mat->ld + col];
    Vh[(size_t)j * n + col] = make_double2(x.x * inv, x.y * inv);
  }
  if (blockIdx.x == 0) {
    for (int j = threadIdx.x; j < k; j += 256) S[j] = sqrt(S2[j]);
    if (threadIdx.x == 0) {
      *k_dev = k;
      *disc_dev = so.disc;
      *norm2_dev = so.norm2;
    }
  }
}

// U[i][j] = sum_c theta[i][c] conj(Vh[j][c]) / s_j  (FP64)
__global__ __launch_bounds__(256) void trunc_u_kernel(const double2* theta, const double2* Vh, const double* S,
                                                      const SelOut* sel, int64_t m, int64_t n, int64_t chi_max,
                                                      double2* U) {
  const int k = sel->k;
  const size_t total = (size_t)m * k;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    int i = (int)(idx / k), j = (int)(idx % k);
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t c = 0; c < n; ++c) {
      double2 a = theta[(size_t)i * n + c], v = Vh[(size_t)j * n + c];
      acc.x += a.x * v.x + a.y * v.y;
      acc.y += a.y * v.x - a.x * v.y;
    }
    double s = S[j];
    double inv = s > 0.0 ? 1.0 / s : 0.0;
    U[(size_t)i * chi_max + j] = make_double2(acc.x * inv, acc.y * inv);
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_jac_prep_bonds(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, int bs,
                                 int32_t* rowmap_ws, double* nrm_ws, int m_cap, uint32_t* status,
                                 unsigned long long* stats) {
  if (n_items <= 0) return hipSuccess;
  jac_desc_bonds_kernel<<<(n_items + 63) / 64, 64, 0, s>>>(items, mats, n_items, bs, rowmap_ws, nrm_ws, m_cap,
                                                           stats);
  jac_row_norms_kernel<<<dim3(n_items, kRowSlices), 256, 0, s>>>(mats);
  jac_fro_kernel<<<n_items, 256, 0, s>>>(mats, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eigendecomposition split of multi-panel matrices: the Gram G = theta' theta'^dag
// on FP64 MFMA, the one-sided Jacobi on the rows of G (rows -> lambda_j u_j^dag),
// the rows normalised (their norms lambda_j = s_j^2 become the squared values
// the selection reads), W = U^dag theta' on MFMA (rows s_j v_j^dag, the form
// the write-back reads).
// ---------------------------------------------------------------------------
__global__ void eig_gram_probs_kernel(const BondItem* __restrict__ items, JacMat* mats, int n, GemmProb* probs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  JacMat& M = mats[i];
  GemmProb P;
  P.A = M.X;
  P.B = M.X;
  P.C = items[i].gram;
  P.M = M.m;
  P.N = M.m;
  P.K = M.n;
  P.lda = M.ld;
  P.ldb = M.ld;
  P.ldc = M.m;
  P.M_dev = P.N_dev = P.K_dev = nullptr;
  P.M_mul = P.N_mul = P.K_mul = 1;
  P.inv_alpha_dev = nullptr;
  P.alpha = 1.0;
  probs[i] = P;
  // the Jacobi now runs on the rows of G (m x m)
  M.X = items[i].gram;
  M.n = M.m;
  M.ld = M.m;
  M.conv = 0;
  M.rot = 0;
  M.fro2 = 0.0;
}

// grid (n_items, kRowSlices): rows of the rotated Gram normalised to u_j^dag,
// nrm2[r] = lambda_j; rows at or below the floor (floor |G|_F^2 in squared
// norm) are not resolved and become zero rows
__global__ __launch_bounds__(256) void eig_rows_kernel(const JacMat* __restrict__ mats, double floor) {
  const JacMat& M = mats[blockIdx.x];
  const int m = M.m, ld = M.ld, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = blockIdx.y * 4 + wave; r < m; r += 4 * kRowSlices) {
    const double n2 = M.nrm2[r];
    const bool keep = n2 > floor * M.fro2 && n2 > 0.0;
    const double inv = keep ? 1.0 / sqrt(n2) : 0.0;
    double2* xr = M.X + (size_t)r * ld;
    for (int c = lane; c < m; c += 64) {
      const double2 v = xr[c];
      xr[c] = make_double2(v.x * inv, v.y * inv);
    }
    if (lane == 0) M.nrm2[r] = keep ? sqrt(n2) : 0.0;
  }
}

__global__ void eig_w_probs_kernel(const BondItem* __restrict__ items, JacMat* mats, int n, GemmProb* probs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BondItem it = items[i];
  JacMat& M = mats[i];
  const int m = M.m, nn = it.d * it.chi[it.b + 2];
  GemmProb P;
  P.A = it.gram;  // normalised rows u_j^dag, [m][m]
  P.B = it.X;     // theta', [m][nn]
  P.C = it.urows;
  P.M = m;
  P.N = nn;
  P.K = m;
  P.lda = m;
  P.ldb = nn;
  P.ldc = nn;
  P.M_dev = P.N_dev = P.K_dev = nullptr;
  P.M_mul = P.N_mul = P.K_mul = 1;
  P.inv_alpha_dev = nullptr;
  P.alpha = 1.0;
  probs[i] = P;
  // selection and write-back read the rows of W with the squared values lambda_j
  M.X = it.urows;
  M.n = nn;
  M.ld = nn;
}

hipError_t launch_eig_gram(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, GemmProb* probs,
                           int m_cap, int32_t* tile_offs, uint32_t* status) {
  if (n_items <= 0) return hipSuccess;
  eig_gram_probs_kernel<<<(n_items + 63) / 64, 64, 0, s>>>(items, mats, n_items, probs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // G = theta' theta'^dag: the batched write-back GEMM form A B^dag with B = A
  e = launch_gemm_bt_conj(s, probs, n_items, m_cap, m_cap, true, nullptr, tile_offs);
  if (e != hipSuccess) return e;
  return launch_jac_prep_plain(s, mats, n_items, status);
}

hipError_t launch_eig_rows(hipStream_t s, const BondItem* items, JacMat* mats, int n_items, GemmProb* probs,
                           int m_cap, int n_cap, double floor) {
  if (n_items <= 0) return hipSuccess;
  eig_rows_kernel<<<dim3(n_items, kRowSlices), 256, 0, s>>>(mats, floor);
  eig_w_probs_kernel<<<(n_items + 63) / 64, 64, 0, s>>>(items, mats, n_items, probs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gemm_nn(s, probs, n_items, m_cap, n_cap, true, nullptr);
}

hipError_t launch_jac_prep_plain(hipStream_t s, JacMat* mats, int n_mats, uint32_t* status) {
  if (n_mats <= 0) return hipSuccess;
  jac_row_norms_kernel<<<dim3(n_mats, kRowSlices), 256, 0, s>>>(mats);
  jac_fro_kernel<<<n_mats, 256, 0, s>>>(mats, status);
  return hipGetLastError();
}

hipError_t launch_jac_list(hipStream_t s, const JacMat* mats, int n, int32_t* list, int32_t* cnt) {
  jac_list_kernel<<<1, 256, 0, s>>>(mats, n, list, cnt);
  return hipGetLastError();
}

hipError_t launch_jac_round(hipStream_t s, JacMat* mats, int n_mats, int nb_cap, int round, double tol,
                            double abs_tol, int inner_sweeps, int loop_sweeps, unsigned long long* stats,
                            int threads, int split_S, double2* split_part, int eig, const int32_t* list,
                            const int32_t* n_list, int n_grid) {
  if (n_mats <= 0) return hipSuccess;
  if (split_S < 1 || (split_S > 1 && (!split_part || loop_sweeps > 0))) return hipErrorInvalidValue;
  if ((list == nullptr) != (n_list == nullptr) || (list && n_grid < 1)) return hipErrorInvalidValue;
  JacSplit sp;
  sp.S = split_S;
  sp.pairs = nb_cap / 2;
  sp.part = split_part;
  sp.eig = eig;
  dim3 grid((nb_cap / 2) * split_S, list ? std::min(n_grid, n_mats) : n_mats);
  for (int phase = split_S > 1 ? 0 : 2; phase <= (split_S > 1 ? 1 : 2); ++phase) {
    sp.phase = phase;
    if (threads == 512)
      jac_round_kernel<512><<<grid, 512, 0, s>>>(mats, n_mats, list, n_list, round, tol, abs_tol, inner_sweeps,
                                                  loop_sweeps, stats, sp);
    else if (threads == 256)
      jac_round_kernel<256><<<grid, 256, 0, s>>>(mats, n_mats, list, n_list, round, tol, abs_tol, inner_sweeps,
                                                  loop_sweeps, stats, sp);
    else
      return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_jac_persist(hipStream_t s, JacMat* mats, const JacSched& sc, double tol, double abs_tol,
                              int inner_sweeps, unsigned long long* stats, int threads, int grid,
                              uint32_t* status) {
  if (sc.n <= 0) return hipSuccess;
  if (sc.nb_cap < 2 || (sc.nb_cap & 1) || grid < 1 || (sc.list == nullptr) != (sc.act == nullptr))
    return hipErrorInvalidValue;
  if (sc.list) jac_list_kernel<<<1, 256, 0, s>>>(mats, sc.n, sc.list, sc.act);
  jac_persist_init_kernel<<<1, 256, 0, s>>>(mats, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (threads == 512)
    jac_persist_kernel<512><<<grid, 512, 0, s>>>(mats, sc, tol, abs_tol, inner_sweeps, stats, status);
  else if (threads == 256)
    jac_persist_kernel<256><<<grid, 256, 0, s>>>(mats, sc, tol, abs_tol, inner_sweeps, stats, status);
  else
    return hipErrorInvalidValue;
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  jac_persist_finish_kernel<<<1, 256, 0, s>>>(mats, sc.n, status);
  return hipGetLastError();
}

hipError_t launch_jac_sweep_end(hipStream_t s, JacMat* mats, int n_mats, int32_t* unconverged) {
  jac_sweep_end_kernel<<<1, 256, 0, s>>>(mats, n_mats, unconverged);
  return hipGetLastError();
}

hipError_t launch_jac_sort(hipStream_t s, JacMat* mats, int n_mats, int m_cap) {
  if (n_mats <= 0) return hipSuccess;
  jac_sort_kernel<<<n_mats, 256, (size_t)m_cap * sizeof(double), s>>>(mats, m_cap);
  return hipGetLastError();
}

hipError_t launch_layer_dims(hipStream_t s, const BondItem* items, int n_items, int32_t* out) {
  layer_dims_kernel<<<1, 256, 0, s>>>(items, n_items, out);
  return hipGetLastError();
}

hipError_t launch_jac_max_nb(hipStream_t s, const JacMat* mats, int n_mats, int32_t* out) {
  jac_max_nb_kernel<<<1, 256, 0, s>>>(mats, n_mats, out);
  return hipGetLastError();
}

hipError_t launch_jac_flag_noconv(hipStream_t s, const int32_t* unconverged, uint32_t* status) {
  jac_flag_noconv_kernel<<<1, 1, 0, s>>>(unconverged, status);
  return hipGetLastError();
}

hipError_t launch_select(hipStream_t s, JacMat* mats, int n_mats, int32_t* perm_ws, double* s2_ws, int m_cap,
                         int kmax_const, double eps, SelOut* out) {
  if (n_mats <= 0) return hipSuccess;
  size_t shm = (size_t)m_cap * (sizeof(double) + sizeof(int));
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)select_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shm);
    if (e != hipSuccess) return e;
  }
  select_kernel<<<n_mats, 256, shm, s>>>(mats, perm_ws, s2_ws, m_cap, kmax_const, eps, out);
  return hipGetLastError();
}

hipError_t launch_wb_right(hipStream_t s, const BondItem* items, int n_items, const JacMat* mats,
                           const int32_t* perm_ws, const double* s2_ws, int m_cap, const SelOut* sel, int chi_cap,
                           int d, bool c128, const DiscLog& lg) {
  if (n_items <= 0) return hipSuccess;
  size_t cap = (size_t)chi_cap * d * chi_cap;
  int gx = (int)((cap + 255) / 256);
  if (gx > 64) gx = 64;
  dim3 grid(gx, n_items);
  if (c128)
    wb_right_kernel<double2><<<grid, 256, 0, s>>>(items, mats, perm_ws, s2_ws, m_cap, sel, d, lg);
  else
    wb_right_kernel<float2><<<grid, 256, 0, s>>>(items, mats, perm_ws, s2_ws, m_cap, sel, d, lg);
  return hipGetLastError();
}

hipError_t launch_set_int(hipStream_t s, int32_t* p, int v) {
  set_int_kernel<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_inc_int(hipStream_t s, int32_t* p) {
  inc_int_kernel<<<1, 1, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_wb_left_probs(hipStream_t s, const BondItem* items, int n_items, const SelOut* sel,
                                GemmProb* probs) {
  if (n_items <= 0) return hipSuccess;
  wb_left_probs_kernel<<<(n_items + 63) / 64, 64, 0, s>>>(items, n_items, sel, probs);
  return hipGetLastError();
}

hipError_t launch_truncate_out(hipStream_t s, const JacMat* mat, const int32_t* perm, const double* s2,
                               const SelOut* sel, const double2* theta, int64_t m, int64_t n, int64_t chi_max,
                               double2* U, double* S, double2* Vh, int32_t* k_dev, double* disc_dev,
                               double* norm2_dev) {
  int g1 = (int)((std::min<int64_t>(chi_max, m) * n + 255) / 256);
  if (g1 > 1024) g1 = 1024;
  if (g1 < 1) g1 = 1;
  trunc_vh_kernel<<<g1, 256, 0, s>>>(mat, perm, s2, sel, n, chi_max, Vh, S, k_dev, disc_dev, norm2_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int g2 = (int)((m * std::min<int64_t>(chi_max, m) + 255) / 256);
  if (g2 > 4096) g2 = 4096;
  if (g2 < 1) g2 = 1;
  trunc_u_kernel<<<g2, 256, 0, s>>>(theta, Vh, S, sel, m, n, chi_max, U);
  return hipGetLastError();
}
