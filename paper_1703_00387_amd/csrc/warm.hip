// Warm start of the batched one-sided Jacobi of a TEBD layer.
//
// The split of a bond update (Sec. "Basic concepts in tensor network
// techniques": the truncated SVD of theta') needs the singular values and the
// right singular vectors of theta' only, in the Hastings form (Sec. "Time
// evolving block decimation"): B_{b+1} <- V^dag, B_b <- theta~' conj(V).  The
// one-sided Jacobi finds them by orthogonalising the rows of theta'; a unitary
// applied on the left changes neither.  Before the gate, the bond's left
// Schmidt vectors are the columns of A = Lambda_l B_b, a (d chi_l) x chi_m
// matrix with orthogonal columns of norms lambda_b when the chain is in
// canonical form, and the gate of a short time step moves them little.  With
// A = Q R (Householder; Q unitary of order d chi_l) the rows of Q^dag theta'
// are therefore close to orthogonal, and the Jacobi converges in fewer sweeps.
// The singular values and V are those of theta' whatever Q is: the warm start
// changes the work, not the result's definition.
//
// Blocked Householder QR in the compact WY form (panels of kWsNb reflectors,
// H_1 ... H_nb = I - V T V^dag with T upper triangular; Q^dag C = C - V T^dag
// V^dag C per panel, in panel order), batched over the bonds of a layer:
//   ws_copy_kernel    A = Lambda_l B_b into the workspace (complex128, the
//                     layout of B_b: row (a, s), pitch chi_max)
//   ws_step_kernel    one launch per panel: a 16-wave workgroup per bond
//                     factors the panel in LDS (V below the diagonal of A's
//                     panel columns, T beside), while the other workgroups
//                     apply the previous panel's block reflector (FP64 MFMA)
//                     to A's later panels and to theta'
// Bond i's workgroups run on XCD i % 8, as in the other layer kernels.
// Matrices of at most 64 rows (one panel pair: their Jacobi finishes in LDS)
// and of more than kWsRows rows (the LDS panel) are left as they are.
#include <algorithm>

#include "common.h"

namespace {

constexpr int kWsRows = 512;     // rows of A the LDS panel holds
constexpr int kWsNb = 16;        // reflectors per panel
constexpr int kWsLd = kWsNb + 1; // LDS pitch of the panel (complex elements)

struct WsDims {
  int m, k, n, r;   // rows of A and theta', columns of A, columns of theta', reflectors
};

__device__ __forceinline__ WsDims ws_dims(const BondItem& it) {
  WsDims g;
  g.m = it.d * it.chi[it.b];
  g.k = it.chi[it.b + 1];
  g.n = it.d * it.chi[it.b + 2];
  g.r = min(g.m, g.k);
  return g;
}

// r_cap: the reflectors the launch sequence factors (a bond needing more is
// left as it is, so no panel is applied that was not factored)
__device__ __forceinline__ bool ws_on(const WsDims& g, int r_cap) {
  return g.m > 64 && g.m <= kWsRows && g.r > 0 && g.r <= r_cap;
}


constexpr int kWsPanelThreads = 1024;   // the panel kernel: one wave per panel column

template <class T>
__global__ __launch_bounds__(256) void ws_copy_kernel(const BondItem* __restrict__ items, int n_items,
                                                      double2* __restrict__ wsA, size_t a_stride, int slabs,
                                                      int r_cap) {
  int item, slab;
  if (!xcd_item_tile(blockIdx.x, n_items, slabs, item, slab)) return;
  const BondItem it = items[item];
  const WsDims g = ws_dims(it);
  if (!ws_on(g, r_cap)) return;
  const T* B = (const T*)it.Bl;
  double2* A = wsA + (size_t)item * a_stride;
  const int ld = it.chi_max;
  const size_t total = (size_t)g.m * g.k;
  for (size_t e = (size_t)slab * 256 + threadIdx.x; e < total; e += (size_t)slabs * 256) {
    const int i = (int)(e / g.k), c = (int)(e % g.k);
    const double la = it.lam_l[i / it.d];
    const T v = B[(size_t)i * ld + c];
    A[(size_t)i * ld + c] = make_double2(la * (double)v.x, la * (double)v.y);
  }
}

// Sum over a full wave (every lane active), the same value returned to all
// lanes: DPP sums within each row of 16 lanes (quad swaps, then the half-row
// and row mirrors), then the four row sums read from lanes 0, 16, 32, 48.
template <int Ctrl>
__device__ __forceinline__ double ws_dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), Ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), Ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double ws_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double ws_wave_sum(double v) {
  v += ws_dpp<0xB1>(v);    // quad_perm [1,0,3,2]
  v += ws_dpp<0x4E>(v);    // quad_perm [2,3,0,1]
  v += ws_dpp<0x141>(v);   // row_half_mirror
  v += ws_dpp<0x140>(v);   // row_mirror
  return (ws_lane(v, 0) + ws_lane(v, 16)) + (ws_lane(v, 32) + ws_lane(v, 48));
}

// LDS arena of the step kernel: the panel and the factorisation's small
// arrays, or the block application's partial sums (the two never overlap in
// time within a workgroup).
constexpr int kWsPanelElems = kWsRows * kWsLd + kWsNb * kWsNb + 2 * kWsNb + kWsNb / 2 + 1;
constexpr int kWsApplyElems = (kWsPanelThreads / 256) * 6 * 256;
constexpr int kWsLdsElems = kWsPanelElems > kWsApplyElems ? kWsPanelElems : kWsApplyElems;

// Factorisation of panel p (columns p .. p + w - 1, rows p .. m - 1) of A,
// by a workgroup of 16 waves with one barrier per reflector.  In the step of
// column j, wave t applies H_j^dag to panel column j + 1 + t from the
// unscaled column j (x_i, with v_i = sc x_i folded into the update); wave 0,
// whose column is the next pivot, then forms that column's norm below the
// diagonal; the last wave, which never has a column, scales the previous
// pivot column into its v.  V and R go back into A, T to Tq.
__device__ __forceinline__ void ws_factor_panel(double2* A, int lda, int p, int w, int m, double2* Tq,
                                                double2* lds) {
  constexpr int kWaves = kWsPanelThreads / 64;
  double2* P = lds;
  double2* Gm = P + kWsRows * kWsLd;      // v_l^dag v_j, l < j
  double2* tau_s = Gm + kWsNb * kWsNb;
  double2* sc_s = tau_s + kWsNb;
  double* beta_s = (double*)(sc_s + kWsNb);
  double* nrm_s = beta_s + kWsNb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mr = m - p;
  for (int e = tid; e < mr * kWsNb; e += kWsPanelThreads) {
    const int i = e / kWsNb, j = e % kWsNb;
    P[i * kWsLd + j] = j < w ? A[(size_t)(p + i) * lda + p + j] : make_double2(0.0, 0.0);
  }
  if (tid < kWsNb) {
    tau_s[tid] = make_double2(0.0, 0.0);
    sc_s[tid] = make_double2(0.0, 0.0);
    beta_s[tid] = 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    double sn = 0.0;
    for (int i = 1 + lane; i < mr; i += 64) {
      const double2 x = P[i * kWsLd];
      sn += x.x * x.x + x.y * x.y;
    }
    sn = ws_wave_sum(sn);
    if (lane == 0) nrm_s[0] = sn;
  }
  __syncthreads();

#pragma unroll 1
  for (int j = 0; j < w; ++j) {
    // the reflector of column j: H^dag (alpha; x) = (beta; 0), beta real,
    // H = I - tau v v^dag, v = (1; sc x), sc = 1 / (alpha - beta)
    const double s = nrm_s[j & 1];
    const double2 al = P[j * kWsLd + j];
    double2 tau = make_double2(0.0, 0.0), sc = make_double2(0.0, 0.0);
    double beta = al.x;
    if (s > 0.0 || al.y != 0.0) {
      const double nrm = sqrt(al.x * al.x + al.y * al.y + s);
      beta = al.x >= 0.0 ? -nrm : nrm;
      tau = make_double2((beta - al.x) / beta, -al.y / beta);
      const double2 dl = make_double2(al.x - beta, al.y);
      const double den = dl.x * dl.x + dl.y * dl.y;
      sc = make_double2(dl.x / den, -dl.y / den);
    }
    if (tid == 0) {
      tau_s[j] = tau;
      sc_s[j] = sc;
      beta_s[j] = beta;
    }
    const int c = j + 1 + wave;
    if (c < w) {
      // w_c = P[j][c] + sum_{i>j} conj(v_i) P[i][c], then P[i][c] -= v_i conj(tau) w_c.
      // A lane's rows i = j + 1 + lane + 64 r (r < kRowsPerLane) are read at
      // once; rows past the panel read row j + 1 (in range) with weight zero.
      constexpr int kRowsPerLane = kWsRows / 64;
      double2 xj[kRowsPerLane], xc[kRowsPerLane];
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) {
        const int i = j + 1 + lane + 64 * r;
        const int ii = i < mr ? i : j + 1;
        xj[r] = P[ii * kWsLd + j];
        xc[r] = P[ii * kWsLd + c];
      }
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) {
        const double wgt = j + 1 + lane + 64 * r < mr ? 1.0 : 0.0;
        const double2 t = cmulc(xj[r], xc[r]);
        acc.x += wgt * t.x;
        acc.y += wgt * t.y;
      }
      acc.x = ws_wave_sum(acc.x);
      acc.y = ws_wave_sum(acc.y);
      const double2 top = P[j * kWsLd + c];
      const double2 u = cmulc(sc, acc);
      const double2 wc = make_double2(top.x + u.x, top.y + u.y);
      const double2 f = cmulc(tau, wc);   // conj(tau) w_c
      const double2 gf = cmul(sc, f);
      if (lane == 0) P[j * kWsLd + c] = make_double2(top.x - f.x, top.y - f.y);
      double sn = 0.0;
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) {
        const int i = j + 1 + lane + 64 * r;
        const double2 d = cmul(xj[r], gf);
        const double2 y = make_double2(xc[r].x - d.x, xc[r].y - d.y);
        if (i < mr) P[i * kWsLd + c] = y;
        // the next pivot (wave 0's column c = j + 1): its norm below the diagonal
        if (i > c && i < mr) sn += y.x * y.x + y.y * y.y;
      }
      if (wave == 0) {
        sn = ws_wave_sum(sn);
        if (lane == 0) nrm_s[c & 1] = sn;
      }
    }
    if (wave == kWaves - 1 && j > 0) {
      // the previous pivot column, which nobody reads in this step
      const int q = j - 1;
      const double2 scq = sc_s[q];
      for (int i = q + 1 + lane; i < mr; i += 64) P[i * kWsLd + q] = cmul(P[i * kWsLd + q], scq);
      if (lane == 0) P[q * kWsLd + q] = make_double2(beta_s[q], 0.0);
    }
    __syncthreads();
  }
  if (wave == kWaves - 1) {
    const int q = w - 1;
    const double2 scq = sc_s[q];
    for (int i = q + 1 + lane; i < mr; i += 64) P[i * kWsLd + q] = cmul(P[i * kWsLd + q], scq);
    if (lane == 0) P[q * kWsLd + q] = make_double2(beta_s[q], 0.0);
  }
  __syncthreads();

  // Gram of the reflectors: G[l][j] = v_l^dag v_j (l < j) over rows >= j
  // (v_j is zero above row j and one at it); one pair per wave at a time
  const int n_pairs = w * (w - 1) / 2;
  for (int q = wave; q < n_pairs; q += kWsPanelThreads / 64) {
    int j = 1;
    while (j * (j + 1) / 2 <= q) ++j;
    const int l = q - j * (j - 1) / 2;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < kWsRows / 64; ++r) {
      const int i = j + 1 + lane + 64 * r;
      const int ii = i < mr ? i : j;
      const double wgt = i < mr ? 1.0 : 0.0;
      const double2 t = cmulc(P[ii * kWsLd + l], P[ii * kWsLd + j]);
      acc.x += wgt * t.x;
      acc.y += wgt * t.y;
    }
    acc.x = ws_wave_sum(acc.x);
    acc.y = ws_wave_sum(acc.y);
    if (lane == 0) {
      const double2 vlj = P[j * kWsLd + l];   // v_l at row j; v_j there is one
      Gm[l * kWsNb + j] = make_double2(vlj.x + acc.x, -vlj.y + acc.y);
    }
  }
  __syncthreads();
  // T (LAPACK's forward, columnwise form): T[j][j] = tau_j and
  // T[0:j, j] = T[0:j, 0:j] z with z_q = -tau_j G[q][j]; row l of T needs
  // only row l, so thread l builds its row alone
  if (tid < kWsNb) {
    // branch-free: row[q] is zero for q < l, so the sum over q < j runs over
    // l <= q < j; entries of Gm beyond the panel's w columns are never selected
    const int l = tid;
    double2 row[kWsNb];
#pragma unroll
    for (int j = 0; j < kWsNb; ++j) {
      double2 t = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < j; ++q) {
        const double2 u = cmul(row[q], Gm[q * kWsNb + j]);
        t.x += u.x;
        t.y += u.y;
      }
      const double2 tj = tau_s[j];
      const double2 nt = cmul(tj, t);
      const bool on = j < w && j >= l && l < w;
      row[j] = !on ? make_double2(0.0, 0.0) : (j == l ? tj : make_double2(-nt.x, -nt.y));
    }
#pragma unroll
    for (int j = 0; j < kWsNb; ++j) Tq[l * kWsNb + j] = row[j];
  }
  for (int e = tid; e < mr * kWsNb; e += kWsPanelThreads) {
    const int i = e / kWsNb, j = e % kWsNb;
    if (j < w) A[(size_t)(p + i) * lda + p + j] = P[i * kWsLd + j];
  }
}

// One 16-column tile C[:, c0 .. c0 + 15] (columns < nc valid), rows p .. m - 1:
// C -= V T^dag (V^dag C) for the panel at column p of A (V(i, l) = A[i][p + l]
// below the diagonal, one on it, zero above; l < w), on FP64 MFMA
// (v_mfma_f64_16x16x4f64: lane t supplies A[t%16][t/16] and B[t/16][t%16];
// accumulator entry r of lane t is C[t/16 + 4r][t%16]).  A complex product
// is three real ones.  256 threads = 4 waves; every lane takes part in every
// MFMA (rows past m read as zero).
typedef double ws_dx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ ws_dx4 ws_mfma(double a, double b, ws_dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double2 ws_v(const double2* A, int lda, int p, int w, int m, int k, int l) {
  const int kl = k - p;
  if (k >= m || l >= w || kl < l) return make_double2(0.0, 0.0);
  return kl == l ? make_double2(1.0, 0.0) : A[(size_t)k * lda + p + l];
}

// In a workgroup of several 256-thread sub-groups, sub-group g works on the
// tile at c0 + 16 g with its own part of sh (6 * 256 elements each); every
// sub-group passes the same barriers.
__device__ __forceinline__ void ws_apply_panel(double2* C, int ldc, int c0, int nc, const double2* A, int lda,
                                               int p, int w, int m, const double2* Tq, double2* sh0) {
  const int sg = threadIdx.x >> 8;
  double2* sh = sh0 + sg * 6 * 256;
  c0 += 16 * sg;
  const int tid = threadIdx.x & 255, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  const bool cv = col < nc;
  // a sub-group whose tile has no valid column skips the products (its
  // partial sums stay zero) but passes the same barriers
  const bool any = c0 < nc;
  // pass 1: W[l][c] = sum_k conj(V[k][l]) C[k][c]; K steps of 4 rows, step st
  // on wave st % 4, four steps' operands loaded before their MFMAs (rows past
  // m read as zero).  Three real products per complex one (a = conj(v), b = x):
  // t1 = a_r b_r, t2 = a_i b_i, t3 = (a_r + a_i)(b_r + b_i).
  ws_dx4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = {0.0, 0.0, 0.0, 0.0}, t3 = {0.0, 0.0, 0.0, 0.0};
  const int nsteps = any ? (m - p + 3) / 4 : 0;
  for (int st0 = wave; st0 < nsteps; st0 += 16) {
    double2 v[4], x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = p + (st0 + 4 * u) * 4 + lk;
      v[u] = ws_v(A, lda, p, w, m, k, li);
      x[u] = (k < m && cv) ? C[(size_t)k * ldc + col] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      t1 = ws_mfma(v[u].x, x[u].x, t1);
      t2 = ws_mfma(-v[u].y, x[u].y, t2);
      t3 = ws_mfma(v[u].x - v[u].y, x[u].x + x[u].y, t3);
    }
  }
  ws_dx4 wr, wi;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wr[r] = t1[r] - t2[r];
    wi[r] = t3[r] - t1[r] - t2[r];
  }
  double2* part = sh;              // [4 waves][16 l][16 c]
  double2* W = sh + 4 * 256;       // [16 l][16 c]
  double2* Wp = W + 256;           // [16 j][16 c]
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave * 256 + (lk + 4 * r) * 16 + li] = make_double2(wr[r], wi[r]);
  __syncthreads();
  {
    double2 t = part[tid];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      t.x += part[q * 256 + tid].x;
      t.y += part[q * 256 + tid].y;
    }
    W[tid] = t;
  }
  __syncthreads();
  {
    // W'[j][c] = sum_{l <= j} conj(T[l][j]) W[l][c]
    const int j = tid >> 4, c = tid & 15;
    double2 t = make_double2(0.0, 0.0);
    for (int l = 0; l <= j; ++l) {
      const double2 u = cmulc(Tq[l * kWsNb + j], W[l * 16 + c]);
      t.x += u.x;
      t.y += u.y;
    }
    Wp[tid] = t;
  }
  __syncthreads();
  // pass 2: C[k][c] -= sum_l V[k][l] W'[l][c]; 16-row blocks, block b on wave b % 4
  const int nblk = any ? (m - p + 15) / 16 : 0;
  for (int b = wave; b < nblk; b += 4) {
    const int q0 = p + b * 16;
    ws_dx4 u1 = {0.0, 0.0, 0.0, 0.0}, u2 = {0.0, 0.0, 0.0, 0.0}, u3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kWsNb / 4; ++kk) {
      const int l = kk * 4 + lk;
      const double2 v = ws_v(A, lda, p, w, m, q0 + li, l);
      const double2 y = Wp[l * 16 + li];
      u1 = ws_mfma(v.x, y.x, u1);
      u2 = ws_mfma(v.y, y.y, u2);
      u3 = ws_mfma(v.x + v.y, y.x + y.y, u3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = q0 + lk + 4 * r;
      if (k < m && cv) {
        double2 x = C[(size_t)k * ldc + col];
        x.x -= u1[r] - u2[r];
        x.y -= u3[r] - u1[r] - u2[r];
        C[(size_t)k * ldc + col] = x;
      }
    }
  }
  __syncthreads();   // sh and C are reused by the next panel
}

// Step q of the blocked QR and of theta' <- Q^dag theta', one launch for all
// bonds (workgroups of 16 waves).  The first n_pad workgroups (n_items
// rounded up to the XCD count) are the bonds' panel workgroups, dispatched
// first: bond i's applies block q - 1 to panel q's columns and factors panel
// q.  The others are the application workgroups, slots per bond: slots
// 0 .. n_tr - 1 apply block q - 1 to the columns of the later panels, the
// rest to theta' (64 columns each).  The roles of one launch touch disjoint
// columns, and launch q + 1 reads what launch q wrote.  The last launch
// (q = number of panels) only applies the last block to theta'.  All of a
// bond's workgroups run on XCD i % 8.
__global__ __launch_bounds__(kWsPanelThreads) void ws_step_kernel(const BondItem* __restrict__ items, int n_items,
                                                                  double2* __restrict__ wsA, size_t a_stride,
                                                                  double2* __restrict__ wsT, size_t t_stride, int q,
                                                                  int r_cap, int n_pad, int slots, int n_tr) {
  __shared__ double2 lds[kWsLdsElems];
  const int L = blockIdx.x;
  int item, slot = -1;
  if (L < n_pad) {
    item = L;
    if (item >= n_items) return;
  } else if (!xcd_item_tile(L - n_pad, n_items, slots, item, slot)) {
    return;
  }
  const BondItem it = items[item];
  const WsDims g = ws_dims(it);
  if (!ws_on(g, r_cap)) return;
  const int n_pan = (g.r + kWsNb - 1) / kWsNb;
  const int lda = it.chi_max;
  double2* A = wsA + (size_t)item * a_stride;
  double2* T0 = wsT + (size_t)item * t_stride;
  if (slot < 0) {
    if (q >= n_pan) return;
    const int p = q * kWsNb, w = min(kWsNb, g.r - p);
    if (q > 0) {
      const int pp = p - kWsNb;
      ws_apply_panel(A, lda, p, p + w, A, lda, pp, kWsNb, g.m, T0 + (size_t)(q - 1) * kWsNb * kWsNb, lds);
    }
    ws_factor_panel(A, lda, p, w, g.m, T0 + (size_t)q * kWsNb * kWsNb, lds);
    return;
  }
  if (q == 0 || q > n_pan) return;
  const int pp = (q - 1) * kWsNb, wp = min(kWsNb, g.r - pp);   // the block applied here
  const double2* Tp = T0 + (size_t)(q - 1) * kWsNb * kWsNb;
  if (slot < n_tr) {
    const int c0 = (q + 1) * kWsNb + slot * 64;
    if (c0 >= g.r) return;
    ws_apply_panel(A, lda, c0, g.r, A, lda, pp, wp, g.m, Tp, lds);
  } else {
    const int c0 = (slot - n_tr) * 64;
    if (c0 >= g.n) return;
    ws_apply_panel(it.X, g.n, c0, g.n, A, lda, pp, wp, g.m, Tp, lds);
  }
}

}  // namespace

size_t warm_a_elems(int d, int chi_cap) { return (size_t)d * chi_cap * chi_cap; }
size_t warm_t_elems(int chi_cap) { return (size_t)((chi_cap + kWsNb - 1) / kWsNb) * kWsNb * kWsNb; }

// chi_cap sizes the per-bond workspace (warm_a_elems, warm_t_elems) and
// bounds chi_m; chi_eff (<= chi_cap) bounds chi_l and chi_r of this layer.
hipError_t launch_warm_start(hipStream_t s, const BondItem* items, int n_items, int d, int chi_cap, int chi_eff,
                             bool c128, double2* wsA, double2* wsT) {
  if (n_items <= 0) return hipSuccess;
  const int m_cap = d * chi_eff;   // rows of A and theta', columns of theta'
  if (m_cap <= 64) return hipSuccess;
  const size_t a_stride = warm_a_elems(d, chi_cap), t_stride = warm_t_elems(chi_cap);
  // reflectors: min(d chi_l, chi_m) <= min(d chi_eff, chi_cap), and the LDS panel's rows
  const int r_cap = std::min(std::min(m_cap, kWsRows), chi_cap);
  const int slabs = 64;
  if (c128)
    ws_copy_kernel<double2><<<(int)xcd_grid(n_items, slabs), 256, 0, s>>>(items, n_items, wsA, a_stride, slabs,
                                                                          r_cap);
  else
    ws_copy_kernel<float2><<<(int)xcd_grid(n_items, slabs), 256, 0, s>>>(items, n_items, wsA, a_stride, slabs,
                                                                         r_cap);
  const int n_pan = (r_cap + kWsNb - 1) / kWsNb;
  const int n_tr = (r_cap + 63) / 64, n_x = (m_cap + 63) / 64;
  const int slots = n_tr + n_x;
  const int n_pad = (n_items + kXcds - 1) / kXcds * kXcds;
  const int grid = n_pad + (int)xcd_grid(n_items, slots);
  for (int q = 0; q <= n_pan; ++q)
    ws_step_kernel<<<grid, kWsPanelThreads, 0, s>>>(items, n_items, wsA, a_stride, wsT, t_stride, q, r_cap, n_pad,
                                                     slots, n_tr);
  return hipGetLastError();
}
