// Reverse-mode gradient of a TEBD2 or TEBD4 run with respect to per-bond
// couplings.
//
// Loss: sum_i w_i <O1 at site i> + sum_b w_b <O2 on bond b> of the final state
// (the observables of Sec. "Observables"; one site with weight 1 and every bond
// with weight 1 for mps_tebd_grad, any weights for mps_tebd_vjp).  The forward run stores the chain at
// the start of every step (checkpoints); the backward pass restores each step,
// re-runs its layers (3 for TEBD2, 15 for TEBD4) keeping a snapshot before
// every layer, and walks the updates in reverse.  Per update (Hastings write-back of the forward):
//   B_b' = theta~' V_k / n_k,  B_{b+1}' = V_k^dag,  lam' = s_k / n_k
//   theta' = lam_b theta~',  theta~' = G theta~,  theta~ = B_b B_{b+1}.
// The truncated-SVD backward is the full reduced-SVD backward with the
// cotangents of the discarded triplets set to zero and U never used (U_bar = 0):
//   theta'_bar = (theta' V) S^-1 [ X V^dag + diag(s/(s^2+eta)) (V_bar^dag - Jv^dag V^dag) ]
//   X_ij = F_ij s_i (Jv - Jv^dag)_ij (i != j),  X_ii = s_bar_i - i Im(Jv_ii) s_i/(2 (s_i^2+eta)),
//   Jv = V^dag V_bar,  F_ij = (s_j^2 - s_i^2) / ((s_j^2 - s_i^2)^2 + eta)
// (Lorentzian broadening eta; theta' V = U S replaces U).  Singular values
// below 1e-7 |theta'| that are not kept are treated as exact zeros and enter
// through the projector (1 - V V^dag).  The coupling gradient of the update is
// J_bar_b += Re <theta~'_bar, dG/dJ_b theta~> with dG/dJ_b = -i tau h0_b G_b.
// The reverse pass runs in complex128 (complex64 chains: on their states
// widened exactly; the forward and its re-runs in the chain's precision).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// out[p][i][r] (+)= sum_j op[i][j] in[p][j][r]   (op D x D; dagger: op^dag)
__global__ void apply_local_kernel(const double2* __restrict__ op, int D, const double2* __restrict__ in,
                                   double2* __restrict__ out, int P, int R, int dagger, int accumulate) {
  const long long total = (long long)P * R;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int p = (int)(idx / R), r = (int)(idx % R);
    const double2* ip = in + (long long)p * D * R + r;
    double2* opp = out + (long long)p * D * R + r;
    for (int i = 0; i < D; ++i) {
      double2 a = make_double2(0.0, 0.0);
      for (int j = 0; j < D; ++j) {
        double2 o = dagger ? make_double2(op[j * D + i].x, -op[j * D + i].y) : op[i * D + j];
        a = cadd(a, cmul(o, ip[(long long)j * R]));
      }
      if (accumulate) a = cadd(a, opp[(long long)i * R]);
      opp[(long long)i * R] = a;
    }
  }
}

// out[r][c] (+)= factor * lam[r / row_div]^power * in[r][c]
__global__ void row_scale_kernel(const double2* __restrict__ in, double2* out, int rows, int cols,
                                 const double* __restrict__ lam, int row_div, int power, double factor,
                                 int accumulate) {
  const long long total = (long long)rows * cols;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int r = (int)(idx / cols);
    double l = lam[r / row_div];
    double f = factor * (power == 2 ? l * l : (power == 1 ? l : 1.0));
    double2 v = in[idx];
    v = make_double2(f * v.x, f * v.y);
    if (accumulate) v = cadd(v, out[idx]);
    out[idx] = v;
  }
}

// lam_bar[a] += mult(a) * Re sum_{rows r: r/row_div = a, c} conj(A[r][c]) B[r][c]
// mult(a) = factor * (mlam ? mlam[a] : 1).  One workgroup per a.
__global__ __launch_bounds__(256) void lam_dot_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                      int row_div, int cols, double* lam_bar,
                                                      const double* __restrict__ mlam, double factor) {
  __shared__ double red[4];
  const int a = blockIdx.x;
  const long long base = (long long)a * row_div * cols;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < (long long)row_div * cols; e += blockDim.x) {
    double2 x = A[base + e], y = B[base + e];
    acc += x.x * y.x + x.y * y.y;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0] + red[1] + red[2] + red[3];
    lam_bar[a] += factor * (mlam ? mlam[a] : 1.0) * t;
  }
}

// Xt (r x r): the SVD-backward matrix with the left factor written as theta' V,
// so that theta'_bar = (theta' V) [Xt V^dag + diag(w) (Vbar^dag - Jv^dag V^dag)]:
//   Xt_ij = F_ij (Jv_ij - conj(Jv_ji))                          (i != j)
//   Xt_ii = sbar_i / s_i - i Im(Jv_ii) / (2 (s_i^2 + eta))       (i < k, else 0)
__global__ void svd_x_kernel(const double2* __restrict__ Jv, const double* __restrict__ s,
                             const double* __restrict__ sbar, int r, int k, double eta, double2* X) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < r * r; e += gridDim.x * blockDim.x) {
    int i = e / r, j = e % r;
    double2 v = make_double2(0.0, 0.0);
    if (i == j) {
      if (i < k) v = make_double2(sbar[i] / s[i], -0.5 * Jv[e].y / (s[i] * s[i] + eta));
    } else {
      double D = s[j] * s[j] - s[i] * s[i];
      double F = D != 0.0 ? D / (D * D + eta) : 0.0;
      double2 a = Jv[i * r + j], b = Jv[j * r + i];
      v = make_double2(F * (a.x - b.x), F * (a.y + b.y));
    }
    X[e] = v;
  }
}

// Y[i][c] = Y1[i][c] + w_i (conj(Vbar[c][i]) - Z[i][c]),  w_i = 1/(s_i^2+eta) for i < k, else 0
__global__ void svd_y_kernel(const double2* __restrict__ Y1, const double2* __restrict__ Z,
                             const double2* __restrict__ Vbar, const double* __restrict__ s, int r, int k, int n,
                             double eta, double2* Y) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)r * n;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e / n), c = (int)(e % n);
    double2 y = Y1[e];
    if (i < k) {
      double w = 1.0 / (s[i] * s[i] + eta);
      double2 vb = Vbar[(long long)c * r + i];
      y = make_double2(y.x + w * (vb.x - Z[e].x), y.y + w * (-vb.y - Z[e].y));
    }
    Y[e] = y;
  }
}

// Number of resolved discarded directions: rows of the sorted residual norms
// s2 (descending) with s2 > thr * (kept weight + residual weight), at most cap;
// written as the row count of a selection (for write_rows) and to rd_out.
__global__ void grad_rd_kernel(const double* __restrict__ s2, const double* __restrict__ kept2, int m, int k,
                               int cap, double thr, SelOut* sel, int* rd_out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) a += fmax(s2[j], 0.0);
  for (int j = threadIdx.x; j < k; j += blockDim.x) a += fmax(kept2[j], 0.0);
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tot = red[0];
    int rd = 0;
    while (rd < cap && s2[rd] > thr * tot) ++rd;
    SelOut o;
    o.k = rd;
    o.m = m;
    o.disc = 0.0;
    o.norm2 = tot;
    o.nk = 1.0;
    *sel = o;
    *rd_out = rd;
  }
}

// Per-update scalars of the reverse pass, from the column norms c2 of
// theta' V (kept j < k, then the resolved discarded ones, zeros after):
//   s_j = |c_j|,  n_k = (sum_{j<k} s_j^2)^(1/2),
//   n_bar = -(Re<B_bar_b', B_b'> + sum_j lam_bar'_j s_j / n_k) / n_k,
//   s_bar_j = lam_bar'_j / n_k + n_bar s_j / n_k  (j < k, else 0).
// scal = {n_k, 1/n_k}; a vanishing n_k sets the non-finite status bit.
__global__ void grad_scalars_kernel(const double* __restrict__ c2, const double* __restrict__ lbm,
                                    const double2* __restrict__ dot, int k, int r, double* sv, double* sbar,
                                    double* scal, uint32_t* status) {
  __shared__ double red[2][256];
  __shared__ double nk_s;
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double sj = sqrt(fmax(c2[j], 0.0));
    a += sj * sj;
    b += lbm[j] * sj;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double nk = sqrt(red[0][0]);
    if (!(nk > 0.0) || !(nk < 1e300)) {
      atomicOr(status, MPS_DEV_NONFINITE);
      nk = 1.0;
    }
    nk_s = nk;
    scal[0] = nk;
    scal[1] = 1.0 / nk;
    scal[2] = -(dot[0].x + red[1][0] / nk) / nk;  // n_bar
  }
  __syncthreads();
  const double nk = nk_s, nbar = scal[2];
  for (int j = threadIdx.x; j < r; j += blockDim.x) {
    double sj = sqrt(fmax(c2[j], 0.0));
    sv[j] = sj;
    sbar[j] = j < k ? lbm[j] / nk + nbar * sj / nk : 0.0;
  }
}

// out[j] = sum_i |P[i][j]|^2   (P rows x cols, row-major)
__global__ void colnorm2_kernel(const double2* __restrict__ P, int rows, int cols, double* out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int i = 0; i < rows; ++i) {
      double2 v = P[(long long)i * cols + j];
      a += v.x * v.x + v.y * v.y;
    }
    out[j] = a;
  }
}

// Vbar[i][j] += conj(Bn_bar[j][i]) for j < k   (Vbar n x r, Bn_bar k x n)
__global__ void add_conj_t_kernel(double2* Vbar, const double2* __restrict__ Bnb, int n, int r, int k) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)n * k;
       e += (long long)gridDim.x * blockDim.x) {
    int i = (int)(e / k), j = (int)(e % k);
    double2 b = Bnb[(long long)j * n + i];
    double2& v = Vbar[(long long)i * r + j];
    v = make_double2(v.x + b.x, v.y - b.y);
  }
}

// site tensor between the chain's capacity layout and a compact [chl][d][chr] block
__global__ void site_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, int chl, int d, int chr,
                                 int chi_max, int to_compact) {
  const long long total = (long long)chl * d * chr;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int c = (int)(e % chr);
    long long as = e / chr;
    long long cap = as * chi_max + c;
    if (to_compact)
      dst[e] = src[cap];
    else
      dst[cap] = src[e];
  }
}

__global__ void fill_zero_kernel(double2* a, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    a[e] = make_double2(0.0, 0.0);
}

__global__ void axpy_kernel(const double2* __restrict__ x, double2* y, long long n, double a) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    y[e] = make_double2(y[e].x + a * x[e].x, y[e].y + a * x[e].y);
}

// J_bar[b] += Re dot
__global__ void jbar_add_kernel(const double2* dot, double* jbar, int b) { jbar[b] += dot[0].x; }

// dG = -i tau h0 G   (d2 x d2)
__global__ void dgate_kernel(const double2* h0, const double2* G, double tau, int D, double2* dG) {
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    int i = e / D, j = e % D;
    double2 a = make_double2(0.0, 0.0);
    for (int k = 0; k < D; ++k) a = cadd(a, cmul(h0[i * D + k], G[k * D + j]));
    dG[e] = make_double2(tau * a.y, -tau * a.x);  // -i tau a
  }
}

namespace {

int g1d(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

struct Ctx {
  mps_handle h;
  hipStream_t s;
};

#define K1(call)                                       \
  do {                                                 \
    call;                                              \
    MPS_TRY_HIP(c.h, hipGetLastError());               \
  } while (0)

mps_status gemm128(Ctx& c, const void* A, long long rsA, long long csA, int conjA, const void* B, long long rsB,
                   long long csB, int conjB, void* C, long long rsC, int M, int N, int K, double alpha,
                   const double* alpha_dev = nullptr) {
  SGemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.rsA = rsA; g.csA = csA; g.conjA = conjA;
  g.B = B; g.rsB = rsB; g.csB = csB; g.conjB = conjB;
  g.C = C; g.rsC = rsC; g.csC = 1;
  g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.alpha_dev = alpha_dev;
  if (K <= 0) {
    K1((fill_zero_kernel<<<g1d((long long)M * N), 256, 0, c.s>>>((double2*)C, (long long)M * N)));
    return MPS_OK;
  }
  MPS_TRY_HIP(c.h, launch_sgemm(c.s, g, true));
  return MPS_OK;
}

// Layout of the caller's arena: (n_steps + 1) step checkpoints, three layer
// snapshots, the site and bond cotangents, the gates and their derivatives.
// n_layers, n_cls: layers of one step and their time-step classes (3 and 2
// for TEBD2, 15 and 4 for TEBD4).
struct GradArena {
  size_t snapB, snapL, snapC, snap;
  size_t oCk, oLay, oBb, oLb, oG, oDG, oGJ, total;
  GradArena(int L, int d, int cm, int n_steps, int n_layers = 3, int n_cls = 2) {
    const size_t site_el = (size_t)cm * d * cm, dd = (size_t)d * d;
    snapB = (size_t)L * site_el * sizeof(double2);
    snapL = (size_t)(L + 1) * cm * sizeof(double);
    snapC = (size_t)(L + 1) * sizeof(int32_t);
    snap = al(snapB) + al(snapL) + al(snapC);
    WsPlan p;
    oCk = p.take<char>((size_t)(n_steps + 1) * snap);
    oLay = p.take<char>((size_t)n_layers * snap);
    oBb = p.take<double2>((size_t)L * site_el);
    oLb = p.take<double>((size_t)(L + 1) * cm);
    oG = p.take<double2>((size_t)n_cls * (L - 1) * dd * dd);
    oDG = p.take<double2>((size_t)n_cls * (L - 1) * dd * dd);
    oGJ = p.take<GateJob>((size_t)n_cls * (L - 1));
    total = p.off;
  }
  static size_t al(size_t x) { return (x + 255) & ~size_t(255); }
  void ptrs(char* base, double2*& B, double*& lam, int32_t*& chi) const {
    B = (double2*)base;
    lam = (double*)(base + al(snapB));
    chi = (int32_t*)(base + al(snapB) + al(snapL));
  }
};

// Per-update scratch in the handle workspace, one slice per bond of a layer
// (the bonds of a layer are updated concurrently on auxiliary streams).  The
// workspace is carved again after every TEBD call, which may regrow it.
struct GradItemBuf {
  double2 *T0, *T1, *P0, *Xj, *Vh, *Vb, *Y1, *Z, *Y, *Pm, *Pb, *T1b, *T0b, *Bnew, *Bbl, *Bnl, *Bbs, *Bns, *Jv, *Xm;
  double2* dot;  // [2]: <B_bar_b', B_b'> and the coupling overlap
  double2* part; // kMdotBlocks shares of one overlap
  double *sv, *sbar, *c2, *kept2, *scal;
  int32_t* rd;
};
// One bond update of a layer in the batched reverse pass: its dimensions and
// the buffers its stages read and write (device array, one entry per bond).
struct GDesc {
  int32_t b, chl, chm, chr, m, n, k, rc, cap, d, cm, pad;
  double2 *T0, *T1, *P0, *Xj, *Vh, *Vb, *Y1, *Z, *Y, *Pm, *Pb, *T1b, *T0b, *Bnew, *Bbl, *Bnl, *Bbs, *Bns, *Jv, *Xm;
  double2* dot;
  double *sv, *sbar, *c2, *kept2, *scal;
  int32_t* rd;
  const double2 *SBb, *SBb1, *NBb, *NBb1;  // capacity-layout sites before / after the update
  double2 *bbar_b, *bbar_b1;                // compact site cotangents
  const double* lam_b;
  double *lbar_b, *lbar_b1;
  const double2 *G, *dG;
  const JacMat* mat;
  const int32_t* perm;
  const double* s2;
  SelOut* seld;
  double* dJ;   // &dJ[b]
};
constexpr int kGradGemmStages = 14;

struct GradScratch {
  std::vector<GradItemBuf> it;
  GDesc* gd;      // [n_items]
  SGemm* sg;      // [kGradGemmStages][n_items]
  double* obs;
  JacMat* mat;    // [n_items]
  SelOut *sel, *seld;
  int32_t *rowmap, *perm, *unc;
  double *s2, *nrm2;
  int m_cap;
};

mps_status grad_scratch(mps_handle h, int L, int d, int cm, GradScratch& g) {
  const int ni = L / 2;  // bonds per layer
  const size_t r = (size_t)d * cm, mn = r * r, site_el = (size_t)cm * d * cm;
  WsPlan p;
  std::vector<size_t> o((size_t)ni * 28);
  for (int i = 0; i < ni; ++i) {
    size_t* q = &o[(size_t)i * 28];
    for (int j = 0; j < 16; ++j) q[j] = p.take<double2>(mn);
    for (int j = 16; j < 20; ++j) q[j] = p.take<double2>(site_el);
    q[20] = p.take<double2>(2);
    q[21] = p.take<double>(r);
    q[22] = p.take<double>(r);
    q[23] = p.take<double>(r);
    q[24] = p.take<double>(r);
    q[25] = p.take<double>(4);
    q[26] = p.take<int32_t>(1);
    q[27] = p.take<double2>(kMdotBlocks);
  }
  size_t oObs = p.take<double>(2 * (size_t)L);
  size_t oGD = p.take<GDesc>(ni), oSG = p.take<SGemm>((size_t)kGradGemmStages * ni);
  size_t oMat = p.take<JacMat>(ni), oSel = p.take<SelOut>(ni), oSeld = p.take<SelOut>(ni);
  size_t oRm = p.take<int32_t>((size_t)ni * r), oPm = p.take<int32_t>((size_t)ni * r), oUnc = p.take<int32_t>(8);
  size_t oS2 = p.take<double>((size_t)ni * r), oNr = p.take<double>((size_t)ni * r);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  g.it.resize(ni);
  for (int i = 0; i < ni; ++i) {
    const size_t* q = &o[(size_t)i * 28];
    GradItemBuf& b = g.it[i];
    double2** mats[20] = {&b.T0, &b.T1, &b.P0, &b.Xj, &b.Vh, &b.Vb, &b.Y1, &b.Z, &b.Y, &b.Pm,
                          &b.Pb, &b.T1b, &b.T0b, &b.Bnew, &b.Jv, &b.Xm, &b.Bbl, &b.Bnl, &b.Bbs, &b.Bns};
    for (int j = 0; j < 20; ++j) *mats[j] = (double2*)(ws + q[j]);
    b.dot = (double2*)(ws + q[20]);
    b.sv = (double*)(ws + q[21]);
    b.sbar = (double*)(ws + q[22]);
    b.c2 = (double*)(ws + q[23]);
    b.kept2 = (double*)(ws + q[24]);
    b.scal = (double*)(ws + q[25]);
    b.rd = (int32_t*)(ws + q[26]);
    b.part = (double2*)(ws + q[27]);
  }
  g.obs = (double*)(ws + oObs);
  g.gd = (GDesc*)(ws + oGD);
  g.sg = (SGemm*)(ws + oSG);
  g.mat = (JacMat*)(ws + oMat);
  g.sel = (SelOut*)(ws + oSel);
  g.seld = (SelOut*)(ws + oSeld);
  g.rowmap = (int32_t*)(ws + oRm);
  g.perm = (int32_t*)(ws + oPm);
  g.unc = (int32_t*)(ws + oUnc);
  g.s2 = (double*)(ws + oS2);
  g.nrm2 = (double*)(ws + oNr);
  g.m_cap = (int)r;
  return MPS_OK;
}

// ---------------------------------------------------------------------------
// Batched reverse pass of one layer: every stage covers all bonds of the
// layer in one launch (grid.y = bond), with the same arithmetic per bond as
// the single-update adjoint (mps_truncate_vjp, mps_theta_gate_vjp).
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long bg_tid() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long bg_stride() { return (long long)gridDim.x * blockDim.x; }

// compact [rows / d][d][cols] block of a capacity-layout site [cm][d][cm]
__device__ __forceinline__ void bg_site_compact(const double2* __restrict__ src, double2* dst, int a_n, int d,
                                                int c_n, int cm) {
  const long long total = (long long)a_n * d * c_n;
  for (long long e = bg_tid(); e < total; e += bg_stride()) {
    const int c = (int)(e % c_n);
    const long long as = e / c_n;
    dst[e] = src[as * cm + c];
  }
}

// cotangents in, the update's tensors compacted
__global__ __launch_bounds__(256) void bg_prep_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  for (long long e = bg_tid(); e < (long long)q.m * q.k; e += bg_stride()) q.Bbl[e] = q.bbar_b[e];
  for (long long e = bg_tid(); e < (long long)q.k * q.n; e += bg_stride()) q.Bnl[e] = q.bbar_b1[e];
  bg_site_compact(q.SBb, q.Bbs, q.chl, q.d, q.chm, q.cm);
  bg_site_compact(q.SBb1, q.Bns, q.chm, q.d, q.chr, q.cm);
  bg_site_compact(q.NBb1, q.Vh, q.k, q.d, q.chr, q.cm);
  bg_site_compact(q.NBb, q.Bnew, q.chl, q.d, q.k, q.cm);
}

// theta~' = G theta~ (T1) and theta' = lam_b theta~' (P0)
__global__ __launch_bounds__(256) void bg_gate_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  const int dd = q.d * q.d, R = q.chr;
  for (long long idx = bg_tid(); idx < (long long)q.chl * R; idx += bg_stride()) {
    const int pp = (int)(idx / R), rr = (int)(idx % R);
    const long long base = (long long)pp * dd * R + rr;
    const double la = q.lam_b[pp];
    for (int i = 0; i < dd; ++i) {
      double2 a = make_double2(0.0, 0.0);
      for (int j = 0; j < dd; ++j) a = cadd(a, cmul(q.G[i * dd + j], q.T0[base + (long long)j * R]));
      q.T1[base + (long long)i * R] = a;
      q.P0[base + (long long)i * R] = make_double2(la * a.x, la * a.y);
    }
  }
}

// residual theta' (1 - V_k V_k^dag) and the kept column weights |theta' V_k|^2
__global__ __launch_bounds__(256) void bg_resid_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  for (long long e = bg_tid(); e < (long long)q.m * q.n; e += bg_stride()) {
    const double2 x = q.P0[e], z = q.Z[e];
    q.Xj[e] = make_double2(x.x + (-1.0) * z.x, x.y + (-1.0) * z.y);
  }
  for (long long j = bg_tid(); j < q.k; j += bg_stride()) {
    double a = 0.0;
    for (int i = 0; i < q.m; ++i) {
      const double2 v = q.Pm[(long long)i * q.k + j];
      a += v.x * v.x + v.y * v.y;
    }
    q.kept2[j] = a;
  }
}

// resolved discarded directions (count), the rows they go to cleared; one workgroup per bond
__global__ __launch_bounds__(256) void bg_rd_kernel(const GDesc* __restrict__ D) {
  __shared__ double red[256];
  const GDesc& q = D[blockIdx.x];
  double a = 0.0;
  for (int j = threadIdx.x; j < q.m; j += blockDim.x) a += fmax(q.s2[j], 0.0);
  for (int j = threadIdx.x; j < q.k; j += blockDim.x) a += fmax(q.kept2[j], 0.0);
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tot = red[0];
    int rd = 0;
    while (rd < q.cap && q.s2[rd] > 1e-26 * tot) ++rd;
    SelOut o;
    o.k = rd;
    o.m = q.m;
    o.disc = 0.0;
    o.norm2 = tot;
    o.nk = 1.0;
    *q.seld = o;
    *q.rd = rd;
  }
  if (q.cap > 0) {
    double2* Vd = q.Vh + (size_t)q.k * q.n;
    for (long long e = threadIdx.x; e < (long long)q.cap * q.n; e += blockDim.x) Vd[e] = make_double2(0.0, 0.0);
  }
}

// the resolved residual rows, normalised, as the discarded rows of V^dag
__global__ __launch_bounds__(256) void bg_rows_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  if (q.cap <= 0) return;
  const int kk = q.seld->k, len = q.n;
  const JacMat M = *q.mat;
  double2* Vd = q.Vh + (size_t)q.k * q.n;
  for (long long idx = bg_tid(); idx < (long long)kk * len; idx += bg_stride()) {
    const int j = (int)(idx / len), e = (int)(idx % len);
    int pj = q.perm[j];
    pj = (pj >= 0 && pj < M.m) ? pj : 0;
    const double sj = sqrt(q.s2[j]);
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    const double2 x = M.X[(size_t)pj * M.ld + e];
    Vd[(size_t)j * len + e] = make_double2(x.x * inv, x.y * inv);
  }
}

// V_d -= (V_d V_k^dag) V_k (the projection formed in Z)
__global__ __launch_bounds__(256) void bg_reproj_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  if (q.cap <= 0) return;
  double2* Vd = q.Vh + (size_t)q.k * q.n;
  for (long long e = bg_tid(); e < (long long)q.cap * q.n; e += bg_stride()) {
    const double2 z = q.Z[e], y = Vd[e];
    Vd[e] = make_double2(y.x + (-1.0) * z.x, y.y + (-1.0) * z.y);
  }
}

// per bond (one workgroup): column weights c2 of P = theta' V, <B_bar_b', B_b'>,
// the scalars n_k, 1/n_k, n_bar, s and s_bar (as in the single-update pass),
// and V_bar cleared
__global__ __launch_bounds__(256) void bg_scal_kernel(const GDesc* __restrict__ D, uint32_t* status) {
  __shared__ double red[2][256];
  __shared__ double nk_s, nbar_s;
  const GDesc& q = D[blockIdx.x];
  const int rc = q.rc, k = q.k;
  for (int j = threadIdx.x; j < rc; j += blockDim.x) {
    double a = 0.0;
    for (int i = 0; i < q.m; ++i) {
      const double2 v = q.Pm[(long long)i * rc + j];
      a += v.x * v.x + v.y * v.y;
    }
    q.c2[j] = a;
  }
  double dr = 0.0;
  for (long long e = threadIdx.x; e < (long long)q.m * k; e += blockDim.x) {
    const double2 v = q.Bbl[e], x = q.Bnew[e];
    dr += v.x * x.x + v.y * x.y;
  }
  for (long long e = threadIdx.x; e < (long long)q.n * rc; e += blockDim.x) q.Vb[e] = make_double2(0.0, 0.0);
  red[0][threadIdx.x] = dr;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[0][threadIdx.x] += red[0][threadIdx.x + o];
    __syncthreads();
  }
  const double dot = red[0][0];
  __syncthreads();
  const double* lbm = q.lbar_b1;
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double sj = sqrt(fmax(q.c2[j], 0.0));
    a += sj * sj;
    b += lbm[j] * sj;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double nk = sqrt(red[0][0]);
    if (!(nk > 0.0) || !(nk < 1e300)) {
      atomicOr(status, MPS_DEV_NONFINITE);
      nk = 1.0;
    }
    nk_s = nk;
    nbar_s = -(dot + red[1][0] / nk) / nk;
    q.scal[0] = nk;
    q.scal[1] = 1.0 / nk;
    q.scal[2] = nbar_s;
    q.dot[0] = make_double2(dot, 0.0);
  }
  __syncthreads();
  const double nk = nk_s, nbar = nbar_s;
  for (int j = threadIdx.x; j < rc; j += blockDim.x) {
    const double sj = sqrt(fmax(q.c2[j], 0.0));
    q.sv[j] = sj;
    q.sbar[j] = j < k ? lbm[j] / nk + nbar * sj / nk : 0.0;
  }
}

// V_bar[i][j] += conj(B_bar_{b+1}'[j][i]) for j < k
__global__ __launch_bounds__(256) void bg_addconj_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  for (long long e = bg_tid(); e < (long long)q.n * q.k; e += bg_stride()) {
    const int i = (int)(e / q.k), j = (int)(e % q.k);
    const double2 b = q.Bnl[(long long)j * q.n + i];
    double2& v = q.Vb[(long long)i * q.rc + j];
    v = make_double2(v.x + b.x, v.y - b.y);
  }
}

// the SVD-backward matrix Xt (as svd_x_kernel) for every bond
__global__ __launch_bounds__(256) void bg_svdx_kernel(const GDesc* __restrict__ D, double eta) {
  const GDesc& q = D[blockIdx.y];
  const int r = q.rc, k = q.k;
  for (long long e = bg_tid(); e < (long long)r * r; e += bg_stride()) {
    const int i = (int)(e / r), j = (int)(e % r);
    double2 v = make_double2(0.0, 0.0);
    if (i == j) {
      if (i < k) v = make_double2(q.sbar[i] / q.sv[i], -0.5 * q.Jv[e].y / (q.sv[i] * q.sv[i] + eta));
    } else {
      const double Dd = q.sv[j] * q.sv[j] - q.sv[i] * q.sv[i];
      const double F = Dd != 0.0 ? Dd / (Dd * Dd + eta) : 0.0;
      const double2 a = q.Jv[(long long)i * r + j], b = q.Jv[(long long)j * r + i];
      v = make_double2(F * (a.x - b.x), F * (a.y + b.y));
    }
    q.Xm[e] = v;
  }
}

// Y = Y1 + diag(w) (V_bar^dag - Jv^dag V^dag) (as svd_y_kernel)
__global__ __launch_bounds__(256) void bg_svdy_kernel(const GDesc* __restrict__ D, double eta) {
  const GDesc& q = D[blockIdx.y];
  const int r = q.rc, k = q.k, n = q.n;
  for (long long e = bg_tid(); e < (long long)r * n; e += bg_stride()) {
    const int i = (int)(e / n), c = (int)(e % n);
    double2 y = q.Y1[e];
    if (i < k) {
      const double w = 1.0 / (q.sv[i] * q.sv[i] + eta);
      const double2 vb = q.Vb[(long long)c * r + i];
      y = make_double2(y.x + w * (vb.x - q.Z[e].x), y.y + w * (-vb.y - q.Z[e].y));
    }
    q.Y[e] = y;
  }
}

// theta~'_bar += lam_b theta'_bar and lam_bar_b += Re<theta'_bar, theta~'>;
// workgroup (a, bond) takes the d rows of left index a
__global__ __launch_bounds__(256) void bg_thetabar_kernel(const GDesc* __restrict__ D) {
  __shared__ double red[4];
  const GDesc& q = D[blockIdx.y];
  const int a = blockIdx.x;
  if (a >= q.chl) return;
  const long long base = (long long)a * q.d * q.n, len = (long long)q.d * q.n;
  const double la = q.lam_b[a];
  double acc = 0.0;
  for (long long e = threadIdx.x; e < len; e += blockDim.x) {
    const double2 x = q.Pb[base + e], y = q.T1[base + e];
    acc += x.x * y.x + x.y * y.y;
    const double2 t = q.T1b[base + e];
    q.T1b[base + e] = make_double2(la * x.x + t.x, la * x.y + t.y);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) q.lbar_b[a] += 1.0 * (red[0] + red[1] + red[2] + red[3]);
}

// dG/dJ theta~ (Z) and theta~_bar = G^dag theta~'_bar (T0b)
__global__ __launch_bounds__(256) void bg_gatebar_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.y];
  const int dd = q.d * q.d, R = q.chr;
  for (long long idx = bg_tid(); idx < (long long)q.chl * R; idx += bg_stride()) {
    const int pp = (int)(idx / R), rr = (int)(idx % R);
    const long long base = (long long)pp * dd * R + rr;
    for (int i = 0; i < dd; ++i) {
      double2 a = make_double2(0.0, 0.0), g = make_double2(0.0, 0.0);
      for (int j = 0; j < dd; ++j) {
        a = cadd(a, cmul(q.dG[i * dd + j], q.T0[base + (long long)j * R]));
        const double2 o = make_double2(q.G[j * dd + i].x, -q.G[j * dd + i].y);
        g = cadd(g, cmul(o, q.T1b[base + (long long)j * R]));
      }
      q.Z[base + (long long)i * R] = a;
      q.T0b[base + (long long)i * R] = g;
    }
  }
}

// J_bar_b += Re<theta~'_bar, dG/dJ_b theta~> (one workgroup per bond), lam_bar_{b+1} cleared
__global__ __launch_bounds__(256) void bg_jbar_kernel(const GDesc* __restrict__ D) {
  __shared__ double red[4];
  const GDesc& q = D[blockIdx.x];
  double acc = 0.0;
  for (long long e = threadIdx.x; e < (long long)q.m * q.n; e += blockDim.x) {
    const double2 v = q.T1b[e], x = q.Z[e];
    acc += v.x * x.x + v.y * x.y;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *q.dJ += red[0] + red[1] + red[2] + red[3];
}

__global__ void bg_zero_lbar_kernel(const GDesc* __restrict__ D) {
  const GDesc& q = D[blockIdx.x];
  for (int j = threadIdx.x; j < q.cm; j += blockDim.x) q.lbar_b1[j] = 0.0;
}

SGemm sg_make(const void* A, long long rsA, long long csA, int conjA, const void* B, long long rsB, long long csB,
              int conjB, void* C, long long rsC, int M, int N, int K, const double* alpha_dev = nullptr) {
  SGemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.rsA = rsA; g.csA = csA; g.conjA = conjA;
  g.B = B; g.rsB = rsB; g.csB = csB; g.conjB = conjB;
  g.C = C; g.rsC = rsC; g.csC = 1;
  g.M = M; g.N = N; g.K = K; g.alpha = 1.0; g.alpha_dev = alpha_dev;
  return g;
}

}  // namespace

extern "C" size_t mps_tebd_grad_arena_bytes(int32_t L, int32_t d, int32_t chi_max, int32_t n_steps) {
  if (L < 2 || d < 1 || chi_max < 1 || n_steps < 1) return 0;
  return GradArena(L, d, chi_max, n_steps).total;
}

int64_t ckpt_shape_sum(const mps_chain_desc* chains, int n_chains) {
  int64_t t = 0;
  for (int c = 0; c < n_chains; ++c)
    t += (int64_t)(c + 1) * (chains[c].L * 1000003LL + chains[c].d * 1009LL + chains[c].chi_max);
  return t;
}

// A chain's block of the checkpoint arena holds the adjoint's arena of the
// larger scheme (TEBD4: 15 layer snapshots, 4 gate classes), so one arena
// serves runs of either order.
size_t ckpt_block_bytes(const mps_chain_desc& ch, int n_steps) {
  return (GradArena(ch.L, ch.d, ch.chi_max, n_steps, 15, 4).total + 255) & ~size_t(255);
}

size_t ckpt_block_offset(const mps_chain_desc* chains, int c, int n_steps) {
  size_t off = kCkptHeader;
  for (int i = 0; i < c; ++i) off += ckpt_block_bytes(chains[i], n_steps);
  return off;
}

extern "C" size_t mps_tebd_ckpt_bytes(const mps_chain_desc* chains, int32_t n_chains, int32_t n_steps) {
  if (!chains || n_chains < 1 || n_steps < 1) return 0;
  for (int c = 0; c < n_chains; ++c)
    if (chains[c].L < 2 || chains[c].d < 1 || chains[c].chi_max < 1) return 0;
  return ckpt_block_offset(chains, n_chains, n_steps);
}

// Checkpoint of step `st` of a chain into its adjoint arena block (the same
// layout the adjoint's own forward writes): B, lam and chi copied device to
// device on `s`.
mps_status grad_ckpt_save(mps_handle h, hipStream_t s, const mps_chain_desc& ch, char* block, int n_steps, int st) {
  const GradArena A(ch.L, ch.d, ch.chi_max, n_steps);
  double2* B;
  double* lam;
  int32_t* chi;
  A.ptrs(block + A.oCk + (size_t)st * A.snap, B, lam, chi);
  if (ch.dtype == MPS_C64)   // complex64 chains: the snapshot widened to complex128 (exact)
    MPS_TRY_HIP(h, launch_convert(s, ch.B, B, (long long)(A.snapB / sizeof(double2)), false));
  else
    MPS_TRY_HIP(h, hipMemcpyAsync(B, ch.B, A.snapB, hipMemcpyDeviceToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(lam, ch.lam, A.snapL, hipMemcpyDeviceToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(chi, ch.chi, A.snapC, hipMemcpyDeviceToDevice, s));
  return MPS_OK;
}

// The adjoint of a TEBD2 (order 2) or TEBD4 (order 4) run for the weighted loss
//   sum_i w1[i] <op1 at i> + sum_b w2[b] <op2 on bond b>   (host weights);
// obs_dev (optional) receives the 2L-1 final observables, loss_dev (optional)
// the loss, dJ_dev the gradient.
// With dB_seed and dLam_seed (device; the chain's B and lam layouts) the
// forward is not run: the arena already holds its checkpoints (written by
// mps_tebd_step_ex with MPS_CHECKPOINT), the chain holds the final state, and
// the reverse pass starts from these state cotangents instead of the loss.
static mps_status tebd_grad_impl(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* h0,
                                 int order, double dt, int32_t n_steps, double eps_local, double eta, const void* op1,
                                 const double* w1, const void* op2, const double* w2, void* arena_ptr,
                                 size_t arena_bytes, double* obs_dev, double* loss_dev, double* dJ_dev,
                                 const void* dB_seed = nullptr, const double* dLam_seed = nullptr) {
  if (!h) return MPS_ERR_INVALID;
  const bool seeded = dB_seed != nullptr;
  if (seeded && !dLam_seed) return mps_fail(h, MPS_ERR_INVALID, "null lambda cotangent");
  if (!chain || !h0 || (!seeded && (!op1 || !op2 || !w1 || !w2)) || !dJ_dev || !arena_ptr)
    return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  const mps_chain_desc ch = *chain;
  if (ch.dtype != MPS_C128 && ch.dtype != MPS_C64) return mps_fail(h, MPS_ERR_INVALID, "bad chain dtype");
  // complex64 chains: the forward (and its re-runs) in the chain's precision,
  // the reverse pass in complex128 on the states widened exactly
  const bool c64 = ch.dtype == MPS_C64;
  if (ch.L < 2 || ch.d < 1 || ch.d > 5 || ch.chi_max < 1) return mps_fail(h, MPS_ERR_SHAPE, "bad chain shape");
  if ((int64_t)ch.d * ch.chi_max > 2560) return mps_fail(h, MPS_ERR_CAPACITY, "d*chi_max is limited to 2560");
  if (!seeded)
    for (int i = 0; i < ch.L; ++i)
      if (!std::isfinite(w1[i]) || (i + 1 < ch.L && !std::isfinite(w2[i])))
        return mps_fail(h, MPS_ERR_INVALID, "non-finite loss weight");
  if (n_steps < 1) return mps_fail(h, MPS_ERR_INVALID, "n_steps must be >= 1");
  if (!(eta >= 0.0) || !(dt > 0.0) || !(eps_local >= 0.0)) return mps_fail(h, MPS_ERR_INVALID, "bad dt, eps or eta");
  if (order != 2 && order != 4) return mps_fail(h, MPS_ERR_INVALID, "the adjoint covers TEBD2 and TEBD4 runs");
  const int L = ch.L, d = ch.d, cm = ch.chi_max, dd = d * d;
  // the layers of one step (parity, time-step class) and the classes' time
  // steps, as the forward schedules them (Strang: odd tau/2, even tau, odd
  // tau/2; TEBD4: five Strang steps of weights p, p, 1 - 4p, p, p)
  std::vector<double> taus;
  std::vector<std::pair<int, int>> lys;
  if (order == 2) {
    taus = {0.5 * dt, dt};
    lys = {{0, 0}, {1, 1}, {0, 0}};
  } else {
    const double pw = 1.0 / (4.0 - std::cbrt(4.0));
    taus = {0.5 * pw * dt, pw * dt, 0.5 * (1.0 - 4.0 * pw) * dt, (1.0 - 4.0 * pw) * dt};
    const int cls5[5] = {0, 0, 2, 0, 0};
    for (int st = 0; st < 5; ++st) {
      lys.push_back({0, cls5[st]});
      lys.push_back({1, cls5[st] + 1});
      lys.push_back({0, cls5[st]});
    }
  }
  const int n_lay = (int)lys.size(), n_cls = (int)taus.size();
  const GradArena A(L, d, cm, n_steps, n_lay, n_cls);
  if (arena_bytes < A.total)
    return mps_fail(h, MPS_ERR_CAPACITY, "arena smaller than mps_tebd_grad_arena_bytes()");
  hipStream_t s = (hipStream_t)stream;
  Ctx c{h, s};
  const size_t site_el = (size_t)cm * d * cm;
  char* arena = (char*)arena_ptr;
  char* lay = arena + A.oLay;
  double2* Bbar = (double2*)(arena + A.oBb);
  double* lbar = (double*)(arena + A.oLb);
  double2* Gt = (double2*)(arena + A.oG);
  double2* dG = (double2*)(arena + A.oDG);
  auto bbar = [&](int i) { return Bbar + (size_t)i * site_el; };
  auto Gp = [&](int k, int b) { return Gt + ((size_t)k * (L - 1) + b) * dd * dd; };
  auto dGp = [&](int k, int b) { return dG + ((size_t)k * (L - 1) + b) * dd * dd; };
  auto save = [&](char* dst) -> mps_status {
    double2* B;
    double* lam;
    int32_t* chi;
    A.ptrs(dst, B, lam, chi);
    if (c64)
      MPS_TRY_HIP(h, launch_convert(s, ch.B, B, (long long)L * site_el, false));
    else
      MPS_TRY_HIP(h, hipMemcpyAsync(B, ch.B, A.snapB, hipMemcpyDeviceToDevice, s));
    MPS_TRY_HIP(h, hipMemcpyAsync(lam, ch.lam, A.snapL, hipMemcpyDeviceToDevice, s));
    MPS_TRY_HIP(h, hipMemcpyAsync(chi, ch.chi, A.snapC, hipMemcpyDeviceToDevice, s));
    return MPS_OK;
  };
  auto restore = [&](char* src) -> mps_status {
    double2* B;
    double* lam;
    int32_t* chi;
    A.ptrs(src, B, lam, chi);
    if (c64)   // back to complex64: exact, the snapshot was widened from it
      MPS_TRY_HIP(h, launch_convert(s, B, ch.B, (long long)L * site_el, true));
    else
      MPS_TRY_HIP(h, hipMemcpyAsync(ch.B, B, A.snapB, hipMemcpyDeviceToDevice, s));
    MPS_TRY_HIP(h, hipMemcpyAsync(ch.lam, lam, A.snapL, hipMemcpyDeviceToDevice, s));
    MPS_TRY_HIP(h, hipMemcpyAsync(ch.chi, chi, A.snapC, hipMemcpyDeviceToDevice, s));
    return MPS_OK;
  };
  mps_status r;

  // ---- forward with a checkpoint per step --------------------------------
  if (!seeded) {
    for (int st = 0; st < n_steps; ++st) {
      if ((r = save(arena + A.oCk + (size_t)st * A.snap)) != MPS_OK) return r;
      if ((r = tebd_impl(h, stream, &ch, 1, order, dt, 1, eps_local, 0, 0, n_lay)) != MPS_OK) return r;
    }
    if ((r = save(arena + A.oCk + (size_t)n_steps * A.snap)) != MPS_OK) return r;
  }

  // ---- gates of every class and dG/dJ
  {
    std::vector<GateJob> jobs;
    for (int k = 0; k < n_cls; ++k)
      for (int b = 0; b < L - 1; ++b) {
        GateJob j;
        std::memset(&j, 0, sizeof(j));
        j.h = (const double2*)ch.hbond + (size_t)b * dd * dd;
        j.G64 = nullptr;
        j.G128 = Gp(k, b);
        j.tau = taus[k];
        jobs.push_back(j);
      }
    MPS_TRY_HIP(h, hipMemcpyAsync(arena + A.oGJ, jobs.data(), jobs.size() * sizeof(GateJob), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    MPS_TRY_HIP(h, launch_gates(s, (const GateJob*)(arena + A.oGJ), (int)jobs.size(), dd));
    for (int k = 0; k < n_cls; ++k)
      for (int b = 0; b < L - 1; ++b)
        K1((dgate_kernel<<<1, 256, 0, s>>>((const double2*)h0 + (size_t)b * dd * dd, Gp(k, b), taus[k], dd,
                                            dGp(k, b))));
  }
  MPS_TRY_HIP(h, hipMemsetAsync(dJ_dev, 0, (L - 1) * sizeof(double), s));

  // ---- loss and its cotangents at the final state -------------------------
  GradScratch g;
  if ((r = grad_scratch(h, L, d, cm, g)) != MPS_OK) return r;
  const GradItemBuf& g0 = g.it[0];
  std::vector<int32_t> chi(L + 1);
  MPS_TRY_HIP(h, hipMemcpyAsync(chi.data(), ch.chi, (L + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  // complex64 chains: the final state (or the state cotangent) read through a
  // complex128 copy in the first layer snapshot's B, which the reverse pass
  // overwrites only later
  const double2* Bfin = (const double2*)ch.B;
  const double2* seedB = (const double2*)dB_seed;
  if (c64) {
    double2* tmpB;
    double* tmpL;
    int32_t* tmpC;
    A.ptrs(lay, tmpB, tmpL, tmpC);
    MPS_TRY_HIP(h, launch_convert(s, seeded ? dB_seed : ch.B, tmpB, (long long)L * site_el, false));
    if (seeded)
      seedB = tmpB;
    else
      Bfin = tmpB;
  }
  if (seeded) {
    // the state cotangents as given: site i's block of B (capacity layout
    // [chi_max][d][chi_max]) into the reverse pass's compact [chi_i][d][chi_i+1]
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    K1((fill_zero_kernel<<<g1d((long long)L * site_el), 256, 0, s>>>(Bbar, (long long)L * site_el)));
    for (int i = 0; i < L; ++i)
      K1((site_copy_kernel<<<g1d((long long)chi[i] * d * chi[i + 1]), 256, 0, s>>>(
          seedB + (size_t)i * site_el, bbar(i), chi[i], d, chi[i + 1], cm, 1)));
    MPS_TRY_HIP(h, hipMemcpyAsync(lbar, dLam_seed, (size_t)(L + 1) * cm * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (!seeded) {  // seeding from the loss
  {
    MPS_TRY_HIP(h, launch_observe(s, ch, (const double2*)op1, g.obs, (const double2*)op2, 0, g.obs + L, nullptr));
    std::vector<double> o(2 * L);
    MPS_TRY_HIP(h, hipMemcpyAsync(o.data(), g.obs, (2 * L - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    double loss = 0.0;
    for (int i = 0; i < L; ++i) loss += w1[i] * o[i];
    for (int b = 0; b < L - 1; ++b) loss += w2[b] * o[L + b];
    if (loss_dev) MPS_TRY_HIP(h, hipMemcpyAsync(loss_dev, &loss, sizeof(double), hipMemcpyHostToDevice, s));
    if (obs_dev) MPS_TRY_HIP(h, hipMemcpyAsync(obs_dev, g.obs, (2 * L - 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
  }
  K1((fill_zero_kernel<<<g1d((long long)L * site_el), 256, 0, s>>>(Bbar, (long long)L * site_el)));
  MPS_TRY_HIP(h, hipMemsetAsync(lbar, 0, (L + 1) * cm * sizeof(double), s));
  for (int i = 0; i < L; ++i) {
    if (w1[i] == 0.0) continue;
    // site term w <O1>_i = w sum_a lam_a^2 <B_a|O1|B_a>: B_bar += 2 w lam^2 O1 B, lam_bar += 2 w lam Re<B, O1 B>
    const int a = chi[i], b2 = chi[i + 1];
    K1((site_copy_kernel<<<g1d((long long)a * d * b2), 256, 0, s>>>(Bfin + i * site_el, g0.Bbs, a, d,
                                                                     b2, cm, 1)));
    K1((apply_local_kernel<<<g1d((long long)a * b2), 256, 0, s>>>((const double2*)op1, d, g0.Bbs, g0.T0, a, b2, 0, 0)));
    K1((row_scale_kernel<<<g1d((long long)a * d * b2), 256, 0, s>>>(g0.T0, bbar(i), a * d, b2, ch.lam + (size_t)i * cm,
                                                                     d, 2, 2.0 * w1[i], 1)));
    K1((lam_dot_kernel<<<a, 256, 0, s>>>(g0.Bbs, g0.T0, d, b2, lbar + (size_t)i * cm, ch.lam + (size_t)i * cm,
                                         2.0 * w1[i])));
  }
  {
    // bond terms w <theta|O2|theta>, theta = lam_b B_b B_{b+1}
    for (int b = 0; b < L - 1; ++b) {
      if (w2[b] == 0.0) continue;
      const int chl = chi[b], chm = chi[b + 1], chr = chi[b + 2], m = chl * d, n = d * chr;
      K1((site_copy_kernel<<<g1d((long long)m * chm), 256, 0, s>>>(Bfin + b * site_el, g0.Bbs, chl, d,
                                                                    chm, cm, 1)));
      K1((site_copy_kernel<<<g1d((long long)chm * n), 256, 0, s>>>(Bfin + (b + 1) * site_el, g0.Bns,
                                                                    chm, d, chr, cm, 1)));
      if ((r = gemm128(c, g0.Bbs, chm, 1, 0, g0.Bns, n, 1, 0, g0.T0, n, m, n, chm, 1.0)) != MPS_OK) return r;
      K1((row_scale_kernel<<<g1d((long long)m * n), 256, 0, s>>>(g0.T0, g0.T1, m, n, ch.lam + (size_t)b * cm, d, 1, 1.0,
                                                                  0)));
      K1((apply_local_kernel<<<g1d((long long)chl * chr), 256, 0, s>>>((const double2*)op2, dd, g0.T1, g0.P0, chl, chr,
                                                                        0, 0)));
      // theta_bar = 2 w O2 theta; lam_bar_b += Re<theta_bar, X>; X_bar = lam_b theta_bar
      K1((lam_dot_kernel<<<chl, 256, 0, s>>>(g0.P0, g0.T0, d, n, lbar + (size_t)b * cm, nullptr, 2.0 * w2[b])));
      K1((row_scale_kernel<<<g1d((long long)m * n), 256, 0, s>>>(g0.P0, g0.Pb, m, n, ch.lam + (size_t)b * cm, d, 1,
                                                                  2.0 * w2[b], 0)));
      if ((r = gemm128(c, g0.Pb, n, 1, 0, g0.Bns, 1, n, 1, g0.Y1, chm, m, chm, n, 1.0)) != MPS_OK) return r;
      if ((r = gemm128(c, g0.Bbs, 1, chm, 1, g0.Pb, n, 1, 0, g0.Z, n, chm, n, m, 1.0)) != MPS_OK) return r;
      K1((axpy_kernel<<<g1d((long long)m * chm), 256, 0, s>>>(g0.Y1, bbar(b), (long long)m * chm, 1.0)));
      K1((axpy_kernel<<<g1d((long long)chm * n), 256, 0, s>>>(g0.Z, bbar(b + 1), (long long)chm * n, 1.0)));
    }
  }
  }  // seeding from the loss

  // ---- backward over steps and layers -------------------------------------
  // Every bond of a layer is an independent update: each stage of the reverse
  // pass runs for all bonds of the layer in one launch (bond = grid.y), the
  // layer's residual SVDs as one batch between the two halves.  No per-update
  // host round trip: the sizes that depend on the data (how many discarded
  // directions are resolved, n_k) stay on the device, and the matrices that
  // depend on them are formed at capacity r_cap = min(m, n) with zero rows.
  std::vector<GDesc> gdh;
  std::vector<SGemm> sgh;
  const double abs_saved = h->jac_abs;
  for (int stp = n_steps - 1; stp >= 0; --stp) {
    if ((r = restore(arena + A.oCk + (size_t)stp * A.snap)) != MPS_OK) return r;
    for (int li = 0; li < n_lay; ++li) {
      if ((r = save(lay + (size_t)li * A.snap)) != MPS_OK) return r;
      if ((r = tebd_impl(h, stream, &ch, 1, order, dt, 1, eps_local, 0, li, li + 1)) != MPS_OK) return r;
    }
    if ((r = grad_scratch(h, L, d, cm, g)) != MPS_OK) return r;
    for (int li = n_lay - 1; li >= 0; --li) {
      double2 *SB, *NB;
      double *SL, *NL;
      int32_t *SC, *NC;
      A.ptrs(lay + (size_t)li * A.snap, SB, SL, SC);
      if (li < n_lay - 1) {
        A.ptrs(lay + (size_t)(li + 1) * A.snap, NB, NL, NC);
      } else if (c64) {
        // the state after the step's last layer is the next step's checkpoint
        // (the re-run is deterministic), there in complex128
        A.ptrs(arena + A.oCk + (size_t)(stp + 1) * A.snap, NB, NL, NC);
      } else {
        NB = (double2*)ch.B;
        NL = ch.lam;
        NC = ch.chi;
      }
      std::vector<int32_t> co(L + 1), cn(L + 1);
      MPS_TRY_HIP(h, hipMemcpyAsync(co.data(), SC, (L + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      MPS_TRY_HIP(h, hipMemcpyAsync(cn.data(), NC, (L + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      MPS_TRY_HIP(h, hipStreamSynchronize(s));
      const int par = lys[li].first, cls = lys[li].second;
      std::vector<int> bonds;
      for (int b = par; b < L - 1; b += 2) bonds.push_back(b);
      const int ni = (int)bonds.size();
      // residual matrices of the layer, described for the batched Jacobi
      std::vector<JacMat> hm(ni);
      for (int i = 0; i < ni; ++i) {
        const int b = bonds[i], m = co[b] * d, n = d * co[b + 2], k = cn[b + 1];
        std::memset(&hm[i], 0, sizeof(JacMat));
        hm[i].X = g.it[i].Xj;
        hm[i].rowmap = g.rowmap + (size_t)i * g.m_cap;
        hm[i].nrm2 = g.nrm2 + (size_t)i * g.m_cap;
        hm[i].m = m;
        hm[i].n = n;
        hm[i].ld = n;
        hm[i].nb = jac_nb(m);
        hm[i].kmax = std::max(0, std::min(m, n) - k);
      }
      MPS_TRY_HIP(h, hipMemcpyAsync(g.mat, hm.data(), ni * sizeof(JacMat), hipMemcpyHostToDevice, s));
      MPS_TRY_HIP(h, hipStreamSynchronize(s));
      int nb_cap = 2, mmax = 1;
      for (int i = 0; i < ni; ++i) {
        nb_cap = std::max(nb_cap, hm[i].nb);
        mmax = std::max(mmax, hm[i].m);
      }

      // -- the layer's bond updates, described once for the batched stages
      gdh.assign(ni, GDesc());
      for (int i = 0; i < ni; ++i) {
        const GradItemBuf& q = g.it[i];
        GDesc& x = gdh[i];
        std::memset(&x, 0, sizeof(x));
        const int b = bonds[i];
        x.b = b;
        x.chl = co[b];
        x.chm = co[b + 1];
        x.chr = co[b + 2];
        x.m = x.chl * d;
        x.n = d * x.chr;
        x.k = cn[b + 1];
        x.rc = std::min(x.m, x.n);
        x.cap = x.rc - x.k;
        x.d = d;
        x.cm = cm;
        x.T0 = q.T0; x.T1 = q.T1; x.P0 = q.P0; x.Xj = q.Xj; x.Vh = q.Vh; x.Vb = q.Vb; x.Y1 = q.Y1; x.Z = q.Z;
        x.Y = q.Y; x.Pm = q.Pm; x.Pb = q.Pb; x.T1b = q.T1b; x.T0b = q.T0b; x.Bnew = q.Bnew; x.Bbl = q.Bbl;
        x.Bnl = q.Bnl; x.Bbs = q.Bbs; x.Bns = q.Bns; x.Jv = q.Jv; x.Xm = q.Xm;
        x.dot = q.dot;
        x.sv = q.sv; x.sbar = q.sbar; x.c2 = q.c2; x.kept2 = q.kept2; x.scal = q.scal;
        x.rd = q.rd;
        x.SBb = SB + b * site_el;
        x.SBb1 = SB + (b + 1) * site_el;
        x.NBb = NB + b * site_el;
        x.NBb1 = NB + (b + 1) * site_el;
        x.bbar_b = bbar(b);
        x.bbar_b1 = bbar(b + 1);
        x.lam_b = SL + (size_t)b * cm;
        x.lbar_b = lbar + (size_t)b * cm;
        x.lbar_b1 = lbar + (size_t)(b + 1) * cm;
        x.G = Gp(cls, b);
        x.dG = dGp(cls, b);
        x.mat = g.mat + i;
        x.perm = g.perm + (size_t)i * g.m_cap;
        x.s2 = g.s2 + (size_t)i * g.m_cap;
        x.seld = g.seld + i;
        x.dJ = dJ_dev + b;
      }
      // the products of every stage, one problem per bond (gemm128 argument order)
      sgh.assign((size_t)kGradGemmStages * ni, SGemm());
      int mx[kGradGemmStages] = {0}, nx[kGradGemmStages] = {0};
      for (int i = 0; i < ni; ++i) {
        const GDesc& q = gdh[i];
        const int m = q.m, n = q.n, k = q.k, rc = q.rc, cap = q.cap, chm = q.chm;
        double2* Vd = q.Vh + (size_t)k * n;
        const double* inv_nk = q.scal + 1;
        SGemm st[kGradGemmStages] = {
            sg_make(q.Bbs, chm, 1, 0, q.Bns, n, 1, 0, q.T0, n, m, n, chm),           // 0: theta~
            sg_make(q.P0, n, 1, 0, q.Vh, 1, n, 1, q.Pm, k, m, k, n),                 // 1: theta' V_k
            sg_make(q.Pm, k, 1, 0, q.Vh, n, 1, 0, q.Z, n, m, n, k),                  // 2: projection
            sg_make(Vd, n, 1, 0, q.Vh, 1, n, 1, q.Jv, k, cap, k, n),                 // 3: V_d V_k^dag
            sg_make(q.Jv, k, 1, 0, q.Vh, n, 1, 0, q.Z, n, cap, n, k),                // 4: its projection
            sg_make(q.P0, n, 1, 0, q.Vh, 1, n, 1, q.Pm, rc, m, rc, n),               // 5: P = theta' V
            sg_make(q.T1, 1, n, 1, q.Bbl, k, 1, 0, q.Vb, rc, n, k, m, inv_nk),       // 6: V_bar kept part
            sg_make(q.Vh, n, 1, 0, q.Vb, rc, 1, 0, q.Jv, rc, rc, rc, n),             // 7: Jv = V^dag V_bar
            sg_make(q.Xm, rc, 1, 0, q.Vh, n, 1, 0, q.Y1, n, rc, n, rc),              // 8: Xt V^dag
            sg_make(q.Jv, 1, rc, 1, q.Vh, n, 1, 0, q.Z, n, rc, n, rc),               // 9: Jv^dag V^dag
            sg_make(q.Pm, rc, 1, 0, q.Y, n, 1, 0, q.Pb, n, m, n, rc),                // 10: theta'_bar
            sg_make(q.Bbl, k, 1, 0, q.Vh, n, 1, 0, q.T1b, n, m, n, k, inv_nk),       // 11: B_bar_b' V_k^dag / n_k
            sg_make(q.T0b, n, 1, 0, q.Bns, 1, n, 1, q.bbar_b, chm, m, chm, n),       // 12: B_bar_b
            sg_make(q.Bbs, 1, chm, 1, q.T0b, n, 1, 0, q.bbar_b1, n, chm, n, m)};     // 13: B_bar_{b+1}
        for (int j = 0; j < kGradGemmStages; ++j) {
          sgh[(size_t)j * ni + i] = st[j];
          mx[j] = std::max(mx[j], st[j].M);
          nx[j] = std::max(nx[j], st[j].N);
        }
      }
      // the previous layer's uploads finished at the synchronisation above
      MPS_TRY_HIP(h, hipMemcpyAsync(g.gd, gdh.data(), ni * sizeof(GDesc), hipMemcpyHostToDevice, s));
      MPS_TRY_HIP(h, hipMemcpyAsync(g.sg, sgh.data(), sgh.size() * sizeof(SGemm), hipMemcpyHostToDevice, s));
      int emax = 1, chl_max = 1;
      for (int i = 0; i < ni; ++i) {
        emax = std::max(emax, std::max(gdh[i].m, gdh[i].rc) * std::max(gdh[i].n, gdh[i].rc));
        chl_max = std::max(chl_max, gdh[i].chl);
      }
      const dim3 eg(std::max(1, std::min(1024, (emax + 255) / 256)), ni);
      auto stage = [&](int j) -> hipError_t {
        return launch_sgemm_batched(s, g.sg + (size_t)j * ni, ni, mx[j], nx[j]);
      };
      const GDesc* D = g.gd;

      // -- first half: recompute the update, form the residual theta'(1 - V_k V_k^dag)
      K1((bg_prep_kernel<<<eg, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(0));
      K1((bg_gate_kernel<<<eg, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(1));
      MPS_TRY_HIP(h, stage(2));
      K1((bg_resid_kernel<<<eg, 256, 0, s>>>(D)));

      // -- the layer's residual SVDs, orthogonalised with the smallest absolute tolerance
      MPS_TRY_HIP(h, launch_jac_prep_plain(s, g.mat, ni, h->status_dev));
      h->jac_abs = kJacAbsFloor;
      // the residual batches are many small matrices: no column split
      r = run_jacobi(h, s, g.mat, ni, nb_cap, g.m_cap, g.unc, false, false);
      h->jac_abs = abs_saved;
      if (r != MPS_OK) return r;
      MPS_TRY_HIP(h, launch_select(s, g.mat, ni, g.perm, g.s2, g.m_cap, 0, 0.0, g.sel));

      // -- second half: discarded directions, SVD backward, gate and contraction adjoints
      K1((bg_rd_kernel<<<ni, 256, 0, s>>>(D)));
      K1((bg_rows_kernel<<<eg, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(3));
      MPS_TRY_HIP(h, stage(4));
      K1((bg_reproj_kernel<<<eg, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(5));
      K1((bg_scal_kernel<<<ni, 256, 0, s>>>(D, h->status_dev)));
      MPS_TRY_HIP(h, stage(6));
      K1((bg_addconj_kernel<<<eg, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(7));
      K1((bg_svdx_kernel<<<eg, 256, 0, s>>>(D, eta)));
      MPS_TRY_HIP(h, stage(8));
      MPS_TRY_HIP(h, stage(9));
      K1((bg_svdy_kernel<<<eg, 256, 0, s>>>(D, eta)));
      MPS_TRY_HIP(h, stage(10));
      MPS_TRY_HIP(h, stage(11));
      K1((bg_thetabar_kernel<<<dim3(chl_max, ni), 256, 0, s>>>(D)));
      K1((bg_gatebar_kernel<<<eg, 256, 0, s>>>(D)));
      K1((bg_jbar_kernel<<<ni, 256, 0, s>>>(D)));
      MPS_TRY_HIP(h, stage(12));
      MPS_TRY_HIP(h, stage(13));
      K1((bg_zero_lbar_kernel<<<ni, 256, 0, s>>>(D)));
    }
  }
  // the chain is left in the final state of the forward run
  if ((r = restore(arena + A.oCk + (size_t)n_steps * A.snap)) != MPS_OK) return r;
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  return MPS_OK;
}

extern "C" mps_status mps_tebd_grad(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* h0,
                                    double dt, int32_t n_steps, double eps_local, double eta, const void* op1,
                                    int32_t site, const void* op2, void* arena_ptr, size_t arena_bytes,
                                    double* loss_dev, double* dJ_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!chain || !loss_dev) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (site < 0 || site >= chain->L) return mps_fail(h, MPS_ERR_INVALID, "site out of range");
  std::vector<double> w1(chain->L, 0.0), w2(chain->L - 1, 1.0);
  w1[site] = 1.0;
  return tebd_grad_impl(h, stream, chain, h0, 2, dt, n_steps, eps_local, eta, op1, w1.data(), op2, w2.data(),
                        arena_ptr, arena_bytes, nullptr, loss_dev, dJ_dev);
}

extern "C" mps_status mps_tebd_vjp(mps_handle h, mps_stream stream, const mps_chain_desc* chain, const void* h0,
                                   double dt, int32_t n_steps, double eps_local, double eta, const void* op1,
                                   const double* w_site, const void* op2, const double* w_bond, void* arena_ptr,
                                   size_t arena_bytes, double* obs_dev, double* dJ_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!chain || chain->L < 2) return mps_fail(h, MPS_ERR_INVALID, "null or short chain");
  return tebd_grad_impl(h, stream, chain, h0, 2, dt, n_steps, eps_local, eta, op1, w_site, op2, w_bond, arena_ptr,
                        arena_bytes, obs_dev, nullptr, dJ_dev);
}

extern "C" mps_status mps_tebd_step_vjp(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                                        int32_t n_chains, const void* const* h0, void* ckpt_arena, size_t ckpt_bytes,
                                        const void* const* dB_final, const double* const* dLam_final,
                                        double* dJ_dev, double eta) {
  if (!h) return MPS_ERR_INVALID;
  if (!chains || n_chains < 1 || !h0 || !ckpt_arena || !dB_final || !dLam_final || !dJ_dev)
    return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (!(eta >= 0.0)) return mps_fail(h, MPS_ERR_INVALID, "eta must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  CkptHeader hd;
  MPS_TRY_HIP(h, hipMemcpyAsync(&hd, ckpt_arena, sizeof(hd), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  if (hd.magic != kCkptMagic || hd.n_chains != n_chains || hd.shape_sum != ckpt_shape_sum(chains, n_chains))
    return mps_fail(h, MPS_ERR_INVALID, "the arena was not written by mps_tebd_step_ex for these chains");
  if (hd.order != 2 && hd.order != 4)
    return mps_fail(h, MPS_ERR_INVALID, "the adjoint covers TEBD2 and TEBD4 (order 2 and 4) runs");
  if (ckpt_bytes < mps_tebd_ckpt_bytes(chains, n_chains, hd.n_steps))
    return mps_fail(h, MPS_ERR_CAPACITY, "arena smaller than mps_tebd_ckpt_bytes()");
  int l_max = 2;
  for (int c = 0; c < n_chains; ++c) l_max = std::max(l_max, (int)chains[c].L);
  MPS_TRY_HIP(h, hipMemsetAsync(dJ_dev, 0, (size_t)n_chains * (l_max - 1) * sizeof(double), s));
  for (int c = 0; c < n_chains; ++c) {
    if (!h0[c] || !dB_final[c] || !dLam_final[c]) return mps_fail(h, MPS_ERR_INVALID, "null per-chain pointer");
    char* block = (char*)ckpt_arena + ckpt_block_offset(chains, c, hd.n_steps);
    const size_t bytes = ckpt_block_bytes(chains[c], hd.n_steps);
    mps_status r = tebd_grad_impl(h, stream, chains + c, h0[c], hd.order, hd.dt, hd.n_steps, hd.eps_local, eta, nullptr,
                                  nullptr, nullptr, nullptr, block, bytes, nullptr, nullptr,
                                  dJ_dev + (size_t)c * (l_max - 1), dB_final[c], dLam_final[c]);
    if (r != MPS_OK) return r;
  }
  return MPS_OK;
}

// ---------------------------------------------------------------------------
// Single-update vector-Jacobian products (the pieces of the reverse pass above)
// ---------------------------------------------------------------------------
namespace {

// dG[e] = sum_{a,c} Tb[a][uv][c] conj(T[a][st][c]),  e = uv * D + st; one workgroup per entry
__global__ __launch_bounds__(256) void gate_bar_kernel(const double2* __restrict__ Tb, const double2* __restrict__ T,
                                                       int P, int D, int R, double2* dG) {
  __shared__ double2 red[4];
  const int uv = blockIdx.x / D, st = blockIdx.x % D;
  double2 acc = make_double2(0.0, 0.0);
  for (long long e = threadIdx.x; e < (long long)P * R; e += blockDim.x) {
    const long long a = e / R, c = e % R;
    const double2 x = Tb[(a * D + uv) * R + c], y = T[(a * D + st) * R + c];
    acc.x += x.x * y.x + x.y * y.y;     // x conj(y)
    acc.y += x.y * y.x - x.x * y.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    acc.x += __shfl_xor(acc.x, o);
    acc.y += __shfl_xor(acc.y, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    dG[blockIdx.x] = make_double2(red[0].x + red[1].x + red[2].x + red[3].x, red[0].y + red[1].y + red[2].y + red[3].y);
}

__global__ void sqrt_kernel(const double* __restrict__ a, double* b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = sqrt(fmax(a[i], 0.0));
}

// Cotangents of the kept factors with U written as theta V_k S^-1 (U_bar
// folded into those of V_k and S).  One workgroup per kept j:
//   w_j = s_j / (s_j^2 + eta),  Wt = U_bar^dag theta (k x n),
//   Vbar[c][j] = conj(Vh_bar[j][c] + w_j Wt[j][c])           (j < k; other columns 0)
//   sbar_j = S_bar_j - w_j^2 Re sum_c Wt[j][c] conj(Vh[j][c])
// Null Vh_bar, S_bar or Wt count as zero.
__global__ __launch_bounds__(256) void trunc_bar_kernel(const double2* __restrict__ vhb, const double* __restrict__ sb,
                                                        const double2* __restrict__ Wt, const double2* __restrict__ Vh,
                                                        const double* __restrict__ s, double eta, int n, int r,
                                                        double2* Vb, double* sbar) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const double w = s[j] / (s[j] * s[j] + eta);
  double acc = 0.0;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const long long e = (long long)j * n + c;
    double2 v = vhb ? vhb[e] : make_double2(0.0, 0.0);
    if (Wt) {
      const double2 t = Wt[e], q = Vh[e];
      v = make_double2(v.x + w * t.x, v.y + w * t.y);
      acc += t.x * q.x + t.y * q.y;
    }
    Vb[(long long)c * r + j] = make_double2(v.x, -v.y);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sbar[j] = (sb ? sb[j] : 0.0) - w * w * (red[0] + red[1] + red[2] + red[3]);
}

// out[i][j] = in[i * ld + j] * s_j / (s_j^2 + eta)   (rows x k)
__global__ void col_inv_scale_kernel(const double2* __restrict__ in, int ld, int rows, int k,
                                     const double* __restrict__ s, double eta, double2* out) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)rows * k;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / k;
    const int j = (int)(e % k);
    const double w = s[j] / (s[j] * s[j] + eta);
    const double2 v = in[i * ld + j];
    out[e] = make_double2(w * v.x, w * v.y);
  }
}

}  // namespace

extern "C" mps_status mps_theta_gate_vjp(mps_handle h, mps_stream stream, const void* Bl, const void* Br,
                                         const double* lam_l, const void* G, const void* theta_bar, int32_t chl,
                                         int32_t d, int32_t chm, int32_t chr, void* dBl, void* dBr, double* dlam_l,
                                         void* dG) {
  if (!h) return MPS_ERR_INVALID;
  if (!Bl || !Br || !lam_l || !G || !theta_bar || !dBl || !dBr || !dlam_l || !dG)
    return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (chl < 1 || chm < 1 || chr < 1 || d < 1 || d > 5) return mps_fail(h, MPS_ERR_SHAPE, "bad dimensions");
  if ((int64_t)d * chl > 4096 || (int64_t)d * chr > 4096 || chm > 4096)
    return mps_fail(h, MPS_ERR_CAPACITY, "d*chi and chi are limited to 4096");
  const int dd = d * d, m = chl * d, n = d * chr;
  const size_t mn = (size_t)m * n;
  WsPlan p;
  const size_t o0 = p.take<double2>(mn), o1 = p.take<double2>(mn), o2 = p.take<double2>(mn),
               o3 = p.take<double2>(mn);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Ctx c{h, s};
  double2* T0 = (double2*)(h->ws + o0);  // theta~ = Bl Br
  double2* T1 = (double2*)(h->ws + o1);  // theta~' = G theta~
  double2* T2 = (double2*)(h->ws + o2);  // theta~'_bar = lam theta'_bar
  double2* T3 = (double2*)(h->ws + o3);  // theta~_bar = G^dag theta~'_bar
  mps_status r;
  if ((r = gemm128(c, Bl, chm, 1, 0, Br, n, 1, 0, T0, n, m, n, chm, 1.0)) != MPS_OK) return r;
  K1((apply_local_kernel<<<g1d((long long)chl * chr), 256, 0, s>>>((const double2*)G, dd, T0, T1, chl, chr, 0, 0)));
  MPS_TRY_HIP(h, hipMemsetAsync(dlam_l, 0, (size_t)chl * sizeof(double), s));
  K1((lam_dot_kernel<<<chl, 256, 0, s>>>((const double2*)theta_bar, T1, d, n, dlam_l, nullptr, 1.0)));
  K1((row_scale_kernel<<<g1d((long long)mn), 256, 0, s>>>((const double2*)theta_bar, T2, m, n, lam_l, d, 1, 1.0, 0)));
  K1((gate_bar_kernel<<<dd * dd, 256, 0, s>>>(T2, T0, chl, dd, chr, (double2*)dG)));
  K1((apply_local_kernel<<<g1d((long long)chl * chr), 256, 0, s>>>((const double2*)G, dd, T2, T3, chl, chr, 1, 0)));
  if ((r = gemm128(c, T3, n, 1, 0, Br, 1, n, 1, dBl, chm, m, chm, n, 1.0)) != MPS_OK) return r;
  if ((r = gemm128(c, Bl, 1, chm, 1, T3, n, 1, 0, dBr, n, chm, n, m, 1.0)) != MPS_OK) return r;
  return MPS_OK;
}

extern "C" mps_status mps_truncate_vjp(mps_handle h, mps_stream stream, const void* theta, int64_t m64, int64_t n64,
                                       int32_t k, const double* S, const void* Vh, const void* U_bar, int64_t ld_ubar,
                                       const double* S_bar, const void* Vh_bar, double eta, void* theta_bar) {
  if (!h) return MPS_ERR_INVALID;
  if (!theta || !S || !Vh || !theta_bar) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (m64 < 1 || n64 < 1 || k < 1 || k > std::min(m64, n64)) return mps_fail(h, MPS_ERR_SHAPE, "bad dimensions");
  if (U_bar && ld_ubar < k) return mps_fail(h, MPS_ERR_SHAPE, "ld_ubar < k");
  if (m64 > 2560 || n64 > 2560) return mps_fail(h, MPS_ERR_CAPACITY, "m and n are limited to 2560");
  if (!(eta >= 0.0)) return mps_fail(h, MPS_ERR_INVALID, "eta must be >= 0");
  const int m = (int)m64, n = (int)n64, rc = std::min(m, n), cap = rc - k;
  const size_t mn = (size_t)m * n;
  WsPlan p;
  const size_t oP = p.take<double2>((size_t)m * rc), oZ = p.take<double2>(mn), oR = p.take<double2>(mn),
               oV = p.take<double2>((size_t)rc * n), oVb = p.take<double2>((size_t)n * rc),
               oJ = p.take<double2>((size_t)rc * rc), oX = p.take<double2>((size_t)rc * rc),
               oY1 = p.take<double2>((size_t)rc * n), oY = p.take<double2>((size_t)rc * n),
               oZ2 = p.take<double2>((size_t)rc * n), oJd = p.take<double2>((size_t)rc * rc),
               oW = p.take<double2>((size_t)k * n), oUs = p.take<double2>((size_t)m * k);
  const size_t oc2 = p.take<double>(rc), osv = p.take<double>(rc), okept = p.take<double>(rc),
               osb = p.take<double>(rc);
  const size_t oMat = p.take<JacMat>(1), oSel = p.take<SelOut>(1), oSeld = p.take<SelOut>(1);
  const size_t oRm = p.take<int32_t>(m), oPm = p.take<int32_t>(m), oS2 = p.take<double>(m), oNr = p.take<double>(m),
               oUnc = p.take<int32_t>(8), oRd = p.take<int32_t>(1);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Ctx c{h, s};
  char* ws = h->ws;
  double2 *P = (double2*)(ws + oP), *Z = (double2*)(ws + oZ), *R = (double2*)(ws + oR), *Vf = (double2*)(ws + oV),
          *Vb = (double2*)(ws + oVb), *Jv = (double2*)(ws + oJ), *Xm = (double2*)(ws + oX),
          *Y1 = (double2*)(ws + oY1), *Y = (double2*)(ws + oY), *Z2 = (double2*)(ws + oZ2), *Jd = (double2*)(ws + oJd),
          *Wt = (double2*)(ws + oW), *Us = (double2*)(ws + oUs);
  double *c2 = (double*)(ws + oc2), *sv = (double*)(ws + osv), *kept2 = (double*)(ws + okept),
         *sbar = (double*)(ws + osb);
  JacMat* mat = (JacMat*)(ws + oMat);
  SelOut *sel = (SelOut*)(ws + oSel), *seld = (SelOut*)(ws + oSeld);
  mps_status r;
  // V rows: the kept rows Vh, then the resolved discarded directions, then zeros
  K1((fill_zero_kernel<<<g1d((long long)rc * n), 256, 0, s>>>(Vf, (long long)rc * n)));
  MPS_TRY_HIP(h, hipMemcpyAsync(Vf, Vh, (size_t)k * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
  if ((r = gemm128(c, theta, n, 1, 0, Vf, 1, n, 1, P, k, m, k, n, 1.0)) != MPS_OK) return r;
  K1((colnorm2_kernel<<<g1d(k), 256, 0, s>>>(P, m, k, kept2)));
  if (cap > 0) {
    // residual theta (1 - V_k V_k^dag), orthogonalised with the smallest
    // absolute tolerance: its rows that carry weight give the discarded directions
    if ((r = gemm128(c, P, k, 1, 0, Vf, n, 1, 0, Z, n, m, n, k, 1.0)) != MPS_OK) return r;
    MPS_TRY_HIP(h, hipMemcpyAsync(R, theta, mn * sizeof(double2), hipMemcpyDeviceToDevice, s));
    K1((axpy_kernel<<<g1d((long long)mn), 256, 0, s>>>(Z, R, (long long)mn, -1.0)));
    JacMat hm;
    std::memset(&hm, 0, sizeof(hm));
    hm.X = R;
    hm.rowmap = (int32_t*)(ws + oRm);
    hm.nrm2 = (double*)(ws + oNr);
    hm.m = m;
    hm.n = n;
    hm.ld = n;
    hm.nb = jac_nb(m);
    hm.kmax = cap;
    MPS_TRY_HIP(h, hipMemcpyAsync(mat, &hm, sizeof(hm), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    MPS_TRY_HIP(h, launch_jac_prep_plain(s, mat, 1, h->status_dev));
    const double abs_saved = h->jac_abs;
    h->jac_abs = kJacAbsFloor;
    r = run_jacobi(h, s, mat, 1, hm.nb, m, (int32_t*)(ws + oUnc), false, true);
    h->jac_abs = abs_saved;
    if (r != MPS_OK) return r;
    MPS_TRY_HIP(h, launch_select(s, mat, 1, (int32_t*)(ws + oPm), (double*)(ws + oS2), m, 0, 0.0, sel));
    K1((grad_rd_kernel<<<1, 256, 0, s>>>((double*)(ws + oS2), kept2, m, k, cap, 1e-26, seld, (int32_t*)(ws + oRd))));
    double2* Vd = Vf + (size_t)k * n;
    MPS_TRY_HIP(h, launch_write_rows(s, mat, (int32_t*)(ws + oPm), (double*)(ws + oS2), seld, Vd, n, 0, true));
    // project them once more against V_k
    if ((r = gemm128(c, Vd, n, 1, 0, Vf, 1, n, 1, Jd, k, cap, k, n, 1.0)) != MPS_OK) return r;
    if ((r = gemm128(c, Jd, k, 1, 0, Vf, n, 1, 0, Z2, n, cap, n, k, 1.0)) != MPS_OK) return r;
    K1((axpy_kernel<<<g1d((long long)cap * n), 256, 0, s>>>(Z2, Vd, (long long)cap * n, -1.0)));
  }
  // P = theta V (m x rc); s_j = |P_j| for the discarded j, the forward's S for the kept
  if ((r = gemm128(c, theta, n, 1, 0, Vf, 1, n, 1, P, rc, m, rc, n, 1.0)) != MPS_OK) return r;
  K1((colnorm2_kernel<<<g1d(rc), 256, 0, s>>>(P, m, rc, c2)));
  K1((sqrt_kernel<<<g1d(rc), 256, 0, s>>>(c2, sv, rc)));
  MPS_TRY_HIP(h, hipMemcpyAsync(sv, S, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, s));
  // cotangents of V and S (U_bar folded in), the backward matrices, theta_bar = P Y
  if (U_bar && (r = gemm128(c, U_bar, 1, ld_ubar, 1, theta, n, 1, 0, Wt, n, k, n, m, 1.0)) != MPS_OK) return r;
  K1((fill_zero_kernel<<<g1d((long long)n * rc), 256, 0, s>>>(Vb, (long long)n * rc)));
  K1((trunc_bar_kernel<<<k, 256, 0, s>>>((const double2*)Vh_bar, S_bar, U_bar ? Wt : nullptr, Vf, sv, eta, n, rc,
                                          Vb, sbar)));
  if ((r = gemm128(c, Vf, n, 1, 0, Vb, rc, 1, 0, Jv, rc, rc, rc, n, 1.0)) != MPS_OK) return r;
  K1((svd_x_kernel<<<g1d((long long)rc * rc), 256, 0, s>>>(Jv, sv, sbar, rc, k, eta, Xm)));
  if ((r = gemm128(c, Xm, rc, 1, 0, Vf, n, 1, 0, Y1, n, rc, n, rc, 1.0)) != MPS_OK) return r;
  if ((r = gemm128(c, Jv, 1, rc, 1, Vf, n, 1, 0, Z2, n, rc, n, rc, 1.0)) != MPS_OK) return r;
  K1((svd_y_kernel<<<g1d((long long)rc * n), 256, 0, s>>>(Y1, Z2, Vb, sv, rc, k, n, eta, Y)));
  if ((r = gemm128(c, P, rc, 1, 0, Y, n, 1, 0, theta_bar, n, m, n, rc, 1.0)) != MPS_OK) return r;
  if (U_bar) {
    // theta_bar += U_bar diag(w) V_k^dag, the direct term of U = theta V_k S^-1
    K1((col_inv_scale_kernel<<<g1d((long long)m * k), 256, 0, s>>>((const double2*)U_bar, (int)ld_ubar, m, k, sv, eta,
                                                                     Us)));
    if ((r = gemm128(c, Us, k, 1, 0, Vf, n, 1, 0, Z, n, m, n, k, 1.0)) != MPS_OK) return r;
    K1((axpy_kernel<<<g1d((long long)mn), 256, 0, s>>>(Z, (double2*)theta_bar, (long long)mn, 1.0)));
  }
  return MPS_OK;
}
