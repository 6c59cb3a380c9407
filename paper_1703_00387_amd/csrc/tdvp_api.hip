// Host drivers of the local Krylov path: structured H_eff apply, Lanczos
// exponential, environment updates and the two-site TDVP sweep.
//
// Two-site TDVP (Sec. "Time-dependent variational principle"; the method of
// the cited Haegeman et al. work, symmetric second order): a left-to-right
// half-sweep with tau = dt/2 evolves each two-site tensor forward with the
// Lanczos exponential of H2_eff, splits it by the FP64 truncated SVD (A_b = U,
// C = S V^dag), updates the left environment and evolves C backward with
// H1_eff (except after the last bond); the right-to-left half-sweep mirrors
// it.  With the orthogonality centre inside the two sites the Krylov vectors
// and their sum stay local (App. "Details of the Krylov method").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace {

struct HeffBufs {
  void* X1;
  void* X2;
  void* X3;
  void* Wm1;
  void* Wm2;
};

struct KryBufs {
  double2* V;      // (n_max+1) vectors of length N
  long long ldv;   // capacity of one vector
  double2* r;
  void* xin;       // dtype copies for the complex64 apply
  void* yout;
  double2* dots;   // 32
  double2* part;   // kMdotBlocks * 32 shares of the overlaps
  double* alpha;   // 32
  double* beta;    // 32
  double2* u;      // 32
  double* err;     // 1
  HeffBufs hb;
};

size_t esize(bool c128) { return c128 ? sizeof(double2) : sizeof(float2); }

// y = H_eff x (two-site when W2 != null, else one-site); all buffers in dtype.
mps_status heff_apply_int(mps_handle h, hipStream_t s, bool c128, const void* L, const void* W1, const void* W2,
                          const void* R, const void* x, void* y, int chl, int d1, int d2, int chr, int wl, int wm,
                          int wr, HeffBufs& b) {
  const bool two = W2 != nullptr;
  SGemm g;
  std::memset(&g, 0, sizeof(g));
  // S1: X1[(a',beta)][rest] = L[(a',beta)][a] x[a][rest]
  const long long rest = two ? (long long)d1 * d2 * chr : (long long)d1 * chr;
  g.A = L; g.rsA = chl; g.csA = 1;
  g.B = x; g.rsB = rest; g.csB = 1;
  g.C = b.X1; g.rsC = rest; g.csC = 1;
  g.M = chl * wl; g.K = chl; g.N = (int)rest; g.alpha = 1.0;
  MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  if (two) {
    // S2: X2[a'][g][s'][t][c] = sum W1[b][g][s'][s] X1[a'][b][s][t][c]
    MPS_TRY_HIP(h, launch_wmix_build(s, W1, b.Wm1, wm, d1, wl, d1, d1 * d1, d1, wm * d1 * d1, 1, c128));
    MixDesc m2;
    m2.P1 = chl; m2.P2 = d2; m2.R = chr; m2.Q1 = wl; m2.Q2 = d1; m2.O1 = wm; m2.O2 = d1;
    m2.is_o1 = (long long)wl * d1 * d2 * chr; m2.is_o2 = chr; m2.is_q1 = (long long)d1 * d2 * chr;
    m2.is_q2 = (long long)d2 * chr; m2.is_r = 1;
    m2.os_o1 = (long long)wm * d1 * d2 * chr; m2.os_o2 = chr; m2.os_q1 = (long long)d1 * d2 * chr;
    m2.os_q2 = (long long)d2 * chr; m2.os_r = 1;
    MPS_TRY_HIP(h, launch_mix(s, m2, b.X1, b.Wm1, b.X2, c128));
    // S3: X3[a'][s'][t'][e][c] = sum W2[g][e][t'][t] X2[a'][g][s'][t][c]
    MPS_TRY_HIP(h, launch_wmix_build(s, W2, b.Wm2, d2, wr, wm, d2, d2, d2 * d2, wr * d2 * d2, 1, c128));
    MixDesc m3;
    m3.P1 = chl; m3.P2 = d1; m3.R = chr; m3.Q1 = wm; m3.Q2 = d2; m3.O1 = d2; m3.O2 = wr;
    m3.is_o1 = (long long)wm * d1 * d2 * chr; m3.is_o2 = (long long)d2 * chr; m3.is_q1 = (long long)d1 * d2 * chr;
    m3.is_q2 = chr; m3.is_r = 1;
    m3.os_o1 = (long long)d1 * d2 * wr * chr; m3.os_o2 = (long long)d2 * wr * chr; m3.os_q1 = (long long)wr * chr;
    m3.os_q2 = chr; m3.os_r = 1;
    MPS_TRY_HIP(h, launch_mix(s, m3, b.X2, b.Wm2, b.X3, c128));
    // S4: y[(a',s',t')][c'] = sum_(e,c) X3[(a',s',t')][(e,c)] R[c'][(e,c)]
    std::memset(&g, 0, sizeof(g));
    g.A = b.X3; g.rsA = (long long)wr * chr; g.csA = 1;
    g.B = R; g.rsB = 1; g.csB = (long long)wr * chr;
    g.C = y; g.rsC = chr; g.csC = 1;
    g.M = chl * d1 * d2; g.K = wr * chr; g.N = chr; g.alpha = 1.0;
    MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  } else {
    // S2: X2[a'][s'][g][c] = sum W[b][g][s'][s] X1[a'][b][s][c]   (wm = right MPO dim)
    MPS_TRY_HIP(h, launch_wmix_build(s, W1, b.Wm1, d1, wm, wl, d1, d1, d1 * d1, wm * d1 * d1, 1, c128));
    MixDesc m2;
    m2.P1 = chl; m2.P2 = 1; m2.R = chr; m2.Q1 = wl; m2.Q2 = d1; m2.O1 = d1; m2.O2 = wm;
    m2.is_o1 = (long long)wl * d1 * chr; m2.is_o2 = 0; m2.is_q1 = (long long)d1 * chr; m2.is_q2 = chr; m2.is_r = 1;
    m2.os_o1 = (long long)d1 * wm * chr; m2.os_o2 = 0; m2.os_q1 = (long long)wm * chr; m2.os_q2 = chr; m2.os_r = 1;
    MPS_TRY_HIP(h, launch_mix(s, m2, b.X1, b.Wm1, b.X2, c128));
    // S3: y[(a',s')][c'] = sum_(g,c) X2[(a',s')][(g,c)] R[c'][(g,c)]
    std::memset(&g, 0, sizeof(g));
    g.A = b.X2; g.rsA = (long long)wm * chr; g.csA = 1;
    g.B = R; g.rsB = 1; g.csB = (long long)wm * chr;
    g.C = y; g.rsC = chr; g.csC = 1;
    g.M = chl * d1; g.K = wm * chr; g.N = chr; g.alpha = 1.0;
    MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  }
  return MPS_OK;
}

// Left environment: Lo[a'][b'][c'] = sum conj(A[a][s'][a']) Li[a][b][c] W[b][b'][s'][s] A[c][s][c']
mps_status env_left_int(mps_handle h, hipStream_t s, bool c128, const void* Li, const void* A, const void* W,
                        void* Lo, int chi, int d, int chi2, int w, int w2, HeffBufs& b) {
  SGemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = Li; g.rsA = chi; g.csA = 1;
  g.B = A; g.rsB = (long long)d * chi2; g.csB = 1;
  g.C = b.X1; g.rsC = (long long)d * chi2; g.csC = 1;
  g.M = chi * w; g.K = chi; g.N = d * chi2; g.alpha = 1.0;
  MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  MPS_TRY_HIP(h, launch_wmix_build(s, W, b.Wm1, d, w2, w, d, d, d * d, w2 * d * d, 1, c128));
  MixDesc m;
  m.P1 = chi; m.P2 = 1; m.R = chi2; m.Q1 = w; m.Q2 = d; m.O1 = d; m.O2 = w2;
  m.is_o1 = (long long)w * d * chi2; m.is_o2 = 0; m.is_q1 = (long long)d * chi2; m.is_q2 = chi2; m.is_r = 1;
  m.os_o1 = (long long)d * w2 * chi2; m.os_o2 = 0; m.os_q1 = (long long)w2 * chi2; m.os_q2 = chi2; m.os_r = 1;
  MPS_TRY_HIP(h, launch_mix(s, m, b.X1, b.Wm1, b.X2, c128));
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.rsA = 1; g.csA = chi2; g.conjA = 1;
  g.B = b.X2; g.rsB = (long long)w2 * chi2; g.csB = 1;
  g.C = Lo; g.rsC = (long long)w2 * chi2; g.csC = 1;
  g.M = chi2; g.K = chi * d; g.N = w2 * chi2; g.alpha = 1.0;
  MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  return MPS_OK;
}

// Right environment: Ro[a'][b][c'] = sum conj(B[a'][t'][a]) W[b][b'][t'][t] Ri[a][b'][c] B[c'][t][c]
// B = [chi2][d][chi] (chi2 = new left dimension), Ri = [chi][w2][chi], W = [w][w2][d][d]
mps_status env_right_int(mps_handle h, hipStream_t s, bool c128, const void* Ri, const void* B, const void* W,
                         void* Ro, int chi, int d, int chi2, int w, int w2, HeffBufs& b) {
  SGemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = B; g.rsA = chi; g.csA = 1;
  g.B = Ri; g.rsB = 1; g.csB = chi;
  g.C = b.X1; g.rsC = (long long)chi * w2; g.csC = 1;
  g.M = chi2 * d; g.K = chi; g.N = chi * w2; g.alpha = 1.0;
  MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  // T2[t'][a][b][c'] = sum_(t,b') W[b][b'][t'][t] T1[c'][t][a][b']
  MPS_TRY_HIP(h, launch_wmix_build(s, W, b.Wm1, d, w, d, w2, d, w2 * d * d, 1, d * d, c128));
  MixDesc m;
  m.P1 = chi2; m.P2 = chi; m.R = 1; m.Q1 = d; m.Q2 = w2; m.O1 = d; m.O2 = w;
  m.is_o1 = (long long)d * chi * w2; m.is_o2 = w2; m.is_q1 = (long long)chi * w2; m.is_q2 = 1; m.is_r = 0;
  m.os_o1 = 1; m.os_o2 = (long long)w * chi2; m.os_q1 = (long long)chi * w * chi2; m.os_q2 = chi2; m.os_r = 0;
  MPS_TRY_HIP(h, launch_mix(s, m, b.X1, b.Wm1, b.X2, c128));
  std::memset(&g, 0, sizeof(g));
  g.A = B; g.rsA = (long long)d * chi; g.csA = 1; g.conjA = 1;
  g.B = b.X2; g.rsB = (long long)w * chi2; g.csB = 1;
  g.C = Ro; g.rsC = (long long)w * chi2; g.csC = 1;
  g.M = chi2; g.K = d * chi; g.N = w * chi2; g.alpha = 1.0;
  MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
  return MPS_OK;
}

// x <- exp(-i tau H_eff) x by Lanczos with full re-orthogonalisation.
// x is complex128 of length N; H_eff is applied in dtype.
mps_status krylov_int(mps_handle h, hipStream_t s, bool c128, const void* L, const void* W1, const void* W2,
                      const void* R, double2* x, int chl, int d1, int d2, int chr, int wl, int wm, int wr,
                      double tau_re, double tau_im, int n_max, double tol, int* n_used, double* err_out, bool* conv,
                      KryBufs& k) {
  const long long N = (long long)chl * d1 * (W2 ? d2 : 1) * chr;
  double2 hd[32];
  MPS_TRY_HIP(h, launch_zero(s, (double*)k.dots, 64));
  MPS_TRY_HIP(h, launch_mdot(s, x, N, 1, x, N, k.dots, k.part));
  MPS_TRY_HIP(h, hipMemcpyAsync(hd, k.dots, sizeof(double2), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  const double nrm = std::sqrt(std::max(hd[0].x, 0.0));
  *n_used = 0;
  *err_out = 0.0;
  *conv = true;
  if (!(nrm > 0.0)) return MPS_OK;
  MPS_TRY_HIP(h, launch_scale_inv_sqrt(s, x, k.V, N, &k.dots[0].x));
  std::vector<double> al, be;
  int n = 0;
  double err = 0.0;
  bool ok = false;
  for (int j = 0; j < n_max; ++j) {
    double2* vj = k.V + (size_t)j * k.ldv;
    if (c128) {
      mps_status st = heff_apply_int(h, s, true, L, W1, W2, R, vj, k.r, chl, d1, d2, chr, wl, wm, wr, k.hb);
      if (st != MPS_OK) return st;
    } else {
      MPS_TRY_HIP(h, launch_convert(s, vj, k.xin, N, true));
      mps_status st = heff_apply_int(h, s, false, L, W1, W2, R, k.xin, k.yout, chl, d1, d2, chr, wl, wm, wr, k.hb);
      if (st != MPS_OK) return st;
      MPS_TRY_HIP(h, launch_convert(s, k.yout, k.r, N, false));
    }
    // first projection gives alpha_j = Re <v_j|r>; then two more passes of
    // full Gram-Schmidt against every Krylov vector
    for (int pass = 0; pass < 3; ++pass) {
      MPS_TRY_HIP(h, launch_zero(s, (double*)k.dots, 64));
      MPS_TRY_HIP(h, launch_mdot(s, k.V, k.ldv, j + 1, k.r, N, k.dots, k.part));
      if (pass == 0) {
        MPS_TRY_HIP(h, hipMemcpyAsync(hd, k.dots, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
        MPS_TRY_HIP(h, hipStreamSynchronize(s));
        al.push_back(hd[j].x);
      }
      MPS_TRY_HIP(h, launch_msub(s, k.V, k.ldv, j + 1, k.dots, k.r, N));
    }
    MPS_TRY_HIP(h, launch_zero(s, (double*)k.dots, 64));
    MPS_TRY_HIP(h, launch_mdot(s, k.r, N, 1, k.r, N, k.dots, k.part));
    MPS_TRY_HIP(h, hipMemcpyAsync(hd, k.dots, sizeof(double2), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    const double bj = std::sqrt(std::max(hd[0].x, 0.0));
    be.push_back(bj);
    n = j + 1;
    MPS_TRY_HIP(h, hipMemcpyAsync(k.alpha, al.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, hipMemcpyAsync(k.beta, be.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, launch_tridiag_expm(s, k.alpha, k.beta, n, tau_re, tau_im, nrm, k.u, k.err));
    MPS_TRY_HIP(h, hipMemcpyAsync(&err, k.err, sizeof(double), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    if (err <= tol || bj <= 1e-14 * nrm) {
      ok = true;
      break;
    }
    if (j + 1 < n_max)
      MPS_TRY_HIP(h, launch_scale_inv_sqrt(s, k.r, k.V + (size_t)(j + 1) * k.ldv, N, &k.dots[0].x));
  }
  MPS_TRY_HIP(h, launch_combine(s, k.V, k.ldv, n, k.u, nrm, x, N));
  *n_used = n;
  *err_out = err;
  *conv = ok;
  if (!ok) {
    uint32_t bit = MPS_DEV_NOCONV_LANCZOS, cur = 0;
    MPS_TRY_HIP(h, hipMemcpyAsync(&cur, h->status_dev, sizeof(cur), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    cur |= bit;
    MPS_TRY_HIP(h, hipMemcpyAsync(h->status_dev, &cur, sizeof(cur), hipMemcpyHostToDevice, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
  }
  return MPS_OK;
}

__global__ void set_boundary_kernel(void* env, int w, int idx, int c128) {
  for (int i = threadIdx.x; i < w; i += blockDim.x) {
    if (c128)
      ((double2*)env)[i] = make_double2(i == idx ? 1.0 : 0.0, 0.0);
    else
      ((float2*)env)[i] = make_float2(i == idx ? 1.f : 0.f, 0.f);
  }
}

struct TdvpWs {
  char* envL;
  char* envR;
  size_t env_block;  // bytes per environment
  HeffBufs hb;
  KryBufs kb;
  double2* th128;
  void* thdt;
  double2* Xj;
  JacMat* mat;
  int32_t* rowmap;
  double* nrm2;
  int32_t* perm;
  double* s2;
  SelOut* sel;
  int32_t* unconv;
  char* u1r;  // charge-carrying chains: workspace of the blockwise split
};

// plan and carve the workspace for a chain with the given capacities
mps_status tdvp_workspace(mps_handle h, bool c128, int chi_max, int d, int w, int L, int n_max, TdvpWs& t,
                          bool u1 = false) {
  const size_t es = esize(c128);
  const long long Nmax = (long long)chi_max * d * d * chi_max;
  const long long Xmax = (long long)chi_max * w * d * d * chi_max;
  const int m_cap = d * chi_max;
  WsPlan p;
  size_t o_envL = p.take<char>((size_t)(L + 1) * chi_max * w * chi_max * es);
  size_t o_envR = p.take<char>((size_t)(L + 1) * chi_max * w * chi_max * es);
  size_t o_X1 = p.take<char>(Xmax * es), o_X2 = p.take<char>(Xmax * es), o_X3 = p.take<char>(Xmax * es);
  size_t o_W1 = p.take<char>(1024 * es), o_W2 = p.take<char>(1024 * es);
  size_t o_V = p.take<double2>((size_t)(n_max + 1) * Nmax);
  size_t o_r = p.take<double2>(Nmax);
  size_t o_xin = p.take<char>(Nmax * es), o_yout = p.take<char>(Nmax * es);
  size_t o_dots = p.take<double2>(32), o_part = p.take<double2>((size_t)kMdotBlocks * 32), o_al = p.take<double>(32), o_be = p.take<double>(32);
  size_t o_u = p.take<double2>(32), o_err = p.take<double>(4);
  size_t o_th = p.take<double2>(Nmax), o_thd = p.take<char>(Nmax * es), o_Xj = p.take<double2>(Nmax);
  size_t o_mat = p.take<JacMat>(1), o_rm = p.take<int32_t>(m_cap), o_pm = p.take<int32_t>(m_cap),
         o_nr = p.take<double>(m_cap);
  size_t o_s2 = p.take<double>(m_cap), o_sel = p.take<SelOut>(1), o_unc = p.take<int32_t>(8);
  size_t o_u1 = u1 ? p.take<char>(u1_layer_bytes(1, m_cap, chi_max)) : 0;
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  t.envL = ws + o_envL;
  t.envR = ws + o_envR;
  t.env_block = (size_t)chi_max * w * chi_max * es;
  t.hb = {ws + o_X1, ws + o_X2, ws + o_X3, ws + o_W1, ws + o_W2};
  t.kb.V = (double2*)(ws + o_V);
  t.kb.ldv = Nmax;
  t.kb.r = (double2*)(ws + o_r);
  t.kb.xin = ws + o_xin;
  t.kb.yout = ws + o_yout;
  t.kb.dots = (double2*)(ws + o_dots);
  t.kb.part = (double2*)(ws + o_part);
  t.kb.alpha = (double*)(ws + o_al);
  t.kb.beta = (double*)(ws + o_be);
  t.kb.u = (double2*)(ws + o_u);
  t.kb.err = (double*)(ws + o_err);
  t.kb.hb = t.hb;
  t.th128 = (double2*)(ws + o_th);
  t.thdt = ws + o_thd;
  t.Xj = (double2*)(ws + o_Xj);
  t.mat = (JacMat*)(ws + o_mat);
  t.rowmap = (int32_t*)(ws + o_rm);
  t.nrm2 = (double*)(ws + o_nr);
  t.perm = (int32_t*)(ws + o_pm);
  t.s2 = (double*)(ws + o_s2);
  t.sel = (SelOut*)(ws + o_sel);
  t.unconv = (int32_t*)(ws + o_unc);
  t.u1r = u1 ? ws + o_u1 : nullptr;
  return MPS_OK;
}

// Truncated SVD of the complex128 matrix t.Xj (m x n, prepared by the caller)
// through the batched Jacobi with one matrix; returns k and the discarded weight.
mps_status svd_select(mps_handle h, hipStream_t s, TdvpWs& t, int m, int n, int kmax, double eps, int* k,
                      double* disc) {
  JacMat hm;
  std::memset(&hm, 0, sizeof(hm));
  hm.X = t.Xj;
  hm.rowmap = t.rowmap;
  hm.nrm2 = t.nrm2;
  hm.m = m;
  hm.n = n;
  hm.ld = n;
  hm.nb = jac_nb(m);
  hm.kmax = std::min(kmax, m);
  MPS_TRY_HIP(h, hipMemcpyAsync(t.mat, &hm, sizeof(hm), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, t.mat, 1, h->status_dev));
  mps_status st = run_jacobi(h, s, t.mat, 1, hm.nb, m, t.unconv, false);
  if (st != MPS_OK) return st;
  MPS_TRY_HIP(h, launch_select(s, t.mat, 1, t.perm, t.s2, m, hm.kmax, count_rule_eps(h, eps), t.sel));
  SelOut so;
  MPS_TRY_HIP(h, hipMemcpyAsync(&so, t.sel, sizeof(so), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  *k = so.k;
  *disc = so.disc;
  return MPS_OK;
}

}  // namespace

mps_status tdvp_impl(mps_handle h, mps_stream stream, const mps_oc_chain* chain, double dt, int32_t n_steps,
                     double eps_local, int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev,
                     const mps_u1_chain* u1);

extern "C" {

mps_status mps_heff_apply(mps_handle h, mps_stream stream, int32_t dtype, const void* Lenv, const void* W1,
                          const void* W2, const void* Renv, const void* x, void* y, int64_t chi_l, int32_t d1,
                          int32_t d2, int64_t chi_r, int32_t w_l, int32_t w_m, int32_t w_r) {
  if (!h) return MPS_ERR_INVALID;
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "bad dtype");
  if (!Lenv || !W1 || !Renv || !x || !y) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  const bool two = W2 != nullptr;
  if (chi_l < 1 || chi_r < 1 || d1 < 1 || w_l < 1 || w_m < 1 || (two && (d2 < 1 || w_r < 1)))
    return mps_fail(h, MPS_ERR_SHAPE, "bad dimensions");
  if (w_l * d1 > 32 || w_m * d1 > 32 || (two && (w_m * d2 > 32 || w_r * d2 > 32)))
    return mps_fail(h, MPS_ERR_CAPACITY, "MPO dimension times d must be <= 32");
  if (chi_l > 8192 || chi_r > 8192) return mps_fail(h, MPS_ERR_CAPACITY, "chi limited to 8192");
  const bool c128 = dtype == MPS_C128;
  const size_t es = esize(c128);
  const int wmx = std::max(w_l, std::max(w_m, two ? w_r : 1));
  const long long X = chi_l * (long long)wmx * d1 * (two ? d2 : 1) * chi_r;
  WsPlan p;
  size_t o1 = p.take<char>(X * es), o2 = p.take<char>(X * es), o3 = p.take<char>(X * es);
  size_t o4 = p.take<char>(1024 * es), o5 = p.take<char>(1024 * es);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  HeffBufs b{h->ws + o1, h->ws + o2, h->ws + o3, h->ws + o4, h->ws + o5};
  return heff_apply_int(h, (hipStream_t)stream, c128, Lenv, W1, W2, Renv, x, y, (int)chi_l, d1, two ? d2 : 1,
                        (int)chi_r, w_l, w_m, two ? w_r : 1, b);
}

mps_status mps_env_update(mps_handle h, mps_stream stream, int32_t dtype, int32_t side, const void* env_in,
                          const void* W, const void* A, void* env_out, int64_t chi_in, int32_t d, int64_t chi_out,
                          int32_t w_in, int32_t w_out) {
  if (!h) return MPS_ERR_INVALID;
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "bad dtype");
  if (!env_in || !W || !A || !env_out) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (side != 0 && side != 1) return mps_fail(h, MPS_ERR_INVALID, "side must be 0 (left) or 1 (right)");
  if (chi_in < 1 || chi_out < 1 || d < 1 || w_in < 1 || w_out < 1) return mps_fail(h, MPS_ERR_SHAPE, "bad dims");
  if (w_in * d > 32 || w_out * d > 32) return mps_fail(h, MPS_ERR_CAPACITY, "MPO dimension times d must be <= 32");
  const bool c128 = dtype == MPS_C128;
  const size_t es = esize(c128);
  const long long X = chi_in * (long long)std::max(w_in, w_out) * d * chi_out;
  WsPlan p;
  size_t o1 = p.take<char>(X * es), o2 = p.take<char>(X * es), o4 = p.take<char>(1024 * es);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  HeffBufs b{h->ws + o1, h->ws + o2, nullptr, h->ws + o4, nullptr};
  if (side == 0)
    return env_left_int(h, (hipStream_t)stream, c128, env_in, A, W, env_out, (int)chi_in, d, (int)chi_out, w_in,
                        w_out, b);
  // right: env_in = [chi_in][w_in][chi_in], A = [chi_out][d][chi_in], W = [w_out][w_in][d][d]
  return env_right_int(h, (hipStream_t)stream, c128, env_in, A, W, env_out, (int)chi_in, d, (int)chi_out, w_out,
                       w_in, b);
}

mps_status mps_krylov_expm(mps_handle h, mps_stream stream, int32_t dtype, const void* Lenv, const void* W1,
                           const void* W2, const void* Renv, void* x, int64_t chi_l, int32_t d1, int32_t d2,
                           int64_t chi_r, int32_t w_l, int32_t w_m, int32_t w_r, double tau_re, double tau_im,
                           int32_t n_max, double tol, int32_t* n_used, double* err_est) {
  if (!h) return MPS_ERR_INVALID;
  if (dtype != MPS_C64 && dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "bad dtype");
  if (!Lenv || !W1 || !Renv || !x) return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (n_max < 1 || n_max > 30) return mps_fail(h, MPS_ERR_CAPACITY, "n_max must be in [1, 30]");
  const bool two = W2 != nullptr;
  if (chi_l < 1 || chi_r < 1 || d1 < 1 || (two && d2 < 1)) return mps_fail(h, MPS_ERR_SHAPE, "bad dimensions");
  if (w_l * d1 > 32 || w_m * d1 > 32 || (two && (w_m * d2 > 32 || w_r * d2 > 32)))
    return mps_fail(h, MPS_ERR_CAPACITY, "MPO dimension times d must be <= 32");
  const bool c128 = dtype == MPS_C128;
  const size_t es = esize(c128);
  const int dd2 = two ? d2 : 1;
  const long long N = chi_l * (long long)d1 * dd2 * chi_r;
  const int wmx = std::max(w_l, std::max(w_m, two ? w_r : 1));
  const long long X = chi_l * (long long)wmx * d1 * dd2 * chi_r;
  WsPlan p;
  size_t o1 = p.take<char>(X * es), o2 = p.take<char>(X * es), o3 = p.take<char>(X * es);
  size_t o4 = p.take<char>(1024 * es), o5 = p.take<char>(1024 * es);
  size_t oV = p.take<double2>((size_t)(n_max + 1) * N), oR = p.take<double2>(N);
  size_t oi = p.take<char>(N * es), oo = p.take<char>(N * es);
  size_t od = p.take<double2>(32), opart = p.take<double2>((size_t)kMdotBlocks * 32), oa = p.take<double>(32), ob = p.take<double>(32), ou = p.take<double2>(32),
         oe = p.take<double>(4), ox = p.take<double2>(N);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  KryBufs k;
  k.V = (double2*)(ws + oV);
  k.ldv = N;
  k.r = (double2*)(ws + oR);
  k.xin = ws + oi;
  k.yout = ws + oo;
  k.dots = (double2*)(ws + od);
  k.part = (double2*)(ws + opart);
  k.alpha = (double*)(ws + oa);
  k.beta = (double*)(ws + ob);
  k.u = (double2*)(ws + ou);
  k.err = (double*)(ws + oe);
  k.hb = {ws + o1, ws + o2, ws + o3, ws + o4, ws + o5};
  hipStream_t s = (hipStream_t)stream;
  // x is given in dtype; the iteration runs on a complex128 copy
  double2* x128 = (double2*)(ws + ox);
  if (c128)
    MPS_TRY_HIP(h, hipMemcpyAsync(x128, x, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  else
    MPS_TRY_HIP(h, launch_convert(s, x, x128, N, false));
  int nu = 0;
  double err = 0.0;
  bool conv = true;
  st = krylov_int(h, s, c128, Lenv, W1, W2, Renv, x128, (int)chi_l, d1, dd2, (int)chi_r, w_l, w_m, two ? w_r : 1,
                  tau_re, tau_im, n_max, tol, &nu, &err, &conv, k);
  if (st != MPS_OK) return st;
  if (c128)
    MPS_TRY_HIP(h, hipMemcpyAsync(x, x128, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  else
    MPS_TRY_HIP(h, launch_convert(s, x128, x, N, true));
  if (n_used) MPS_TRY_HIP(h, hipMemcpyAsync(n_used, &nu, sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (err_est) MPS_TRY_HIP(h, hipMemcpyAsync(err_est, &err, sizeof(double), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  return MPS_OK;
}

mps_status mps_tdvp2_step(mps_handle h, mps_stream stream, const mps_oc_chain* chain, double dt, int32_t n_steps,
                          double eps_local, int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev) {
  return tdvp_impl(h, stream, chain, dt, n_steps, eps_local, n_max, tol, disc_dev, krylov_max_dev, nullptr);
}

mps_status mps_tdvp2_step_u1(mps_handle h, mps_stream stream, const mps_oc_chain* chain,
                             const mps_u1_chain* charges, double dt, int32_t n_steps, double eps_local,
                             int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!charges || !charges->qbond) return mps_fail(h, MPS_ERR_INVALID, "null charges");
  if (charges->modulus < 0 || charges->modulus == 1)
    return mps_fail(h, MPS_ERR_INVALID, "modulus must be 0 (U(1)) or at least 2 (Z_n)");
  return tdvp_impl(h, stream, chain, dt, n_steps, eps_local, n_max, tol, disc_dev, krylov_max_dev, charges);
}

}  // extern "C"

mps_status tdvp_impl(mps_handle h, mps_stream stream, const mps_oc_chain* chain, double dt, int32_t n_steps,
                     double eps_local, int32_t n_max, double tol, double* disc_dev, int32_t* krylov_max_dev,
                     const mps_u1_chain* u1) {
  if (!h) return MPS_ERR_INVALID;
  if (!chain) return mps_fail(h, MPS_ERR_INVALID, "null chain");
  const mps_oc_chain& c = *chain;
  if (c.dtype != MPS_C64 && c.dtype != MPS_C128) return mps_fail(h, MPS_ERR_INVALID, "bad dtype");
  if (c.L < 2 || c.d < 1 || c.d > 8 || c.chi_max < 1 || c.w < 1) return mps_fail(h, MPS_ERR_SHAPE, "bad chain shape");
  if (c.w * c.d > 32) return mps_fail(h, MPS_ERR_CAPACITY, "MPO dimension times d must be <= 32");
  if ((int64_t)c.d * c.chi_max > 4096) return mps_fail(h, MPS_ERR_CAPACITY, "d*chi_max is limited to 4096");
  if (!c.M || !c.chi || !c.W) return mps_fail(h, MPS_ERR_INVALID, "null chain pointer");
  if (n_max < 1 || n_max > 30) return mps_fail(h, MPS_ERR_CAPACITY, "n_max must be in [1, 30]");
  if (n_steps < 0) return mps_fail(h, MPS_ERR_INVALID, "n_steps < 0");
  hipStream_t s = (hipStream_t)stream;
  const bool c128 = c.dtype == MPS_C128;
  const size_t es = esize(c128);
  const int L = c.L, d = c.d, w = c.w, cm = c.chi_max;
  TdvpWs t;
  if (u1 && d > 5) return mps_fail(h, MPS_ERR_SHAPE, "charge-carrying chains need d <= 5");
  mps_status st = tdvp_workspace(h, c128, cm, d, w, L, n_max, t, u1 != nullptr);
  if (st != MPS_OK) return st;
  std::vector<int32_t> chi(L + 1);
  MPS_TRY_HIP(h, hipMemcpyAsync(chi.data(), c.chi, (L + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  // charge-carrying chains: the bond charges on the host for the sweep
  std::vector<int32_t> qb(u1 ? (size_t)(L + 1) * cm : 0), rq, cq, qk(cm);
  if (u1) MPS_TRY_HIP(h, hipMemcpyAsync(qb.data(), u1->qbond, qb.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  const int32_t md = u1 ? u1->modulus : 0;
  auto red = [md](int64_t v) -> int32_t { return md == 0 ? (int32_t)v : (int32_t)(((v % md) + md) % md); };
  // row (a, s1) and column (s2, g) charges of theta at bond b (chl x d, d x chr)
  auto charges_of = [&](int b, int chl, int chr) {
    rq.resize((size_t)chl * d);
    cq.resize((size_t)d * chr);
    for (int a = 0; a < chl; ++a)
      for (int s1 = 0; s1 < d; ++s1) rq[a * d + s1] = red((int64_t)qb[(size_t)b * cm + a] + u1->qsite[s1]);
    for (int s2 = 0; s2 < d; ++s2)
      for (int g = 0; g < chr; ++g) cq[s2 * chr + g] = red((int64_t)qb[(size_t)(b + 2) * cm + g] - u1->qsite[s2]);
  };
  for (int i = 0; i <= L; ++i)
    if (chi[i] < 1 || chi[i] > cm) return mps_fail(h, MPS_ERR_SHAPE, "chi entries must be in [1, chi_max]");
  const size_t site = (size_t)cm * d * cm * es;
  auto Mp = [&](int i) { return (char*)c.M + (size_t)i * site; };
  auto Wp = [&](int i) { return (const char*)c.W + (size_t)i * w * w * d * d * es; };
  auto Lp = [&](int i) { return t.envL + (size_t)i * t.env_block; };
  auto Rp = [&](int i) { return t.envR + (size_t)i * t.env_block; };
  std::vector<double> disc(L - 1, 0.0);
  int kry_max = 0;

  set_boundary_kernel<<<1, 64, 0, s>>>(Lp(0), w, w - 1, c128);
  set_boundary_kernel<<<1, 64, 0, s>>>(Rp(L), w, 0, c128);
  MPS_TRY_HIP(h, hipGetLastError());
  for (int i = L - 1; i >= 2; --i) {
    st = env_right_int(h, s, c128, Rp(i + 1), Mp(i), Wp(i), Rp(i), chi[i + 1], d, chi[i], w, w, t.hb);
    if (st != MPS_OK) return st;
  }
  const double tau = 0.5 * dt;

  // theta = M_b M_{b+1} into t.th128 (complex128)
  auto build_theta = [&](int b) -> mps_status {
    SGemm g;
    std::memset(&g, 0, sizeof(g));
    g.A = Mp(b); g.rsA = chi[b + 1]; g.csA = 1;
    g.B = Mp(b + 1); g.rsB = (long long)d * chi[b + 2]; g.csB = 1;
    g.C = c128 ? (void*)t.th128 : t.thdt; g.rsC = (long long)d * chi[b + 2]; g.csC = 1;
    g.M = chi[b] * d; g.K = chi[b + 1]; g.N = d * chi[b + 2]; g.alpha = 1.0;
    MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
    if (!c128) MPS_TRY_HIP(h, launch_convert(s, t.thdt, t.th128, (long long)g.M * g.N, false));
    return MPS_OK;
  };
  auto evolve2 = [&](int b) -> mps_status {
    int nu;
    double err;
    bool cv;
    mps_status r = krylov_int(h, s, c128, Lp(b), Wp(b), Wp(b + 1), Rp(b + 2), t.th128, chi[b], d, d, chi[b + 2], w, w,
                              w, tau, 0.0, n_max, tol, &nu, &err, &cv, t.kb);
    kry_max = std::max(kry_max, nu);
    return r;
  };
  // one-site backward step on the tensor stored at M_i (dims chl x d x chr)
  auto evolve1 = [&](int i, const void* Le, const void* Re, int chl, int chr) -> mps_status {
    const long long N = (long long)chl * d * chr;
    double2* x = c128 ? (double2*)Mp(i) : t.th128;
    if (!c128) MPS_TRY_HIP(h, launch_convert(s, Mp(i), t.th128, N, false));
    int nu;
    double err;
    bool cv;
    mps_status r = krylov_int(h, s, c128, Le, Wp(i), nullptr, Re, x, chl, d, 1, chr, w, w, 1, -tau, 0.0, n_max, tol,
                              &nu, &err, &cv, t.kb);
    if (r != MPS_OK) return r;
    kry_max = std::max(kry_max, nu);
    if (!c128) MPS_TRY_HIP(h, launch_convert(s, t.th128, Mp(i), N, true));
    return MPS_OK;
  };

  for (int step = 0; step < n_steps; ++step) {
    // ---- left to right ----
    for (int b = 0; b <= L - 2; ++b) {
      const int chl = chi[b], chr = chi[b + 2], m = chl * d, n = d * chr;
      if ((st = build_theta(b)) != MPS_OK) return st;
      if ((st = evolve2(b)) != MPS_OK) return st;
      // U from the Jacobi rows of theta^T (columns of theta)
      MPS_TRY_HIP(h, launch_transpose_c128(s, t.th128, t.Xj, m, n));
      int k;
      double w_disc;
      if (u1) {
        // the rows of theta^T carry the column charges; A_b = U_k as [chl*d][k]
        charges_of(b, chl, chr);
        if ((st = u1_split_one(h, s, t.Xj, n, m, cq.data(), rq.data(), cm, eps_local, t.u1r, d * cm, cm, t.sel, Mp(b),
                               1, c128, &k, &w_disc, qk.data())) != MPS_OK)
          return st;
        std::copy(qk.begin(), qk.begin() + k, qb.begin() + (size_t)(b + 1) * cm);
      } else {
        if ((st = svd_select(h, s, t, n, m, cm, eps_local, &k, &w_disc)) != MPS_OK) return st;
        // A_b = U_k, column-major rows -> [chl*d][k]
        MPS_TRY_HIP(h, launch_write_rows(s, t.mat, t.perm, t.s2, t.sel, Mp(b), m, 1, c128));
      }
      disc[b] += w_disc;
      // C = U_k^dag theta -> M_{b+1} [k][d*chr]
      if (!c128) MPS_TRY_HIP(h, launch_convert(s, t.th128, t.thdt, (long long)m * n, true));
      SGemm g;
      std::memset(&g, 0, sizeof(g));
      g.A = Mp(b); g.rsA = 1; g.csA = k; g.conjA = 1;
      g.B = c128 ? (const void*)t.th128 : (const void*)t.thdt; g.rsB = n; g.csB = 1;
      g.C = Mp(b + 1); g.rsC = n; g.csC = 1;
      g.M = k; g.K = m; g.N = n; g.alpha = 1.0;
      MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
      chi[b + 1] = k;
      if ((st = env_left_int(h, s, c128, Lp(b), Mp(b), Wp(b), Lp(b + 1), chl, d, k, w, w, t.hb)) != MPS_OK)
        return st;
      if (b < L - 2)
        if ((st = evolve1(b + 1, Lp(b + 1), Rp(b + 2), k, chr)) != MPS_OK) return st;
    }
    // ---- right to left ----
    for (int b = L - 2; b >= 0; --b) {
      const int chl = chi[b], chr = chi[b + 2], m = chl * d, n = d * chr;
      if ((st = build_theta(b)) != MPS_OK) return st;
      if ((st = evolve2(b)) != MPS_OK) return st;
      MPS_TRY_HIP(h, hipMemcpyAsync(t.Xj, t.th128, (size_t)m * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      int k;
      double w_disc;
      if (u1) {
        // B_{b+1} = V_k^dag, row-major [k][d*chr], zero off each vector's block
        charges_of(b, chl, chr);
        if ((st = u1_split_one(h, s, t.Xj, m, n, rq.data(), cq.data(), cm, eps_local, t.u1r, d * cm, cm, t.sel,
                               Mp(b + 1), 0, c128, &k, &w_disc, qk.data())) != MPS_OK)
          return st;
        std::copy(qk.begin(), qk.begin() + k, qb.begin() + (size_t)(b + 1) * cm);
      } else {
        if ((st = svd_select(h, s, t, m, n, cm, eps_local, &k, &w_disc)) != MPS_OK) return st;
        // B_{b+1} = V_k^dag, row-major [k][d*chr]
        MPS_TRY_HIP(h, launch_write_rows(s, t.mat, t.perm, t.s2, t.sel, Mp(b + 1), n, 0, c128));
      }
      disc[b] += w_disc;
      // C = theta V_k -> M_b [chl*d][k]
      if (!c128) MPS_TRY_HIP(h, launch_convert(s, t.th128, t.thdt, (long long)m * n, true));
      SGemm g;
      std::memset(&g, 0, sizeof(g));
      g.A = c128 ? (const void*)t.th128 : (const void*)t.thdt; g.rsA = n; g.csA = 1;
      g.B = Mp(b + 1); g.rsB = 1; g.csB = n; g.conjB = 1;
      g.C = Mp(b); g.rsC = k; g.csC = 1;
      g.M = m; g.K = n; g.N = k; g.alpha = 1.0;
      MPS_TRY_HIP(h, launch_sgemm(s, g, c128));
      chi[b + 1] = k;
      if ((st = env_right_int(h, s, c128, Rp(b + 2), Mp(b + 1), Wp(b + 1), Rp(b + 1), chr, d, k, w, w, t.hb)) != MPS_OK)
        return st;
      if (b > 0)
        if ((st = evolve1(b, Lp(b), Rp(b + 1), chl, k)) != MPS_OK) return st;
    }
  }
  MPS_TRY_HIP(h, hipMemcpyAsync(c.chi, chi.data(), (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (u1) MPS_TRY_HIP(h, hipMemcpyAsync(u1->qbond, qb.data(), qb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (disc_dev) {
    std::vector<double> old(L - 1);
    MPS_TRY_HIP(h, hipMemcpyAsync(old.data(), disc_dev, (L - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    MPS_TRY_HIP(h, hipStreamSynchronize(s));
    for (int b = 0; b < L - 1; ++b) old[b] += disc[b];
    MPS_TRY_HIP(h, hipMemcpyAsync(disc_dev, old.data(), (L - 1) * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if (krylov_max_dev) MPS_TRY_HIP(h, hipMemcpyAsync(krylov_max_dev, &kry_max, sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  return MPS_OK;
}
