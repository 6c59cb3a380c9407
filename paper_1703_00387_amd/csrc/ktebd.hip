// Krylov TEBD: the local Lanczos exponential of a bond term, batched over the
// bonds of one sweep layer.
//
// In the Sornborger-Stewart sweep the centre of the chain sits inside the two
// sites of the bond being updated, so (App. "Details of the Krylov method")
// the Krylov basis built with the bond term h_b, the overlaps of its vectors
// and their weighted sum live on the two-site tensor theta'[a, p, c] alone,
// with h_b acting on the pair p = (s t) of physical indices.  Every Krylov
// vector is v_j = Q_j(h) theta' for a polynomial Q_j of degree j in the D x D
// matrix h (D = d^2), and the overlap of two of them involves only the D x D
// reduced matrix rho[p][q] = sum_{a,c} theta'[a,p,c] conj(theta'[a,q,c]):
//   <Q theta', R theta'> = Tr(Q^dag R rho) = <Q W, R W>_F   for rho = W W^dag.
// The paper's Lanczos iteration (v_1 = theta'/|theta'|; r = h v_j;
// alpha_j = Re<v_j|r>; r -= alpha_j v_j + beta_{j-1} v_{j-1}; two passes of
// full Gram-Schmidt; beta_j = |r|; exponential of the tridiagonal matrix and
// the a-posteriori estimate) therefore runs here on the D x D matrices
// Z_j = Q_j(h) W with the Frobenius inner product: the same iteration, written
// in the coordinates of the Schmidt decomposition of theta' between the two
// sites and the rest of the chain, with W = U sqrt(sigma) from rho's
// eigendecomposition.  The recurrence applied to Q_0 = I/|theta'| with the
// same coefficients carries the polynomials themselves, so the Krylov sum
// |theta'| sum_j u_j v_j equals G theta' for the D x D matrix
// G = |theta'| sum_j u_j Q_j(h).  G is the bond's propagator in the plain
// update (theta~' = G theta~, FP64 SVD, B_b = theta~' V_k / n_k); the
// Hastings write-back needs G itself, since theta' carries the left Schmidt
// values and theta~ does not.
//
//   ktebd_rho_kernel    partial sums of rho over slices of the (a, c) pairs,
//                       grid (nblk, items); reads theta' once (HBM-bound)
//   ktebd_krylov_kernel one workgroup per bond: eigendecomposition of rho,
//                       Lanczos iteration, tridiagonal exponential, stopping
//                       test and G, all in FP64
#include "common.h"
#include "jacobi_small.h"
#include "krylov_small.h"

#define KT_CHUNK 64   // (a, c) pairs staged per pass
#define KT_DMAX 25    // D = d^2 <= 25

__global__ void ktebd_identity_kernel(void* G, int dd, int c128) {
  for (int e = threadIdx.x; e < dd * dd; e += blockDim.x) {
    const double v = (e / dd == e % dd) ? 1.0 : 0.0;
    if (c128)
      ((double2*)G)[e] = make_double2(v, 0.0);
    else
      ((float2*)G)[e] = make_float2((float)v, 0.f);
  }
}

// rho partial sums: block x of item y covers pairs [P x / nblk, P (x+1) / nblk)
// of the P = chi_l chi_r pairs (a, c), pair index a * chi_r + c.
__global__ __launch_bounds__(256) void ktebd_rho_kernel(const BondItem* __restrict__ items,
                                                        const KryJob* __restrict__ jobs, int d, int nblk) {
  __shared__ double2 xs[KT_CHUNK * KT_DMAX];
  const BondItem it = items[blockIdx.y];
  const KryJob jb = jobs[blockIdx.y];
  const int D = d * d, DD = D * D;
  const int chl = it.chi[it.b], chr = it.chi[it.b + 2];
  const long long n = (long long)d * chr;   // row length of theta' (row a*d+u, column v*chi_r+c)
  const long long P = (long long)chl * chr;
  const long long p0 = P * blockIdx.x / nblk, p1 = P * (blockIdx.x + 1) / nblk;
  const int tid = threadIdx.x;
  double2 acc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) acc[r] = make_double2(0.0, 0.0);
  for (long long base = p0; base < p1; base += KT_CHUNK) {
    for (int idx = tid; idx < KT_CHUNK * D; idx += 256) {
      const int pl = idx % KT_CHUNK, p = idx / KT_CHUNK;
      const long long pi = base + pl;
      double2 v = make_double2(0.0, 0.0);
      if (pi < p1) {
        const long long a = pi / chr, c = pi % chr;
        const int u = p / d, w = p % d;
        v = it.X[(a * d + u) * n + (long long)w * chr + c];
      }
      xs[pl * D + p] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int e = tid + 256 * r;
      if (e < DD) {
        const int p = e / D, q = e % D;
        double2 a = acc[r];
        for (int pl = 0; pl < KT_CHUNK; ++pl) {
          const double2 x = xs[pl * D + p], y = xs[pl * D + q];
          a.x += x.x * y.x + x.y * y.y;   // x conj(y)
          a.y += x.y * y.x - x.x * y.y;
        }
        acc[r] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int e = tid + 256 * r;
    if (e < DD) jb.part[(size_t)blockIdx.x * DD + e] = acc[r];
  }
}

__device__ __forceinline__ double kt_block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double2 kt_cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void ktebd_krylov_kernel(const KryJob* __restrict__ jobs, int D, int nblk,
                                                           int n_max, double tol, double tau, int c128,
                                                           uint32_t* status) {
  __shared__ double2 G[JS_N * JS_LD];
  __shared__ double2 Qm[JS_N * JS_LD];
  __shared__ double4 rot[16];
  __shared__ int flag;
  __shared__ double2 hs[KT_DMAX * KT_DMAX], RZ[KT_DMAX * KT_DMAX], RQ[KT_DMAX * KT_DMAX];
  __shared__ double al[JS_N], be[JS_N];
  __shared__ double2 u[JS_N], cd[JS_N];
  __shared__ double red[256];
  __shared__ double err_s;
  const KryJob jb = jobs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int DD = D * D;
  double2* Zh = jb.hist;                               // Z_j at Zh + j DD
  double2* Qh = jb.hist + (size_t)(n_max + 1) * DD;    // Q_j at Qh + j DD

  // rho (Hermitian part of the summed partials, zero-padded to 32 x 32) and h
  double f2 = 0.0;
  for (int e = tid; e < JS_N * JS_N; e += blockDim.x) {
    const int r = e / JS_N, c = e % JS_N;
    double2 v = make_double2(0.0, 0.0);
    if (r < D && c < D) {
      double2 x = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
      for (int k = 0; k < nblk; ++k) {
        const double2 pr = jb.part[(size_t)k * DD + r * D + c], pc = jb.part[(size_t)k * DD + c * D + r];
        x.x += pr.x; x.y += pr.y;
        y.x += pc.x; y.y += pc.y;
      }
      v = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
    G[r * JS_LD + c] = v;
    f2 += v.x * v.x + v.y * v.y;
  }
  for (int e = tid; e < DD; e += blockDim.x) hs[e] = jb.h[e];
  const double fro = sqrt(kt_block_sum(f2, red));
  herm_jacobi32(G, Qm, D, 1e-15 * fro + 1e-300, 0.0, 40, rot, &flag);

  // W = U sqrt(sigma): Z_0 = W / |theta'|, |theta'|^2 = |W|_F^2 = Tr rho
  double w2 = 0.0;
  for (int e = tid; e < DD; e += blockDim.x) {
    const int p = e / D, k = e % D;
    const double sg = sqrt(fmax(G[k * JS_LD + k].x, 0.0));
    const double2 q = Qm[p * JS_LD + k];
    RZ[e] = make_double2(q.x * sg, q.y * sg);
    w2 += (q.x * q.x + q.y * q.y) * sg * sg;
  }
  const double nrm = sqrt(kt_block_sum(w2, red));
  if (!(nrm > 0.0)) {   // theta' = 0: nothing to propagate
    for (int e = tid; e < DD; e += blockDim.x) {
      const double v = (e / D == e % D) ? 1.0 : 0.0;
      if (c128)
        ((double2*)jb.G)[e] = make_double2(v, 0.0);
      else
        ((float2*)jb.G)[e] = make_float2((float)v, 0.f);
    }
    if (tid == 0 && jb.n_used) *jb.n_used = 0;
    return;
  }
  const double inv0 = 1.0 / nrm;
  for (int e = tid; e < DD; e += blockDim.x) {
    Zh[e] = make_double2(RZ[e].x * inv0, RZ[e].y * inv0);
    Qh[e] = make_double2((e / D == e % D) ? inv0 : 0.0, 0.0);
  }
  __syncthreads();

  int n = n_max;
  bool conv = false;
  double beta_prev = 0.0;
  for (int j = 0; j < n_max; ++j) {
    const double2* Zj = Zh + (size_t)j * DD;
    const double2* Qj = Qh + (size_t)j * DD;
    // r = h v_j (both the vector and its polynomial); alpha_j = Re <v_j|r>
    double pa = 0.0;
    for (int e = tid; e < DD; e += blockDim.x) {
      const int p = e / D, q = e % D;
      double2 rz = make_double2(0.0, 0.0), rq = make_double2(0.0, 0.0);
      for (int k = 0; k < D; ++k) {
        const double2 hk = hs[p * D + k];
        const double2 z = Zj[k * D + q], y = Qj[k * D + q];
        rz.x += hk.x * z.x - hk.y * z.y;
        rz.y += hk.x * z.y + hk.y * z.x;
        rq.x += hk.x * y.x - hk.y * y.y;
        rq.y += hk.x * y.y + hk.y * y.x;
      }
      RZ[e] = rz;
      RQ[e] = rq;
      const double2 zj = Zj[e];
      pa += zj.x * rz.x + zj.y * rz.y;
    }
    const double a = kt_block_sum(pa, red);
    // r -= alpha_j v_j + beta_{j-1} v_{j-1}
    for (int e = tid; e < DD; e += blockDim.x) {
      double2 rz = RZ[e], rq = RQ[e];
      const double2 z = Zj[e], y = Qj[e];
      rz.x -= a * z.x; rz.y -= a * z.y;
      rq.x -= a * y.x; rq.y -= a * y.y;
      if (j > 0) {
        const double2 zp = Zh[(size_t)(j - 1) * DD + e], yp = Qh[(size_t)(j - 1) * DD + e];
        rz.x -= beta_prev * zp.x; rz.y -= beta_prev * zp.y;
        rq.x -= beta_prev * yp.x; rq.y -= beta_prev * yp.y;
      }
      RZ[e] = rz;
      RQ[e] = rq;
    }
    __syncthreads();
    // two passes of Gram-Schmidt against every Krylov vector
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wave; i <= j; i += 4) {
        const double2* Zi = Zh + (size_t)i * DD;
        double sx = 0.0, sy = 0.0;
        for (int e = lane; e < DD; e += 64) {
          const double2 z = Zi[e], r = RZ[e];
          sx += z.x * r.x + z.y * r.y;   // conj(z) r
          sy += z.x * r.y - z.y * r.x;
        }
        for (int off = 32; off > 0; off >>= 1) {
          sx += __shfl_xor(sx, off);
          sy += __shfl_xor(sy, off);
        }
        if (lane == 0) cd[i] = make_double2(sx, sy);
      }
      __syncthreads();
      for (int e = tid; e < DD; e += blockDim.x) {
        double2 rz = RZ[e], rq = RQ[e];
        for (int i = 0; i <= j; ++i) {
          const double2 c = cd[i];
          const double2 tz = kt_cmul(c, Zh[(size_t)i * DD + e]), tq = kt_cmul(c, Qh[(size_t)i * DD + e]);
          rz.x -= tz.x; rz.y -= tz.y;
          rq.x -= tq.x; rq.y -= tq.y;
        }
        RZ[e] = rz;
        RQ[e] = rq;
      }
      __syncthreads();
    }
    double pb = 0.0;
    for (int e = tid; e < DD; e += blockDim.x) pb += RZ[e].x * RZ[e].x + RZ[e].y * RZ[e].y;
    const double bj = sqrt(fmax(kt_block_sum(pb, red), 0.0));
    if (tid == 0) {
      al[j] = a;
      be[j] = bj;
    }
    __syncthreads();
    tridiag_expm_block(al, be, j + 1, tau, 0.0, nrm, u, &err_s, G, Qm, rot, &flag);
    const double err = err_s;
    if (err <= tol || bj <= 1e-14 * nrm) {
      n = j + 1;
      conv = true;
      break;
    }
    if (j + 1 < n_max) {
      const double inv = 1.0 / bj;
      for (int e = tid; e < DD; e += blockDim.x) {
        Zh[(size_t)(j + 1) * DD + e] = make_double2(RZ[e].x * inv, RZ[e].y * inv);
        Qh[(size_t)(j + 1) * DD + e] = make_double2(RQ[e].x * inv, RQ[e].y * inv);
      }
    }
    beta_prev = bj;
    __syncthreads();
  }

  // G = |theta'| sum_{i<n} u_i Q_i(h)
  for (int e = tid; e < DD; e += blockDim.x) {
    double2 g = make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
      const double2 t = kt_cmul(u[i], Qh[(size_t)i * DD + e]);
      g.x += t.x;
      g.y += t.y;
    }
    g.x *= nrm;
    g.y *= nrm;
    if (c128)
      ((double2*)jb.G)[e] = g;
    else
      ((float2*)jb.G)[e] = make_float2((float)g.x, (float)g.y);
  }
  if (tid == 0) {
    if (jb.n_used) *jb.n_used = n;
    if (!conv) atomicOr(status, MPS_DEV_NOCONV_LANCZOS);
  }
}

hipError_t launch_ktebd_identity(hipStream_t s, void* G, int dd, bool c128) {
  ktebd_identity_kernel<<<1, 256, 0, s>>>(G, dd, c128 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ktebd_rho(hipStream_t s, const BondItem* items, const KryJob* jobs, int n_items, int d, int nblk) {
  if (n_items <= 0) return hipSuccess;
  if (d < 1 || d > 5 || nblk < 1) return hipErrorInvalidValue;
  ktebd_rho_kernel<<<dim3(nblk, n_items), 256, 0, s>>>(items, jobs, d, nblk);
  return hipGetLastError();
}

hipError_t launch_ktebd_krylov(hipStream_t s, const KryJob* jobs, int n_items, int d, int nblk, int n_max, double tol,
                               double tau, bool c128, uint32_t* status) {
  if (n_items <= 0) return hipSuccess;
  if (d < 1 || d > 5 || nblk < 1 || n_max < 1 || n_max > JS_N) return hipErrorInvalidValue;
  ktebd_krylov_kernel<<<n_items, 256, 0, s>>>(jobs, d * d, nblk, n_max, tol, tau, c128 ? 1 : 0, status);
  return hipGetLastError();
}
