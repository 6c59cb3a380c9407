// Exponential of the Lanczos tridiagonal matrix, run by one 256-thread
// workgroup (Sec. "Krylov time evolution": the propagated state in the Krylov
// basis is |psi| exp(-i tau T) e_1).
//
// T = tridiag(beta, alpha, beta) of order n <= 32 is diagonalised by the LDS
// Jacobi solver, T = Q diag(theta) Q^T (real orthogonal Q), and
//   u = Q (exp(-i tau theta) * Q^T e_1),
//   err = nrm * |beta_{n-1}| * |u_{n-1}|   (a-posteriori estimate),
// with tau = tau_re + i tau_im.  alpha and beta may live in LDS or global
// memory; u and err are written by threads 0..n-1 and 0.  G, Q (JS_N x JS_LD),
// rot and flag are LDS scratch.  Every thread must call it.
#pragma once
#include "jacobi_small.h"

__device__ __forceinline__ void tridiag_expm_block(const double* alpha, const double* beta, int n, double tau_re,
                                                   double tau_im, double nrm, double2* u, double* err, double2* G,
                                                   double2* Q, double4* rot, int* flag) {
  const int tid = threadIdx.x;
  double scale = 0.0;
  for (int i = 0; i < n; ++i)
    scale = fmax(scale, fabs(alpha[i]) + (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i + 1 < n ? fabs(beta[i]) : 0.0));
  for (int e = tid; e < JS_N * JS_N; e += blockDim.x) {
    int r = e / JS_N, c = e % JS_N;
    double v = 0.0;
    if (r < n && c < n) {
      if (r == c) v = alpha[r];
      else if (c == r + 1) v = beta[r];
      else if (r == c + 1) v = beta[c];
    }
    G[r * JS_LD + c] = make_double2(v, 0.0);
  }
  __syncthreads();
  herm_jacobi32(G, Q, n, 1e-16 * scale + 1e-300, 0.0, 60, rot, flag);
  if (tid < n) {
    int i = tid;
    double2 a = make_double2(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
      double th = G[k * JS_LD + k].x;
      // exp(-i tau th) = exp(tau_im th) (cos(tau_re th) - i sin(tau_re th))
      double mag = exp(tau_im * th), sn, cs;
      sincos(tau_re * th, &sn, &cs);
      double q0 = Q[0 * JS_LD + k].x;  // real orthogonal eigenvectors
      double qi = Q[i * JS_LD + k].x;
      a.x += qi * mag * cs * q0;
      a.y -= qi * mag * sn * q0;
    }
    u[i] = a;
  }
  __syncthreads();
  if (tid == 0) {
    double2 un = u[n - 1];
    *err = nrm * fabs(beta[n - 1]) * sqrt(un.x * un.x + un.y * un.y);
  }
  __syncthreads();
}
