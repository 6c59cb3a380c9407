// Cyclic parallel Jacobi eigensolver for a Hermitian matrix of order <= 32
// held in LDS, run by one 256-thread workgroup, in FP64.
//
// G  : [32][JS_LD] complex128 in LDS, overwritten with Q^dag G Q (diagonal)
// Q  : [32][JS_LD] complex128 in LDS, overwritten with the accumulated unitary
//      (initialised here to the identity); G_in = Q diag(G_out) Q^dag.
// Each step rotates 16 disjoint index pairs chosen by the circle method, so
// a sweep of 31 steps visits every pair once.  The 2x2 rotation for the
// pair (p, q) with a = G_pp, b = G_qq, c = G_pq = |c| e^{i phi} is
//   J = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]],
//   t = sign(tau) / (|tau| + sqrt(1 + tau^2)),  tau = (b - a) / (2|c|),
//   cs = 1/sqrt(1+t^2), sn = t cs,
// which zeroes (J^dag G J)_pq and moves the diagonal to a - t|c|, b + t|c|.
// A pair is skipped when |c| <= max(abs_thr, rel_thr * sqrt(|a b|)).
#pragma once

#define JS_N 32
#define JS_LD 33

__device__ __forceinline__ void js_pair(int step, int k, int& p, int& q) {
  // circle method over 32 players, 31 rounds
  if (k == 0) {
    p = 31;
    q = step;
  } else {
    p = (step + k) % 31;
    q = (step - k + 31) % 31;
  }
}

// Returns the number of sweeps used (<= max_sweeps).  All 256 threads call it.
__device__ int herm_jacobi32(double2* G, double2* Q, int n, double abs_thr, double rel_thr,
                             int max_sweeps, double4* rot /* LDS [16] */, int* flag /* LDS */) {
  const int tid = threadIdx.x;
  for (int i = tid; i < JS_N * JS_N; i += blockDim.x) {
    int r = i / JS_N, c = i % JS_N;
    Q[r * JS_LD + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int step = 0; step < 31; ++step) {
      if (tid < 16) {
        int p, q;
        js_pair(step, tid, p, q);
        if (p > q) { int t = p; p = q; q = t; }
        double4 r = make_double4(1.0, 0.0, 1.0, 0.0);  // cs, sn, ph.re, ph.im ; identity
        if (q < n) {
          double a = G[p * JS_LD + p].x, b = G[q * JS_LD + q].x;
          double2 c = G[p * JS_LD + q];
          double ac = sqrt(c.x * c.x + c.y * c.y);
          double thr = fmax(abs_thr, rel_thr * sqrt(fabs(a * b)));
          if (ac > thr && ac > 0.0) {
            double tau = (b - a) / (2.0 * ac);
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            double cs = 1.0 / sqrt(1.0 + t * t);
            r = make_double4(cs, t * cs, c.x / ac, c.y / ac);
            *flag = 1;
          }
        }
        rot[tid] = r;
      }
      __syncthreads();
      // columns: G <- G J, Q <- Q J
      for (int it = tid; it < JS_N * 16; it += blockDim.x) {
        int row = it >> 4, k = it & 15;
        double4 r = rot[k];
        if (r.y == 0.0) continue;
        int p, q;
        js_pair(step, k, p, q);
        if (p > q) { int t = p; p = q; q = t; }
        double2 em = make_double2(r.z, -r.w);  // e^{-i phi}
        double2 gp = G[row * JS_LD + p], gq = G[row * JS_LD + q];
        double2 gqe = cmul(gq, em);
        G[row * JS_LD + p] = make_double2(r.x * gp.x - r.y * gqe.x, r.x * gp.y - r.y * gqe.y);
        G[row * JS_LD + q] = make_double2(r.y * gp.x + r.x * gqe.x, r.y * gp.y + r.x * gqe.y);
        double2 qp = Q[row * JS_LD + p], qq = Q[row * JS_LD + q];
        double2 qqe = cmul(qq, em);
        Q[row * JS_LD + p] = make_double2(r.x * qp.x - r.y * qqe.x, r.x * qp.y - r.y * qqe.y);
        Q[row * JS_LD + q] = make_double2(r.y * qp.x + r.x * qqe.x, r.y * qp.y + r.x * qqe.y);
      }
      __syncthreads();
      // rows: G <- J^dag G
      for (int it = tid; it < JS_N * 16; it += blockDim.x) {
        int col = it >> 4, k = it & 15;
        double4 r = rot[k];
        if (r.y == 0.0) continue;
        int p, q;
        js_pair(step, k, p, q);
        if (p > q) { int t = p; p = q; q = t; }
        double2 ep = make_double2(r.z, r.w);  // e^{+i phi}
        double2 gp = G[p * JS_LD + col], gq = G[q * JS_LD + col];
        double2 gqe = cmul(gq, ep);
        G[p * JS_LD + col] = make_double2(r.x * gp.x - r.y * gqe.x, r.x * gp.y - r.y * gqe.y);
        G[q * JS_LD + col] = make_double2(r.y * gp.x + r.x * gqe.x, r.y * gp.y + r.x * gqe.y);
      }
      __syncthreads();
      // exact zeros on the rotated pairs keep rounding from accumulating
      if (tid < 16) {
        double4 r = rot[tid];
        if (r.y != 0.0) {
          int p, q;
          js_pair(step, tid, p, q);
          if (p > q) { int t = p; p = q; q = t; }
          G[p * JS_LD + q] = make_double2(0.0, 0.0);
          G[q * JS_LD + p] = make_double2(0.0, 0.0);
          G[p * JS_LD + p].y = 0.0;
          G[q * JS_LD + q].y = 0.0;
        }
      }
      __syncthreads();
    }
    if (*flag == 0) break;
    __syncthreads();
  }
  __syncthreads();
  return sweep;
}
