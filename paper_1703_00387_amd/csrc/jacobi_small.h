// Cyclic parallel Jacobi eigensolver for a Hermitian matrix of order <= N
// (N = 32 or 64) held in LDS, run by one 256-thread workgroup, in FP64.
//
// G  : [N][N+1] complex128 in LDS, overwritten with Q^dag G Q (diagonal)
// Q  : [N][N+1] complex128 in LDS, overwritten with the accumulated unitary
//      (initialised here to the identity); G_in = Q diag(G_out) Q^dag.
// Each step rotates N/2 disjoint index pairs chosen by the circle method, so
// a sweep of N-1 steps visits every pair once.  The 2x2 rotation for the
// pair (p, q) with a = G_pp, b = G_qq, c = G_pq = |c| e^{i phi} is
//   J = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]],
//   t = sign(tau) / (|tau| + sqrt(1 + tau^2)),  tau = (b - a) / (2|c|),
//   cs = 1/sqrt(1+t^2), sn = t cs,
// which zeroes (J^dag G J)_pq and moves the diagonal to a - t|c|, b + t|c|.
// A pair is skipped when |c| <= max(abs_thr, rel_thr * sqrt(|a b|)).
#pragma once

#define JS_N 32
#define JS_LD 33

template <int N>
__device__ __forceinline__ void js_pair(int step, int k, int& p, int& q) {
  // circle method over N players, N-1 rounds
  if (k == 0) {
    p = N - 1;
    q = step;
  } else {
    p = (step + k) % (N - 1);
    q = (step - k + N - 1) % (N - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

// Returns the number of sweeps used (<= max_sweeps).  Exactly 256 threads call it.
template <int N>
__device__ int herm_jacobi(double2* G, double2* Q, int n, double abs_thr, double rel_thr, int max_sweeps,
                           double4* rot /* LDS [N/2] */, int* flag /* LDS */) {
  constexpr int LD = N + 1, NP = N / 2;
  const int tid = threadIdx.x;
  for (int i = tid; i < N * N; i += blockDim.x) {
    int r = i / N, c = i % N;
    Q[r * LD + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int step = 0; step < N - 1; ++step) {
      if (tid < NP) {
        int p, q;
        js_pair<N>(step, tid, p, q);
        double4 r = make_double4(1.0, 0.0, 1.0, 0.0);  // cs, sn, ph.re, ph.im ; identity
        if (q < n) {
          double a = G[p * LD + p].x, b = G[q * LD + q].x;
          double2 c = G[p * LD + q];
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
      // columns: G <- G J, Q <- Q J.  Every thread owns IT items; all their
      // LDS loads are issued before any arithmetic so the latencies overlap.
      {
        constexpr int IT = (N * NP + 255) / 256;
        double4 rr[IT];
        int pp[IT], qq_[IT], row_[IT];
        double2 gp[IT], gq[IT], qp[IT], qv[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
          int it = tid + 256 * u;
          int row = it / NP, k = it % NP;
          row_[u] = row;
          js_pair<N>(step, k, pp[u], qq_[u]);
          rr[u] = rot[k];
          gp[u] = G[row * LD + pp[u]];
          gq[u] = G[row * LD + qq_[u]];
          qp[u] = Q[row * LD + pp[u]];
          qv[u] = Q[row * LD + qq_[u]];
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
          const double4 r = rr[u];
          if (r.y == 0.0) continue;
          const double2 em = make_double2(r.z, -r.w);  // e^{-i phi}
          const int row = row_[u];
          double2 gqe = cmul(gq[u], em), qqe = cmul(qv[u], em);
          G[row * LD + pp[u]] = make_double2(r.x * gp[u].x - r.y * gqe.x, r.x * gp[u].y - r.y * gqe.y);
          G[row * LD + qq_[u]] = make_double2(r.y * gp[u].x + r.x * gqe.x, r.y * gp[u].y + r.x * gqe.y);
          Q[row * LD + pp[u]] = make_double2(r.x * qp[u].x - r.y * qqe.x, r.x * qp[u].y - r.y * qqe.y);
          Q[row * LD + qq_[u]] = make_double2(r.y * qp[u].x + r.x * qqe.x, r.y * qp[u].y + r.x * qqe.y);
        }
      }
      __syncthreads();
      // rows: G <- J^dag G
      {
        constexpr int IT = (N * NP + 255) / 256;
        double4 rr[IT];
        int pp[IT], qq_[IT], col_[IT];
        double2 gp[IT], gq[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
          int it = tid + 256 * u;
          int col = it / NP, k = it % NP;
          col_[u] = col;
          js_pair<N>(step, k, pp[u], qq_[u]);
          rr[u] = rot[k];
          gp[u] = G[pp[u] * LD + col];
          gq[u] = G[qq_[u] * LD + col];
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
          const double4 r = rr[u];
          if (r.y == 0.0) continue;
          const double2 ep = make_double2(r.z, r.w);  // e^{+i phi}
          const int col = col_[u];
          double2 gqe = cmul(gq[u], ep);
          G[pp[u] * LD + col] = make_double2(r.x * gp[u].x - r.y * gqe.x, r.x * gp[u].y - r.y * gqe.y);
          G[qq_[u] * LD + col] = make_double2(r.y * gp[u].x + r.x * gqe.x, r.y * gp[u].y + r.x * gqe.y);
        }
      }
      __syncthreads();
      // exact zeros on the rotated pairs keep rounding from accumulating
      if (tid < NP) {
        double4 r = rot[tid];
        if (r.y != 0.0) {
          int p, q;
          js_pair<N>(step, tid, p, q);
          G[p * LD + q] = make_double2(0.0, 0.0);
          G[q * LD + p] = make_double2(0.0, 0.0);
          G[p * LD + p].y = 0.0;
          G[q * LD + q].y = 0.0;
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

__device__ __forceinline__ int herm_jacobi32(double2* G, double2* Q, int n, double abs_thr, double rel_thr,
                                             int max_sweeps, double4* rot, int* flag) {
  return herm_jacobi<32>(G, Q, n, abs_thr, rel_thr, max_sweeps, rot, flag);
}
