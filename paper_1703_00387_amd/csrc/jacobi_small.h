// Cyclic parallel Jacobi eigensolver for a Hermitian matrix of order <= N
// (N = 32 or 64) held in LDS, run by one workgroup of NT (256 or 512) threads, in FP64.
//
// G  : [N][LD] complex128 in LDS (LD >= N, default N+1), overwritten with Q^dag G Q
// Q  : [N][LD] complex128 in LDS, overwritten with the accumulated unitary
//      (initialised here to the identity); G_in = Q diag(G_out) Q^dag.
// Each step rotates up to N/2 disjoint index pairs of the odd-even ordering
// below, so a sweep of N steps visits every pair once.  The 2x2 rotation for the
// pair (p, q) with a = G_pp, b = G_qq, c = G_pq = |c| e^{i phi} is
//   J = [[cs, sn], [-sn e^{-i phi}, cs e^{-i phi}]],
//   t = sign(tau) / (|tau| + sqrt(1 + tau^2)),  tau = (b - a) / (2|c|),
//   cs = 1/sqrt(1+t^2), sn = t cs,
// which zeroes (J^dag G J)_pq and moves the diagonal to a - t|c|, b + t|c|.
// A pair is skipped when |c| <= max(abs_thr, rel_thr * sqrt(|a b|)).
#pragma once

#define JS_N 32
#define JS_LD 33

// Odd-even transposition ordering with exchange: N slots (N even) hold the N
// indices; step t rotates the index pairs in slots (2k, 2k+1) (t even) or
// (2k+1, 2k+2) (t odd) and then swaps the two indices between their slots,
// so all N(N-1)/2 pairs meet once in N steps.  Unfolding the line of slots
// onto a circle of 2N points (slot x <-> points x and 2N-1-x), every index
// advances one point per step: index e starts at point e (e even) or
// 2N-1-e (e odd).  That gives the index in slot x at step t in closed form.
__device__ __forceinline__ int oe_index(int N, int t, int x) {
  const int y = ((x ^ t) & 1) ? 2 * N - 1 - x : x;   // the occupied point of slot x
  int y0 = (y - t) % (2 * N);
  if (y0 < 0) y0 += 2 * N;
  return y0 < N ? y0 : 2 * N - 1 - y0;
}

// Pair k of step t (p < q); false when slot 2k+1+(t&1) is past the end.
__device__ __forceinline__ bool oe_pair(int N, int t, int k, int& p, int& q) {
  const int x = 2 * k + (t & 1);
  if (x + 1 >= N) return false;
  const int a = oe_index(N, t, x), b = oe_index(N, t, x + 1);
  p = a < b ? a : b;
  q = a < b ? b : a;
  return true;
}

template <int N>
__device__ __forceinline__ bool js_pair(int step, int k, int& p, int& q) {
  return oe_pair(N, step, k, p, q);
}

// Returns the number of sweeps used (<= max_sweeps).  Exactly NT threads call it.
template <int N, int LD = N + 1, int NT = 256>
__device__ int herm_jacobi(double2* G, double2* Q, int n, double abs_thr, double rel_thr, int max_sweeps,
                           double4* rot /* LDS [N/2] */, int* flag /* LDS */) {
  constexpr int NP = N / 2;
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
    for (int step = 0; step < N; ++step) {
      if (tid < NP) {
        int p, q;
        const bool valid = js_pair<N>(step, tid, p, q);
        double4 r = make_double4(1.0, 0.0, 1.0, 0.0);  // cs, sn, ph.re, ph.im ; identity
        if (valid && q < n) {
          double a = G[p * LD + p].x, b = G[q * LD + q].x;
          double2 c = G[p * LD + q];
          double ac2 = c.x * c.x + c.y * c.y;
          // |c| > max(abs_thr, rel_thr sqrt|ab|), compared in squares
          double thr2 = fmax(abs_thr * abs_thr, rel_thr * rel_thr * fabs(a * b));
          if (ac2 > thr2 && ac2 > 0.0) {
            double iac = 1.0 / sqrt(ac2);
            double tau = 0.5 * (b - a) * iac;
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            double cs = 1.0 / sqrt(1.0 + t * t);
            r = make_double4(cs, t * cs, c.x * iac, c.y * iac);
            *flag = 1;
          }
        }
        rot[tid] = r;
      }
      __syncthreads();
      // G <- J^dag G J with the rotations of this step (disjoint pairs):
      // first the columns, G <- G J and Q <- Q J, then the rows, G <- J^dag G.
      // Item (k, row) of the column pass updates entries (row, p_k) and
      // (row, q_k); the lanes of a wave take consecutive rows of one pair, so
      // their LDS accesses fall in distinct banks.  Item u of a thread is pair
      // k = tid / N + u NT / N at row (or column) tid % N (NT is a multiple of
      // N).  Items go in batches of UB, every load of a batch issued before
      // its arithmetic; with two waves per SIMD, batches of two keep the
      // registers within the halved budget.
      static_assert(NT % N == 0, "thread count must be a multiple of the order");
      // for a small order (N * NP < NT) the first N * NP threads hold one item each
      constexpr int IT = (N * NP + NT - 1) / NT, KS = NT / N;
      constexpr int UB = NT >= 512 ? (IT < 2 ? IT : 2) : IT;
      const int row = tid % N, k0 = tid / N;
      const bool active = k0 < NP;
#pragma unroll
      for (int u0 = 0; u0 < IT && active; u0 += UB) {
        double4 rr[UB];
        int pp[UB], qq_[UB];
        double2 gp[UB], gq[UB], qp[UB], qv[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int k = k0 + (u0 + u) * KS;
          rr[u] = rot[k];
          if (!js_pair<N>(step, k, pp[u], qq_[u])) rr[u].y = 0.0;
          if (rr[u].y != 0.0) {
            gp[u] = G[row * LD + pp[u]];
            gq[u] = G[row * LD + qq_[u]];
            qp[u] = Q[row * LD + pp[u]];
            qv[u] = Q[row * LD + qq_[u]];
          }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const double4 r = rr[u];
          if (r.y == 0.0) continue;
          const double2 em = make_double2(r.z, -r.w);  // e^{-i phi}
          double2 gqe = cmul(gq[u], em), qqe = cmul(qv[u], em);
          G[row * LD + pp[u]] = make_double2(r.x * gp[u].x - r.y * gqe.x, r.x * gp[u].y - r.y * gqe.y);
          G[row * LD + qq_[u]] = make_double2(r.y * gp[u].x + r.x * gqe.x, r.y * gp[u].y + r.x * gqe.y);
          Q[row * LD + pp[u]] = make_double2(r.x * qp[u].x - r.y * qqe.x, r.x * qp[u].y - r.y * qqe.y);
          Q[row * LD + qq_[u]] = make_double2(r.y * qp[u].x + r.x * qqe.x, r.y * qp[u].y + r.x * qqe.y);
        }
      }
      __syncthreads();
      // Rows: G <- J^dag G, item (k, col); the rotated pair's own entries are
      // set exactly (zero coupling, real diagonal) so rounding does not build up.
      const int col = tid % N;
#pragma unroll
      for (int u0 = 0; u0 < IT && active; u0 += UB) {
        double4 rr[UB];
        int pp[UB], qq_[UB];
        double2 gp[UB], gq[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int k = k0 + (u0 + u) * KS;
          rr[u] = rot[k];
          if (!js_pair<N>(step, k, pp[u], qq_[u])) rr[u].y = 0.0;
          if (rr[u].y != 0.0) {
            gp[u] = G[pp[u] * LD + col];
            gq[u] = G[qq_[u] * LD + col];
          }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const double4 r = rr[u];
          if (r.y == 0.0) continue;
          const double2 ep = make_double2(r.z, r.w);  // e^{+i phi}
          double2 gqe = cmul(gq[u], ep);
          double2 np_ = make_double2(r.x * gp[u].x - r.y * gqe.x, r.x * gp[u].y - r.y * gqe.y);
          double2 nq_ = make_double2(r.y * gp[u].x + r.x * gqe.x, r.y * gp[u].y + r.x * gqe.y);
          if (col == pp[u]) {
            np_.y = 0.0;
            nq_ = make_double2(0.0, 0.0);
          } else if (col == qq_[u]) {
            np_ = make_double2(0.0, 0.0);
            nq_.y = 0.0;
          }
          G[pp[u] * LD + col] = np_;
          G[qq_[u] * LD + col] = nq_;
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

// Order n <= 32 in the JS_N x JS_LD arrays: the sweep runs over the smallest
// power of two >= n (4 ... 32), so a small matrix takes fewer steps per sweep.
__device__ __forceinline__ int herm_jacobi32(double2* G, double2* Q, int n, double abs_thr, double rel_thr,
                                             int max_sweeps, double4* rot, int* flag) {
  if (n <= 4) return herm_jacobi<4, JS_LD>(G, Q, n, abs_thr, rel_thr, max_sweeps, rot, flag);
  if (n <= 8) return herm_jacobi<8, JS_LD>(G, Q, n, abs_thr, rel_thr, max_sweeps, rot, flag);
  if (n <= 16) return herm_jacobi<16, JS_LD>(G, Q, n, abs_thr, rel_thr, max_sweeps, rot, flag);
  return herm_jacobi<32, JS_LD>(G, Q, n, abs_thr, rel_thr, max_sweeps, rot, flag);
}

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by
// two Newton steps (quadratic convergence from the estimate; the last step
// leaves about one ulp).  Four dependent FMAs each instead of the rounded
// library square root and division.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double r = fma(-h * y, y, 0.5);
    y = fma(y, r, y);
  }
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

// Order 64: herm_jacobi<64> (same ordering, thresholds, 2x2 rotations and
// order of operations; the angle comes from refined reciprocal estimates, so
// results agree to rounding) arranged for the case that matters in the block
// Jacobi, where the 64 x 64 Gram is nearly diagonal and only a few of a
// step's 32 pairs rotate (about 4 on average in TEBD).  A step is then bound
// by its chain of dependent LDS round trips, not by arithmetic:
//  * the 32 lanes that form the step's rotations also list the rotating
//    pairs, with their rotation and indices (p, q), in LDS;
//  * the column and row passes run over the items (listed pair, row or
//    column) spread evenly over the workgroup; a thread reads its items'
//    records once, together with the count, and keeps them for both passes;
//  * a step with no rotation costs one barrier.
// The list is double-buffered by the step's parity, so the next step can
// start forming its own while a slower wave still reads it.
// scr: LDS scratch of at least kJac64Scratch double2.
constexpr int kJac64Scratch = 2 * (32 * 2 + 32 / 2) + 1;
template <int NT, int LD = 65>
__device__ int herm_jacobi64(double2* G, double2* Q, double abs_thr, double rel_thr, int max_sweeps,
                             double2* scr, int* flag) {
  constexpr int N = 64, NP = 32, MI = N * NP / NT;  // MI: items per thread at most
  double4* lrot = reinterpret_cast<double4*>(scr);  // [2][32] rotation of listed pair j: cs, sn, e^{i phi}
  int2* lpq = reinterpret_cast<int2*>(lrot + 2 * NP);  // [2][32] its (p, q)
  int* nrot = reinterpret_cast<int*>(lpq + 2 * NP);    // [2]
  const int tid = threadIdx.x;
  for (int i = tid; i < N * N; i += NT) {
    const int r = i / N, c = i % N;
    Q[r * LD + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // wave 0: the pair of lane tid in the coming step, formed while the
  // previous step's writes drain
  int p = 0, q = 0;
  bool valid = tid < NP && js_pair<N>(0, tid, p, q);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int step = 0; step < N; ++step) {
      const int bf = step & 1;
      if (tid < 64) {  // wave 0 forms and lists the step's rotations
        bool rotating = false;
        double4 r = make_double4(1.0, 0.0, 1.0, 0.0);
        if (valid) {
          const double a = G[p * LD + p].x, b = G[q * LD + q].x;
          const double2 c = G[p * LD + q];
          const double ac2 = c.x * c.x + c.y * c.y;
          const double thr2 = fmax(abs_thr * abs_thr, rel_thr * rel_thr * fabs(a * b));
          if (ac2 > thr2 && ac2 > 0.0) {
            // the angle is on the step's critical path: t and the unit phase
            // from refined reciprocal estimates (t needs no last-bit accuracy;
            // cs = (1 + t^2)^(-1/2) and e^{i phi} = c / |c| keep the rotation
            // unitary to about an ulp)
            // (a coupling near the bottom of the normal range takes the
            // library square root, which handles subnormal |c|^2)
            const double iac = ac2 > 1e-280 ? rsqrt_nr(ac2) : 1.0 / sqrt(ac2);
            const double tau = 0.5 * (b - a) * iac;
            const double w = fma(tau, tau, 1.0);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + w * rsqrt_nr(w));
            const double cs = rsqrt_nr(fma(t, t, 1.0));
            r = make_double4(cs, t * cs, c.x * iac, c.y * iac);
            rotating = true;
          }
        }
        const unsigned long long m = __ballot(rotating);
        if (rotating) {
          const int j = __popcll(m & ((1ull << tid) - 1ull));
          lrot[bf * NP + j] = r;
          lpq[bf * NP + j] = make_int2(p, q);
        }
        if (tid == 0) {
          nrot[bf] = __popcll(m);
          if (m) *flag = 1;
        }
        p = 0;
        q = 0;
        valid = tid < NP && js_pair<N>(step + 1 < N ? step + 1 : 0, tid, p, q);
      }
      __syncthreads();
      // this thread's items i = tid + u NT: listed pair i / 64 at row (column) i % 64;
      // the records are read with the count (entries past it are not used)
      const int nr = nrot[bf];
      double4 ir[MI];
      int2 ik[MI];
#pragma unroll
      for (int u = 0; u < MI; ++u) {
        const int j = (tid + u * NT) >> 6;
        ir[u] = lrot[bf * NP + j];
        ik[u] = lpq[bf * NP + j];
      }
      if (nr == 0) continue;  // the same for every thread
      const int rc = tid & 63;
      // columns: G <- G J and Q <- Q J
#pragma unroll
      for (int u = 0; u < MI; ++u) {
        if (((tid + u * NT) >> 6) >= nr) break;
        const double4 r = ir[u];
        const int2 kk = ik[u];
        const double2 gp = G[rc * LD + kk.x], gq = G[rc * LD + kk.y];
        const double2 qp = Q[rc * LD + kk.x], qv = Q[rc * LD + kk.y];
        const double2 em = make_double2(r.z, -r.w);  // e^{-i phi}
        const double2 gqe = cmul(gq, em), qqe = cmul(qv, em);
        G[rc * LD + kk.x] = make_double2(r.x * gp.x - r.y * gqe.x, r.x * gp.y - r.y * gqe.y);
        G[rc * LD + kk.y] = make_double2(r.y * gp.x + r.x * gqe.x, r.y * gp.y + r.x * gqe.y);
        Q[rc * LD + kk.x] = make_double2(r.x * qp.x - r.y * qqe.x, r.x * qp.y - r.y * qqe.y);
        Q[rc * LD + kk.y] = make_double2(r.y * qp.x + r.x * qqe.x, r.y * qp.y + r.x * qqe.y);
      }
      __syncthreads();
      // rows: G <- J^dag G; the pair's own entries exactly
#pragma unroll
      for (int u = 0; u < MI; ++u) {
        if (((tid + u * NT) >> 6) >= nr) break;
        const double4 r = ir[u];
        const int2 kk = ik[u];
        const double2 gp = G[kk.x * LD + rc], gq = G[kk.y * LD + rc];
        const double2 ep = make_double2(r.z, r.w);  // e^{+i phi}
        const double2 gqe = cmul(gq, ep);
        double2 np_ = make_double2(r.x * gp.x - r.y * gqe.x, r.x * gp.y - r.y * gqe.y);
        double2 nq_ = make_double2(r.y * gp.x + r.x * gqe.x, r.y * gp.y + r.x * gqe.y);
        if (rc == kk.x) {
          np_.y = 0.0;
          nq_ = make_double2(0.0, 0.0);
        } else if (rc == kk.y) {
          np_ = make_double2(0.0, 0.0);
          nq_.y = 0.0;
        }
        G[kk.x * LD + rc] = np_;
        G[kk.y * LD + rc] = nq_;
      }
      __syncthreads();
    }
    __syncthreads();
    if (*flag == 0) break;
    __syncthreads();
  }
  __syncthreads();
  return sweep;
}
