// Bond propagators G = exp(-i tau h) for Hermitian two-site h (d*d <= 32).
//
// The local propagator of the plain TEBD update (step 2 of the update listed in
// the appendix on the Krylov method, "calculate local propagator", O(d^6)).
// One workgroup per propagator: h is diagonalised in FP64 by the LDS Jacobi
// solver, h = Q diag(e) Q^dag, then G = Q diag(exp(-i tau e)) Q^dag.
#include "common.h"
#include "jacobi_small.h"

__global__ __launch_bounds__(256) void gates_kernel(const GateJob* __restrict__ jobs, int dd) {
  __shared__ double2 G[JS_N * JS_LD];
  __shared__ double2 Q[JS_N * JS_LD];
  __shared__ double4 rot[16];
  __shared__ int flag;
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const GateJob job = jobs[blockIdx.x];
  const double2* h = job.h;
  double f2 = 0.0;
  for (int i = tid; i < JS_N * JS_N; i += blockDim.x) {
    int r = i / JS_N, c = i % JS_N;
    double2 v = (r < dd && c < dd) ? h[r * dd + c] : make_double2(0.0, 0.0);
    G[r * JS_LD + c] = v;
    f2 += v.x * v.x + v.y * v.y;
  }
  red[tid] = f2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double fro = sqrt(red[0]);
  herm_jacobi32(G, Q, dd, 1e-15 * fro + 1e-300, 0.0, 40, rot, &flag);
  const double t = job.tau;
  for (int i = tid; i < dd * dd; i += blockDim.x) {
    int r = i / dd, c = i % dd;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < dd; ++k) {
      double e = G[k * JS_LD + k].x;
      double sn, cs;
      sincos(-t * e, &sn, &cs);
      double2 qrk = Q[r * JS_LD + k], qck = Q[c * JS_LD + k];
      double2 ph = make_double2(cs, sn);
      double2 v = cmul(qrk, ph);
      acc = cadd(acc, make_double2(v.x * qck.x + v.y * qck.y, v.y * qck.x - v.x * qck.y));
    }
    if (job.G128) job.G128[i] = acc;
    if (job.G64) job.G64[i] = make_float2((float)acc.x, (float)acc.y);
  }
}

hipError_t launch_gates(hipStream_t s, const GateJob* jobs, int n, int dd) {
  if (n <= 0) return hipSuccess;
  if (dd < 1 || dd > 32) return hipErrorInvalidValue;
  gates_kernel<<<n, 256, 0, s>>>(jobs, dd);
  return hipGetLastError();
}
