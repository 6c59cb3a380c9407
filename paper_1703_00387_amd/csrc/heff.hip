// Structured effective Hamiltonian, environment updates and Lanczos vector
// kernels for the local Krylov (two-site TDVP) path.
//
// Effective Hamiltonian (Sec. "Fundamentals of the library", Fig.
// LanczosMPS): the left and right environments and the MPO matrices of the
// active sites are applied to the two-site tensor one contraction at a time,
// never forming the chi^2 d^2 square matrix:
//   X1[a',b,s,t,c]  = sum_a   L[a',b,a] x[a,s,t,c]                  (MFMA GEMM)
//   X2[a',g,s',t,c] = sum_b,s W1[b,g,s',s] X1[a',b,s,t,c]           (MPO mix)
//   X3[a',s',t',e,c]= sum_g,t W2[g,e,t',t] X2[a',g,s',t,c]          (MPO mix)
//   y[a',s',t',c']  = sum_e,c X3[a',s',t',e,c] R[c',e,c]             (MFMA GEMM)
// The Lanczos recurrence of Sec. "Krylov time evolution" (Eq.
// krylov:approx) runs on FP64 vectors: multi-vector inner products, the
// Gram-Schmidt subtraction and the final combination are wavefront
// reductions / streaming kernels; the exponential of the small tridiagonal
// matrix uses the LDS Jacobi eigensolver in one workgroup.
#include <algorithm>
#include <type_traits>

#include "mfma_3m.h"
#include "jacobi_small.h"
#include "krylov_small.h"

// ---------------------------------------------------------------------------
// strided complex GEMM: C = alpha op(A) op(B), element strides, optional conj
// ---------------------------------------------------------------------------

// Tile (32 MI) x (32 NJ) per 256-thread workgroup (2 x 2 waves); the shape is
// chosen per (precision, shape class) from the table the autotuner fills.
template <class T, int MI, int NJ>
struct SGemmLds {
  static constexpr int kElems = 2 * TBK * (32 * MI + 4 + 32 * NJ + 4);
};

// Output tile (tm, tn) of P; stage holds SGemmLds<T, MI, NJ>::kElems elements
// (two staging buffers, each an A and a B chunk).
template <class T, int MI, int NJ>
__device__ __forceinline__ void sgemm_tile(const SGemm& P, int tm, int tn, T* stage) {
  constexpr int BM = 32 * MI, BN = 32 * NJ, LDA = BM + 4, LDB = BN + 4;
  constexpr int PA = BM >= 64 ? BM / 64 : 1, PB = BN >= 64 ? BN / 64 : 1;
  // chunks in flight in registers: two for complex128, one for complex64
  // (measured fastest with the three accumulators of either precision)
  constexpr int kPf = sizeof(T) == 16 ? 2 : 1;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * MI * 16, wn = (wave & 1) * NJ * 16;
  const T* A = (const T*)P.A;
  const T* B = (const T*)P.B;
  T* C = (T*)P.C;
  // three real products per complex one (mfma_3m.h)
  Acc3<T, MI, NJ> acc;
  acc_clear(acc);
  const int ia = tid >> 2, kqa = (tid & 3) * 4;
  const int kb = tid >> 4, jqb = (tid & 15) * 4;
  T va[kPf][PA][4], vb[kPf][PB][4];
  auto load = [&](int ci, T (*da)[4], T (*db)[4]) {
    const int k0 = ci * TBK;
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int row = ia + 64 * q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int k = k0 + kqa + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (row < BM && m0 + row < P.M && k < P.K) {
          v = A[(long long)(m0 + row) * P.rsA + (long long)k * P.csA];
          if (P.conjA) v.y = -v.y;
        }
        da[q][e] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int j = jqb + 64 * q + e;
        T v = Cx<T>::make(0.0, 0.0);
        if (j < BN && n0 + j < P.N && k0 + kb < P.K) {
          v = B[(long long)(k0 + kb) * P.rsB + (long long)(n0 + j) * P.csB];
          if (P.conjB) v.y = -v.y;
        }
        db[q][e] = v;
      }
    }
  };
  auto store = [&](int buf, T (*da)[4], T (*db)[4]) {
    T* As = stage + buf * TBK * (LDA + LDB);
    T* Bs = As + TBK * LDA;
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int row = ia + 64 * q;
      if (row < BM) {
#pragma unroll
        for (int e = 0; e < 4; ++e) As[(kqa + e) * LDA + row] = da[q][e];
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = jqb + 64 * q + e;
        if (j < BN) Bs[kb * LDB + j] = db[q][e];
      }
    }
  };
  const int nch = (P.K + TBK - 1) / TBK;
#pragma unroll
  for (int u = 0; u < kPf; ++u)
    if (u < nch) load(u, va[u], vb[u]);
  if (nch > 0) store(0, va[0], vb[0]);
  __syncthreads();
  for (int base = 0; base < nch; base += kPf) {
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
      const int ci = base + u;
      if (ci < nch) {
        if (ci + kPf < nch) load(ci + kPf, va[u], vb[u]);  // chunk ci's registers were staged already
        const T* As = stage + (ci & 1) * TBK * (LDA + LDB);
        acc_chunk(As, LDA, As + TBK * LDA, LDB, acc, wm, wn, lane);
        if (ci + 1 < nch) store((ci + 1) & 1, va[(u + 1) % kPf], vb[(u + 1) % kPf]);
        __syncthreads();
      }
    }
  }
  typedef typename Cx<T>::R R;
  const R alpha = P.alpha_dev ? (R)(*P.alpha_dev) : (R)P.alpha;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm + i * 16 + Cx<T>::acc_row(lane, r);
        int col = n0 + wn + j * 16 + (lane & 15);
        if (row < P.M && col < P.N) {
          T v = acc_value(acc, i, j, r);
          v.x *= alpha;
          v.y *= alpha;
          C[(long long)row * P.rsC + (long long)col * P.csC] = v;
        }
      }
}

template <class T, int MI, int NJ>
__global__ __launch_bounds__(256) void sgemm_kernel(SGemm P, int ntn) {
  __shared__ T stage[SGemmLds<T, MI, NJ>::kElems];
  sgemm_tile<T, MI, NJ>(P, blockIdx.x / ntn, blockIdx.x % ntn, stage);
}

// A batch of independent products, problem blockIdx.y; the grid covers the
// largest, tiles past a problem's dimensions return at once.
template <class T, int MI, int NJ>
__global__ __launch_bounds__(256) void sgemm_batched_kernel(const SGemm* __restrict__ probs, int ntn) {
  __shared__ T stage[SGemmLds<T, MI, NJ>::kElems];
  const SGemm P = probs[blockIdx.y];
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  if (tm * 32 * MI >= P.M || tn * 32 * NJ >= P.N) return;
  sgemm_tile<T, MI, NJ>(P, tm, tn, stage);
}

hipError_t launch_sgemm_batched(hipStream_t s, const SGemm* probs, int n_probs, int M_max, int N_max) {
  if (n_probs <= 0 || M_max <= 0 || N_max <= 0) return hipSuccess;
  if (n_probs > 65535) return hipErrorInvalidValue;
  const int ntm = (M_max + 63) / 64, ntn = (N_max + 63) / 64;
  sgemm_batched_kernel<double2, 2, 2><<<dim3(ntm * ntn, n_probs), 256, 0, s>>>(probs, ntn);
  return hipGetLastError();
}

// Tile shape per (precision, shape class), candidate indices of
// gemm_cand_mi / gemm_cand_nj; 0 (64 x 64) until the autotuner sets one.
static int g_sgemm_choice[2][kGemmShapeClasses] = {};

int gemm_shape_class(long long M, long long N) {
  if (M * N <= 64LL * 64 * 64) return 0;   // at most 64 default tiles: few workgroups
  if (M >= 2 * N) return 1;                // tall
  if (N >= 2 * M) return 2;                // wide
  return 3;
}

void set_sgemm_choice(bool c128, int shape_class, int cand) { g_sgemm_choice[c128 ? 1 : 0][shape_class] = cand; }
int get_sgemm_choice(bool c128, int shape_class) { return g_sgemm_choice[c128 ? 1 : 0][shape_class]; }

template <class T, int MI, int NJ>
static hipError_t sgemm_go(hipStream_t s, const SGemm& P) {
  const int ntm = (P.M + 32 * MI - 1) / (32 * MI), ntn = (P.N + 32 * NJ - 1) / (32 * NJ);
  sgemm_kernel<T, MI, NJ><<<ntm * ntn, 256, 0, s>>>(P, ntn);
  return hipGetLastError();
}

template <class T>
static hipError_t sgemm_cand(hipStream_t s, const SGemm& P, int cand) {
  switch (cand) {
    case 1: return sgemm_go<T, 4, 2>(s, P);
    case 2: return sgemm_go<T, 2, 4>(s, P);
    case 3: return sgemm_go<T, 1, 2>(s, P);
    case 4: return sgemm_go<T, 2, 1>(s, P);
    case 5: return sgemm_go<T, 1, 1>(s, P);
    default: return sgemm_go<T, 2, 2>(s, P);
  }
}

hipError_t launch_sgemm_cand(hipStream_t s, const SGemm& P, bool c128, int cand) {
  if (P.M <= 0 || P.N <= 0) return hipSuccess;
  return c128 ? sgemm_cand<double2>(s, P, cand) : sgemm_cand<float2>(s, P, cand);
}

hipError_t launch_sgemm(hipStream_t s, const SGemm& P, bool c128) {
  return launch_sgemm_cand(s, P, c128, get_sgemm_choice(c128, gemm_shape_class(P.M, P.N)));
}

// ---------------------------------------------------------------------------
// MPO mix: out[o1,o2,(qo1,qo2),r] = sum_(qi1,qi2) Wm[(qo1 qo2),(qi1 qi2)] in[o1,o2,(qi1,qi2),r]
// with independent strides; Wm is built on the device from the MPO tensor.
// ---------------------------------------------------------------------------

// Wm[(qo1*O2+qo2)*(Q1*Q2) + qi1*Q2+qi2] = W[qo1*ws_o1 + qo2*ws_o2 + qi1*ws_i1 + qi2*ws_i2]
template <class T>
__global__ void wmix_build_kernel(const T* W, T* Wm, int O1, int O2, int Q1, int Q2, int ws_o1, int ws_o2,
                                  int ws_i1, int ws_i2) {
  int n = O1 * O2 * Q1 * Q2;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int qi = e % (Q1 * Q2), qo = e / (Q1 * Q2);
    int qo1 = qo / O2, qo2 = qo % O2, qi1 = qi / Q2, qi2 = qi % Q2;
    Wm[e] = W[qo1 * ws_o1 + qo2 * ws_o2 + qi1 * ws_i1 + qi2 * ws_i2];
  }
}

template <class T>
__global__ __launch_bounds__(256) void mix_kernel(MixDesc D, const T* __restrict__ in, const T* __restrict__ Wm,
                                                  T* __restrict__ out) {
  __shared__ T Ws[32 * 32];
  typedef typename Cx<T>::R R;
  const int Qi = D.Q1 * D.Q2, Qo = D.O1 * D.O2;
  for (int e = threadIdx.x; e < Qi * Qo; e += blockDim.x) Ws[e] = Wm[e];
  __syncthreads();
  const long long total = (long long)D.P1 * D.P2 * D.R;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    int r = (int)(idx % D.R);
    long long rest = idx / D.R;
    int o2 = (int)(rest % D.P2), o1 = (int)(rest / D.P2);
    const T* ip = in + o1 * D.is_o1 + o2 * D.is_o2 + r * D.is_r;
    // the (up to 32) inputs of this position, fully unrolled so they stay in registers
    T x[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      x[q] = Cx<T>::make(0.0, 0.0);
      if (q < Qi) {
        const int q1 = q / D.Q2, q2 = q - q1 * D.Q2;
        x[q] = ip[q1 * D.is_q1 + q2 * D.is_q2];
      }
    }
    T* op = out + o1 * D.os_o1 + o2 * D.os_o2 + r * D.os_r;
    for (int p = 0; p < Qo; ++p) {
      const int p1 = p / D.O2, p2 = p - p1 * D.O2;
      const T* w = Ws + p * Qi;
      R ar = 0, ai = 0;
#pragma unroll
      for (int q = 0; q < 32; ++q) {
        if (q < Qi) {
          const T wq = w[q];
          ar += wq.x * x[q].x - wq.y * x[q].y;
          ai += wq.x * x[q].y + wq.y * x[q].x;
        }
      }
      T v;
      v.x = ar;
      v.y = ai;
      op[p1 * D.os_q1 + p2 * D.os_q2] = v;
    }
  }
}

hipError_t launch_wmix_build(hipStream_t s, const void* W, void* Wm, int O1, int O2, int Q1, int Q2, int ws_o1,
                             int ws_o2, int ws_i1, int ws_i2, bool c128) {
  if (c128)
    wmix_build_kernel<double2><<<1, 256, 0, s>>>((const double2*)W, (double2*)Wm, O1, O2, Q1, Q2, ws_o1, ws_o2,
                                                ws_i1, ws_i2);
  else
    wmix_build_kernel<float2><<<1, 256, 0, s>>>((const float2*)W, (float2*)Wm, O1, O2, Q1, Q2, ws_o1, ws_o2, ws_i1,
                                               ws_i2);
  return hipGetLastError();
}

hipError_t launch_mix(hipStream_t s, const MixDesc& D, const void* in, const void* Wm, void* out, bool c128) {
  long long total = (long long)D.P1 * D.P2 * D.R;
  if (total <= 0) return hipSuccess;
  int g = (int)std::min<long long>((total + 255) / 256, 8192);
  if (c128)
    mix_kernel<double2><<<g, 256, 0, s>>>(D, (const double2*)in, (const double2*)Wm, (double2*)out);
  else
    mix_kernel<float2><<<g, 256, 0, s>>>(D, (const float2*)in, (const float2*)Wm, (float2*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 Lanczos vector kernels
// ---------------------------------------------------------------------------
__global__ void zero_kernel(double* a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0.0;
}

// part[block][i] = this block's share of <V_i, r> for i < nv (complex,
// V_i = V + i*ldv); a fixed grid-stride order, wave shuffles and a fixed
// order over the waves, so the shares do not depend on scheduling
__global__ __launch_bounds__(256) void mdot_kernel(const double2* __restrict__ V, long long ldv, int nv,
                                                   const double2* __restrict__ r, long long n, double2* part) {
  __shared__ double red[2 * 32 * 4];
  double2 acc[32];
  for (int i = 0; i < nv; ++i) acc[i] = make_double2(0.0, 0.0);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double2 x = r[e];
    for (int i = 0; i < nv; ++i) {
      double2 v = V[i * ldv + e];
      acc[i].x += v.x * x.x + v.y * x.y;
      acc[i].y += v.x * x.y - v.y * x.x;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = 0; i < nv; ++i) {
    double a = acc[i].x, b = acc[i].y;
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      b += __shfl_xor(b, o);
    }
    if (lane == 0) {
      red[(i * 4 + wave) * 2] = a;
      red[(i * 4 + wave) * 2 + 1] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    int i = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 4; ++w) {
      a += red[(i * 4 + w) * 2];
      b += red[(i * 4 + w) * 2 + 1];
    }
    part[(long long)blockIdx.x * nv + i] = make_double2(a, b);
  }
}

// out[i] += sum over the blocks' shares, in block order (deterministic)
__global__ void mdot_sum_kernel(const double2* __restrict__ part, int n_blocks, int nv, double2* out) {
  const int i = threadIdx.x;
  if (i >= nv) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < n_blocks; ++k) {
    const double2 v = part[(long long)k * nv + i];
    a += v.x;
    b += v.y;
  }
  out[i] = make_double2(out[i].x + a, out[i].y + b);
}

// r -= sum_i c_i V_i ; if alpha_out: alpha_out[0] = Re c_{nv-1} (first pass only)
__global__ __launch_bounds__(256) void msub_kernel(const double2* __restrict__ V, long long ldv, int nv,
                                                   const double2* __restrict__ c, double2* r, long long n) {
  __shared__ double2 cs[32];
  if (threadIdx.x < nv) cs[threadIdx.x] = c[threadIdx.x];
  __syncthreads();
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double2 x = r[e];
    for (int i = 0; i < nv; ++i) {
      double2 v = V[i * ldv + e];
      x.x -= cs[i].x * v.x - cs[i].y * v.y;
      x.y -= cs[i].x * v.y + cs[i].y * v.x;
    }
    r[e] = x;
  }
}

// y = x * (1 / sqrt(*norm2))
__global__ void scale_inv_sqrt_kernel(const double2* x, double2* y, long long n, const double* norm2) {
  double s = *norm2 > 0.0 ? 1.0 / sqrt(*norm2) : 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double2 v = x[e];
    y[e] = make_double2(v.x * s, v.y * s);
  }
}

// x = nrm * sum_i u_i V_i
__global__ void combine_kernel(const double2* __restrict__ V, long long ldv, int nv, const double2* __restrict__ u,
                               double nrm, double2* x, long long n) {
  __shared__ double2 us[32];
  if (threadIdx.x < nv) us[threadIdx.x] = u[threadIdx.x];
  __syncthreads();
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double2 a = make_double2(0.0, 0.0);
    for (int i = 0; i < nv; ++i) {
      double2 v = V[i * ldv + e];
      a.x += us[i].x * v.x - us[i].y * v.y;
      a.y += us[i].x * v.y + us[i].y * v.x;
    }
    x[e] = make_double2(nrm * a.x, nrm * a.y);
  }
}

// precision conversion between the FP64 Krylov vectors and the apply dtype
__global__ void c128_to_c64_kernel(const double2* a, float2* b, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    b[e] = make_float2((float)a[e].x, (float)a[e].y);
}
__global__ void c64_to_c128_kernel(const float2* a, double2* b, long long n) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    b[e] = make_double2(a[e].x, a[e].y);
}

// Tridiagonal exponential of the Lanczos matrix (one workgroup).
__global__ __launch_bounds__(256) void tridiag_expm_kernel(const double* alpha, const double* beta, int n,
                                                           double tau_re, double tau_im, double nrm,
                                                           double2* u, double* err) {
  __shared__ double2 G[JS_N * JS_LD];
  __shared__ double2 Q[JS_N * JS_LD];
  __shared__ double4 rot[16];
  __shared__ int flag;
  tridiag_expm_block(alpha, beta, n, tau_re, tau_im, nrm, u, err, G, Q, rot, &flag);
}

static int vgrid(long long n) { return (int)std::min<long long>((n + 255) / 256, 4096); }

hipError_t launch_zero(hipStream_t s, double* a, int n) {
  zero_kernel<<<std::max(1, std::min(64, (n + 255) / 256)), 256, 0, s>>>(a, n);
  return hipGetLastError();
}
hipError_t launch_mdot(hipStream_t s, const double2* V, long long ldv, int nv, const double2* r, long long n,
                       double2* out, double2* part) {
  if (nv < 1 || nv > 32) return hipErrorInvalidValue;
  const int g = std::min(vgrid(n), kMdotBlocks);
  mdot_kernel<<<g, 256, 0, s>>>(V, ldv, nv, r, n, part);
  mdot_sum_kernel<<<1, 64, 0, s>>>(part, g, nv, out);
  return hipGetLastError();
}
hipError_t launch_msub(hipStream_t s, const double2* V, long long ldv, int nv, const double2* c, double2* r,
                       long long n) {
  msub_kernel<<<vgrid(n), 256, 0, s>>>(V, ldv, nv, c, r, n);
  return hipGetLastError();
}
hipError_t launch_scale_inv_sqrt(hipStream_t s, const double2* x, double2* y, long long n, const double* norm2) {
  scale_inv_sqrt_kernel<<<vgrid(n), 256, 0, s>>>(x, y, n, norm2);
  return hipGetLastError();
}
hipError_t launch_combine(hipStream_t s, const double2* V, long long ldv, int nv, const double2* u, double nrm,
                          double2* x, long long n) {
  combine_kernel<<<vgrid(n), 256, 0, s>>>(V, ldv, nv, u, nrm, x, n);
  return hipGetLastError();
}
hipError_t launch_convert(hipStream_t s, const void* a, void* b, long long n, bool to_c64) {
  if (to_c64)
    c128_to_c64_kernel<<<vgrid(n), 256, 0, s>>>((const double2*)a, (float2*)b, n);
  else
    c64_to_c128_kernel<<<vgrid(n), 256, 0, s>>>((const float2*)a, (double2*)b, n);
  return hipGetLastError();
}
hipError_t launch_tridiag_expm(hipStream_t s, const double* alpha, const double* beta, int n, double tau_re,
                               double tau_im, double nrm, double2* u, double* err) {
  tridiag_expm_kernel<<<1, 256, 0, s>>>(alpha, beta, n, tau_re, tau_im, nrm, u, err);
  return hipGetLastError();
}

// b[j][i] = a[i][j], a: m x n complex128
__global__ void transpose_c128_kernel(const double2* a, double2* b, int m, int n) {
  __shared__ double2 t[32][33];
  int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    int i = by + k, j = bx + threadIdx.x;
    if (i < m && j < n) t[k][threadIdx.x] = a[(size_t)i * n + j];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    int j = bx + k, i = by + threadIdx.x;
    if (i < m && j < n) b[(size_t)j * m + i] = t[threadIdx.x][k];
  }
}

hipError_t launch_transpose_c128(hipStream_t s, const double2* a, double2* b, int m, int n) {
  dim3 grid((n + 31) / 32, (m + 31) / 32), block(32, 8);
  transpose_c128_kernel<<<grid, block, 0, s>>>(a, b, m, n);
  return hipGetLastError();
}

// normalised kept rows of a converged Jacobi matrix: row j (sorted) divided
// by s_j, written as dst[j*len + e] (row-major) or dst[e*k + j] (column-major)
template <class T>
__global__ void write_rows_kernel(const JacMat* mat, const int32_t* perm, const double* s2, const SelOut* sel, T* dst,
                                  int len, int col_major) {
  const int k = sel->k;
  const JacMat M = *mat;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < (long long)k * len;
       idx += (long long)gridDim.x * blockDim.x) {
    int j = (int)(idx / len), e = (int)(idx % len);
    int pj = perm[j];
    pj = (pj >= 0 && pj < M.m) ? pj : 0;
    double s = sqrt(s2[j]);
    double inv = s > 0.0 ? 1.0 / s : 0.0;
    double2 x = M.X[(size_t)pj * M.ld + e];
    T v;
    v.x = x.x * inv;
    v.y = x.y * inv;
    if (col_major)
      dst[(size_t)e * k + j] = v;
    else
      dst[(size_t)j * len + e] = v;
  }
}

hipError_t launch_write_rows(hipStream_t s, const JacMat* mat, const int32_t* perm, const double* s2, const SelOut* sel,
                             void* dst, int len, int col_major, bool c128) {
  int g = std::max(1, std::min(4096, (len * 64 + 255) / 256));
  if (c128)
    write_rows_kernel<double2><<<g, 256, 0, s>>>(mat, perm, s2, sel, (double2*)dst, len, col_major);
  else
    write_rows_kernel<float2><<<g, 256, 0, s>>>(mat, perm, s2, sel, (float2*)dst, len, col_major);
  return hipGetLastError();
}
