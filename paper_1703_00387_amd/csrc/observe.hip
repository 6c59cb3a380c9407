// observables of a Hastings-form chain with FP64 accumulation.
//
// Local expectation values from the one-site reduced density matrix
// rho_i = sum lam_i^2 B_i B_i^dag, two-site expectation values from
// theta_b = lam_b B_b B_{b+1}, and the bond entropy S = -sum lam^2 ln lam^2
// (Sec. "Observables", Eq. reducedrho; Sec. "Basic concepts", bond entropy).
#include "common.h"

__global__ void obs_zero_kernel(double* a, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = 0.0;
}

__device__ double obs_block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
  __syncthreads();
  return r;
}

template <class T>
__device__ __forceinline__ double2 ld2(const void* p, size_t i) {
  T v = ((const T*)p)[i];
  return make_double2((double)v.x, (double)v.y);
}

// one workgroup per site
// site_out[i], or with step: site_out[(*step) * step_stride + i] (a log whose
// row the device counter selects, so a replayed graph writes the right row)
template <class T>
__global__ __launch_bounds__(256) void obs_site_kernel(mps_chain_desc c, const double2* __restrict__ op1,
                                                       double* site_out, const int32_t* step = nullptr,
                                                       long long step_stride = 0) {
  __shared__ double red[4];
  const int i = blockIdx.x, d = c.d, cm = c.chi_max;
  const int chl = c.chi[i], chr = c.chi[i + 1];
  const size_t Boff = (size_t)i * cm * d * cm;
  const double* lam = c.lam + (size_t)i * cm;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < chl * chr; idx += blockDim.x) {
    int a = idx / chr, cc = idx % chr;
    double2 v[5];
    for (int s = 0; s < d; ++s) v[s] = ld2<T>(c.B, Boff + ((size_t)a * d + s) * cm + cc);
    double part = 0.0;
    for (int sp = 0; sp < d; ++sp) {
      double2 ov = make_double2(0.0, 0.0);
      for (int s = 0; s < d; ++s) ov = cadd(ov, cmul(op1[sp * d + s], v[s]));
      part += v[sp].x * ov.x + v[sp].y * ov.y;  // Re(conj(v_sp) * ov)
    }
    acc += lam[a] * lam[a] * part;
  }
  double r = obs_block_sum(acc, red);
  if (threadIdx.x == 0) site_out[(step ? (long long)(*step) * step_stride : 0) + i] = r;
}

// grid (chi_max, L-1): workgroup (a, b) adds row a of <theta_b|op2|theta_b>
template <class T>
__global__ __launch_bounds__(256) void obs_bond_kernel(mps_chain_desc c, const double2* __restrict__ op2,
                                                       int per_bond, double* bond_out) {
  __shared__ double2 Bl[2560];  // d * chi <= 2560
  __shared__ double red[4];
  const int a = blockIdx.x, b = blockIdx.y, d = c.d, cm = c.chi_max, dd = d * d;
  const int chl = c.chi[b], chm = c.chi[b + 1], chr = c.chi[b + 2];
  if (a >= chl) return;
  const size_t B0 = (size_t)b * cm * d * cm;
  const size_t B1 = (size_t)(b + 1) * cm * d * cm;
  const double2* O = op2 + (per_bond ? (size_t)b * dd * dd : 0);
  for (int idx = threadIdx.x; idx < d * chm; idx += blockDim.x) {
    int s = idx / chm, be = idx % chm;
    Bl[s * chm + be] = ld2<T>(c.B, B0 + ((size_t)a * d + s) * cm + be);
  }
  __syncthreads();
  double acc = 0.0;
  for (int cc = threadIdx.x; cc < chr; cc += blockDim.x) {
    double2 th[25];
    for (int q = 0; q < dd; ++q) th[q] = make_double2(0.0, 0.0);
    for (int be = 0; be < chm; ++be) {
      for (int t = 0; t < d; ++t) {
        double2 r = ld2<T>(c.B, B1 + ((size_t)be * d + t) * cm + cc);
        for (int s = 0; s < d; ++s) th[s * d + t] = cadd(th[s * d + t], cmul(Bl[s * chm + be], r));
      }
    }
    double part = 0.0;
    for (int p = 0; p < dd; ++p) {
      double2 ov = make_double2(0.0, 0.0);
      for (int q = 0; q < dd; ++q) ov = cadd(ov, cmul(O[p * dd + q], th[q]));
      part += th[p].x * ov.x + th[p].y * ov.y;
    }
    acc += part;
  }
  const double la = c.lam[(size_t)b * cm + a];
  double r = obs_block_sum(acc, red);
  if (threadIdx.x == 0) atomicAdd(&bond_out[b], la * la * r);
}

__global__ void obs_entropy_kernel(mps_chain_desc c, double* ent) {
  __shared__ double red[4];
  const int b = blockIdx.x, cm = c.chi_max;
  const int k = c.chi[b + 1];
  const double* lam = c.lam + (size_t)(b + 1) * cm;
  double acc = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double p = lam[j] * lam[j];
    if (p > 0.0) acc -= p * log(p);
  }
  double r = obs_block_sum(acc, red);
  if (threadIdx.x == 0) ent[b] = r;
}

hipError_t launch_observe(hipStream_t s, const mps_chain_desc& c, const double2* op1, double* site_out,
                          const double2* op2, int op2_per_bond, double* bond_out, double* entropy_out) {
  if (op1 && site_out) {
    if (c.dtype == 1)
      obs_site_kernel<double2><<<c.L, 256, 0, s>>>(c, op1, site_out);
    else
      obs_site_kernel<float2><<<c.L, 256, 0, s>>>(c, op1, site_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (op2 && bond_out && c.L > 1) {
    obs_zero_kernel<<<1, 256, 0, s>>>(bond_out, c.L - 1);
    dim3 grid(c.chi_max, c.L - 1);
    if (c.dtype == 1)
      obs_bond_kernel<double2><<<grid, 256, 0, s>>>(c, op2, op2_per_bond, bond_out);
    else
      obs_bond_kernel<float2><<<grid, 256, 0, s>>>(c, op2, op2_per_bond, bond_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (entropy_out && c.L > 1) {
    obs_entropy_kernel<<<c.L - 1, 256, 0, s>>>(c, entropy_out);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_observe_log(hipStream_t s, const mps_chain_desc& c, const double2* op1, double* log,
                              const int32_t* step, long long step_stride) {
  if (c.dtype == 1)
    obs_site_kernel<double2><<<c.L, 256, 0, s>>>(c, op1, log, step, step_stride);
  else
    obs_site_kernel<float2><<<c.L, 256, 0, s>>>(c, op1, log, step, step_stride);
  return hipGetLastError();
}
