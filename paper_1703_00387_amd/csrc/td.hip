// Time-dependent Hamiltonians: commutator-free Magnus expansions over the
// Trotter steps of tebd_impl.
//
// Sec. "Time evolution methods" (time ordering): for H(t) = sum_k f_k(t) H_k
// the propagator over [t, t + dt] is a product of exponentials of linear
// combinations of H at the nodes t + c_j dt.  Scheme 2 (the paper's default,
// one exponential) is the midpoint rule exp(-i dt H(t + dt/2)); scheme 4 has
// two exponentials, nodes c_{1,2} = 1/2 -+ sqrt(3)/6 and weights
// a_1 = (3 - 2 sqrt 3)/12, a_2 = (3 + 2 sqrt 3)/12: first
// exp(-i dt (a_2 H_1 + a_1 H_2)), then exp(-i dt (a_1 H_1 + a_2 H_2)).
// Every exponential is one Trotter step (even/odd TEBD2/TEBD4 or the sweep)
// of the bond Hamiltonians h_b = sum_k w_k h_b^(k), combined on the device.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace {

constexpr int kMaxTerms = 16;

struct TermWeights {
  double w[kMaxTerms];
};

// dst[e] = sum_k w_k src[k * stride + e], e < count (complex128)
__global__ void combine_terms_kernel(const double2* __restrict__ src, double2* __restrict__ dst, long long count,
                                     long long stride, int n_terms, TermWeights tw) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    double2 a = make_double2(0.0, 0.0);
    for (int k = 0; k < n_terms; ++k) {
      const double2 v = src[k * stride + e];
      a.x += tw.w[k] * v.x;
      a.y += tw.w[k] * v.y;
    }
    dst[e] = a;
  }
}

// nodes and the weight matrix W[e][j] (exponentials in application order)
int scheme_table(int scheme, double* nodes, double W[2][2], int* n_exp) {
  const double s3 = std::sqrt(3.0);
  if (scheme == 2) {
    nodes[0] = 0.5;
    W[0][0] = 1.0;
    *n_exp = 1;
    return 1;
  }
  if (scheme == 4) {
    nodes[0] = 0.5 - s3 / 6.0;
    nodes[1] = 0.5 + s3 / 6.0;
    const double a1 = (3.0 - 2.0 * s3) / 12.0, a2 = (3.0 + 2.0 * s3) / 12.0;
    W[0][0] = a2;
    W[0][1] = a1;
    W[1][0] = a1;
    W[1][1] = a2;
    *n_exp = 2;
    return 2;
  }
  return 0;
}

}  // namespace

mps_status td_impl(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains, int32_t order,
                   double dt, int32_t n_steps, double eps_local, uint32_t flags, int32_t n_terms, int32_t scheme,
                   const double* f_nodes, void* hwork, const mps_u1_chain* u1);

extern "C" {

mps_status mps_cfme_nodes(int32_t scheme, double* nodes, int32_t* n_nodes) {
  if (!nodes || !n_nodes) return MPS_ERR_INVALID;
  double W[2][2];
  int n_exp = 0;
  const int nn = scheme_table(scheme, nodes, W, &n_exp);
  if (nn == 0) return MPS_ERR_INVALID;
  *n_nodes = nn;
  return MPS_OK;
}

mps_status mps_tebd_td_step(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains,
                            int32_t order, double dt, int32_t n_steps, double eps_local, uint32_t flags,
                            int32_t n_terms, int32_t scheme, const double* f_nodes, void* hwork) {
  return td_impl(h, stream, chains, n_chains, order, dt, n_steps, eps_local, flags, n_terms, scheme, f_nodes, hwork,
                 nullptr);
}

mps_status mps_tebd_td_step_u1(mps_handle h, mps_stream stream, const mps_chain_desc* chains,
                               const mps_u1_chain* charges, int32_t n_chains, int32_t order, double dt,
                               int32_t n_steps, double eps_local, uint32_t flags, int32_t n_terms, int32_t scheme,
                               const double* f_nodes, void* hwork) {
  if (!h) return MPS_ERR_INVALID;
  if (!charges) return mps_fail(h, MPS_ERR_INVALID, "null charges");
  return td_impl(h, stream, chains, n_chains, order, dt, n_steps, eps_local, flags, n_terms, scheme, f_nodes, hwork,
                 charges);
}

}  // extern "C"

mps_status td_impl(mps_handle h, mps_stream stream, const mps_chain_desc* chains, int32_t n_chains, int32_t order,
                   double dt, int32_t n_steps, double eps_local, uint32_t flags, int32_t n_terms, int32_t scheme,
                   const double* f_nodes, void* hwork, const mps_u1_chain* u1) {
  if (!h) return MPS_ERR_INVALID;
  if (!chains || n_chains < 1) return mps_fail(h, MPS_ERR_INVALID, "need at least one chain");
  if (n_terms < 1 || n_terms > kMaxTerms) return mps_fail(h, MPS_ERR_INVALID, "n_terms must be in 1..16");
  if (!f_nodes || !hwork) return mps_fail(h, MPS_ERR_INVALID, "null f_nodes or hwork");
  if (n_steps < 0) return mps_fail(h, MPS_ERR_INVALID, "n_steps < 0");
  double nodes[2], W[2][2];
  int n_exp = 0;
  const int n_nodes = scheme_table(scheme, nodes, W, &n_exp);
  if (n_nodes == 0) return mps_fail(h, MPS_ERR_INVALID, "scheme must be 2 or 4");
  for (long long i = 0; i < (long long)n_steps * n_nodes * n_terms; ++i)
    if (!std::isfinite(f_nodes[i])) return mps_fail(h, MPS_ERR_INVALID, "non-finite f_nodes entry");
  // the chains as tebd_impl sees them: bond Hamiltonians in hwork
  std::vector<mps_chain_desc> tmp(chains, chains + n_chains);
  size_t off = 0;
  for (int c = 0; c < n_chains; ++c) {
    const mps_chain_desc& ch = chains[c];
    if (ch.L < 2 || ch.d < 1 || ch.d > 5) return mps_fail(h, MPS_ERR_SHAPE, "bad chain shape");
    if (!ch.hbond) return mps_fail(h, MPS_ERR_INVALID, "null chain pointer");
    tmp[c].hbond = (const double2*)hwork + off;
    off += (size_t)(ch.L - 1) * ch.d * ch.d * ch.d * ch.d;
  }
  hipStream_t s = (hipStream_t)stream;
  for (int n = 0; n < n_steps; ++n) {
    const double* fn = f_nodes + (size_t)n * n_nodes * n_terms;
    for (int e = 0; e < n_exp; ++e) {
      TermWeights tw;
      std::memset(&tw, 0, sizeof(tw));
      for (int k = 0; k < n_terms; ++k)
        for (int j = 0; j < n_nodes; ++j) tw.w[k] += W[e][j] * fn[j * n_terms + k];
      for (int c = 0; c < n_chains; ++c) {
        const mps_chain_desc& ch = chains[c];
        const long long cnt = (long long)(ch.L - 1) * ch.d * ch.d * ch.d * ch.d;
        const int grid = (int)std::min<long long>((cnt + 255) / 256, 1024);
        combine_terms_kernel<<<grid, 256, 0, s>>>((const double2*)ch.hbond, (double2*)tmp[c].hbond, cnt, cnt,
                                                  n_terms, tw);
        MPS_TRY_HIP(h, hipGetLastError());
      }
      mps_status st = tebd_impl(h, stream, tmp.data(), n_chains, order, dt, 1, eps_local, flags, 0, 1 << 30, nullptr,
                                u1);
      if (st != MPS_OK) return st;
    }
  }
  return MPS_OK;
}
