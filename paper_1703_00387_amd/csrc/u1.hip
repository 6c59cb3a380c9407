// U(1)-symmetric truncated SVD: the two-site tensor cut at a bond is block
// diagonal in the charge the bond carries, so the decomposition runs on every
// charge block (App. "Convenient features", symmetry conservation).  The blocks
// of one matrix are gathered into separate matrices and go through the
// batched block Jacobi together; one selection ranks the squared singular
// values of all blocks (the count rule of Sec. "Basic concepts" applied to
// their union); the kept right vectors are scattered back to the full column
// space with the charge of their block, and U = theta V / s.
#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "common.h"

namespace {

struct U1Block {
  int32_t q, m, n, row_off, col_off, pad;  // charge, shape, offsets into the row and column lists
  int64_t x_off;                           // offset of the gathered block (complex128 elements)
};

// X_b[i][j] = theta[rows[i]][cols[j]], grid (chunks, blocks)
__global__ __launch_bounds__(256) void u1_gather_kernel(const double2* __restrict__ theta, int64_t ldt,
                                                        const U1Block* __restrict__ blk,
                                                        const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ cols, double2* __restrict__ Xw) {
  const U1Block b = blk[blockIdx.y];
  const int64_t tot = (int64_t)b.m * b.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / b.n), j = (int)(e % b.n);
    Xw[b.x_off + e] = theta[(size_t)rows[b.row_off + i] * ldt + cols[b.col_off + j]];
  }
}

// the block holding entry e of the concatenated row list (blocks by ascending offset)
__device__ __forceinline__ int u1_block_of(const U1Block* blk, int nblk, int e) {
  int lo = 0, hi = nblk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk[mid].row_off <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One workgroup.  Entry e of the concatenated row list (blocks by ascending
// charge, rows in order) holds a squared singular value: the converged row
// norm of its block.  They are ranked descending (ties by e, that is by
// charge, then by row), the count rule is applied to the sorted list, and the
// sorted entries, their values and the selection summary are written.
__global__ __launch_bounds__(256) void u1_select_kernel(const JacMat* __restrict__ mats,
                                                        const U1Block* __restrict__ blk, int nblk, int R,
                                                        int kmax, double eps, int32_t* pe, double* s2o,
                                                        SelOut* out) {
  extern __shared__ double dyn[];
  double* v = dyn;                // [R]
  int* perm = (int*)(v + R);      // [R]
  const int tid = threadIdx.x;
  for (int e = tid; e < R; e += 256) {
    const int b = u1_block_of(blk, nblk, e);
    const double a = mats[b].nrm2[e - blk[b].row_off];
    v[e] = (a >= 0.0 && a <= 1.0e300) ? a : -1.0;  // non-finite entries sort last (flagged by the preparation)
  }
  __syncthreads();
  for (int e = tid; e < R; e += 256) {
    const double x = v[e];
    int rank = 0;
    for (int f = 0; f < R; ++f) {
      const double w = v[f];
      rank += (w > x) || (w == x && f < e);
    }
    perm[rank] = e;
  }
  __syncthreads();
  for (int r = tid; r < R; r += 256) {
    pe[r] = perm[r];
    s2o[r] = fmax(v[perm[r]], 0.0);
  }
  __syncthreads();
  if (tid == 0) {
    double total = 0.0;
    for (int r = R - 1; r >= 0; --r) total += fmax(v[perm[r]], 0.0);
    int k = R;
    double tail = 0.0;
    if (eps >= 0.0) {
      for (int kk = R - 1; kk >= 1; --kk) {
        const double t2 = tail + fmax(v[perm[kk]], 0.0);
        if (t2 <= eps * total) {
          tail = t2;
          k = kk;
        } else {
          break;
        }
      }
    }
    if (k > kmax) k = kmax;
    if (k < 1) k = 1;
    double disc = 0.0, kept = 0.0;
    for (int r = R - 1; r >= k; --r) disc += fmax(v[perm[r]], 0.0);
    for (int r = k - 1; r >= 0; --r) kept += fmax(v[perm[r]], 0.0);
    SelOut o;
    o.k = k;
    o.m = R;
    o.disc = disc;
    o.norm2 = total;
    o.nk = kept > 0.0 ? sqrt(kept) : 1.0;
    *out = o;
  }
}

// One workgroup per kept vector j: row j of Vh is the block's row divided by
// s_j, on the block's columns, and zero elsewhere; S, the charges and the
// summary are written alongside.
__global__ __launch_bounds__(256) void u1_vh_kernel(const JacMat* __restrict__ mats,
                                                    const U1Block* __restrict__ blk, int nblk,
                                                    const int32_t* __restrict__ cols,
                                                    const int32_t* __restrict__ pe, const double* __restrict__ s2o,
                                                    const SelOut* __restrict__ sel, int64_t n, double2* Vh,
                                                    double* S, int32_t* q_out, int32_t* k_dev, double* disc_dev,
                                                    double* norm2_dev) {
  const SelOut so = *sel;
  const int j = blockIdx.x;
  if (j == 0 && threadIdx.x == 0) {
    *k_dev = so.k;
    *disc_dev = so.disc;
    *norm2_dev = so.norm2;
  }
  if (j >= so.k) return;
  const int e = pe[j];
  const int b = u1_block_of(blk, nblk, e);
  const U1Block B = blk[b];
  const JacMat M = mats[b];
  const int i = e - B.row_off;
  const double s = sqrt(s2o[j]);
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  double2* vrow = Vh + (size_t)j * n;
  for (int64_t c = threadIdx.x; c < n; c += 256) vrow[c] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int c = threadIdx.x; c < B.n; c += 256) {
    const double2 x = M.X[(size_t)i * M.ld + c];
    vrow[cols[B.col_off + c]] = make_double2(x.x * inv, x.y * inv);
  }
  if (threadIdx.x == 0) {
    S[j] = s;
    q_out[j] = B.q;
  }
}

// U[i][j] = (theta Vh^dag)[i][j] / s_j for j < k on the rows of the vector's
// charge, zero on the others (the left vectors follow from the right ones:
// theta v_j = s_j u_j; Vh_j vanishes off its block's columns, and rows of
// another charge are outside the block, so entries of theta off the blocks
// never enter)
__global__ __launch_bounds__(256) void u1_u_kernel(const double2* __restrict__ theta, const double2* __restrict__ Vh,
                                                   const double* __restrict__ S, const SelOut* __restrict__ sel,
                                                   const int32_t* __restrict__ rowq, const int32_t* __restrict__ q_out,
                                                   int64_t m, int64_t n, int64_t chi_max, double2* U) {
  const int k = sel->k;
  const size_t total = (size_t)m * k;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx / k), j = (int)(idx % k);
    double2 acc = make_double2(0.0, 0.0);
    if (rowq[i] != q_out[j]) {
      U[(size_t)i * chi_max + j] = acc;
      continue;
    }
    for (int64_t c = 0; c < n; ++c) {
      const double2 a = theta[(size_t)i * n + c], v = Vh[(size_t)j * n + c];
      acc.x += a.x * v.x + a.y * v.y;
      acc.y += a.y * v.x - a.x * v.y;
    }
    const double sj = S[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    U[(size_t)i * chi_max + j] = make_double2(acc.x * inv, acc.y * inv);
  }
}

}  // namespace

extern "C" mps_status mps_truncate_u1(mps_handle h, mps_stream stream, const void* theta, int64_t m, int64_t n,
                                      const int32_t* row_q, const int32_t* col_q, int64_t chi_max, double eps,
                                      void* U, double* S, void* Vh, int32_t* q_out, int32_t* k_dev,
                                      double* disc_dev, double* norm2_dev) {
  if (!h) return MPS_ERR_INVALID;
  if (!theta || !row_q || !col_q || !U || !S || !Vh || !q_out || !k_dev || !disc_dev || !norm2_dev)
    return mps_fail(h, MPS_ERR_INVALID, "null pointer");
  if (m < 1 || n < 1 || chi_max < 1) return mps_fail(h, MPS_ERR_SHAPE, "m, n, chi_max must be >= 1");
  if (m > 4096 || n > 4096) return mps_fail(h, MPS_ERR_CAPACITY, "m and n are limited to 4096");
  if (!(eps == eps)) return mps_fail(h, MPS_ERR_INVALID, "eps is NaN");
  // the charge blocks, ascending charge, rows and columns in order
  std::map<int32_t, std::pair<std::vector<int32_t>, std::vector<int32_t>>> sec;
  for (int64_t r = 0; r < m; ++r) sec[row_q[r]].first.push_back((int32_t)r);
  for (int64_t c = 0; c < n; ++c) sec[col_q[c]].second.push_back((int32_t)c);
  std::vector<U1Block> blocks;
  std::vector<int32_t> rows, cols;
  int64_t xw = 0;
  int max_m = 1;
  for (auto& kv : sec) {
    const auto& rr = kv.second.first;
    const auto& cc = kv.second.second;
    if (rr.empty() || cc.empty()) continue;
    U1Block b;
    b.q = kv.first;
    b.m = (int32_t)rr.size();
    b.n = (int32_t)cc.size();
    b.row_off = (int32_t)rows.size();
    b.col_off = (int32_t)cols.size();
    b.pad = 0;
    b.x_off = xw;
    xw += (int64_t)b.m * b.n;
    max_m = std::max(max_m, b.m);
    rows.insert(rows.end(), rr.begin(), rr.end());
    cols.insert(cols.end(), cc.begin(), cc.end());
    blocks.push_back(b);
  }
  const int nblk = (int)blocks.size();
  if (nblk == 0) return mps_fail(h, MPS_ERR_SHAPE, "no charge is shared by rows and columns");
  const int R = (int)rows.size();
  hipStream_t s = (hipStream_t)stream;
  WsPlan p;
  const size_t oX = p.take<double2>((size_t)xw);
  const size_t oM = p.take<JacMat>(nblk);
  const size_t oB = p.take<U1Block>(nblk);
  const size_t oRows = p.take<int32_t>(R);
  const size_t oCols = p.take<int32_t>(cols.size());
  const size_t oRm = p.take<int32_t>(R);
  const size_t oNr = p.take<double>(R);
  const size_t oPe = p.take<int32_t>(R);
  const size_t oS2 = p.take<double>(R);
  const size_t oSel = p.take<SelOut>(1);
  const size_t oU = p.take<int32_t>(4);
  const size_t oRq = p.take<int32_t>(m);
  mps_status st = mps_ensure_ws(h, p.off);
  if (st != MPS_OK) return st;
  char* ws = h->ws;
  std::vector<JacMat> hm(nblk);
  for (int i = 0; i < nblk; ++i) {
    std::memset(&hm[i], 0, sizeof(JacMat));
    hm[i].X = (double2*)(ws + oX) + blocks[i].x_off;
    hm[i].rowmap = (int32_t*)(ws + oRm) + blocks[i].row_off;
    hm[i].nrm2 = (double*)(ws + oNr) + blocks[i].row_off;
    hm[i].m = blocks[i].m;
    hm[i].n = blocks[i].n;
    hm[i].ld = blocks[i].n;
    hm[i].nb = jac_nb(blocks[i].m);
    hm[i].kmax = blocks[i].m;
  }
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oM, hm.data(), nblk * sizeof(JacMat), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oB, blocks.data(), nblk * sizeof(U1Block), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oRows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oCols, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oRq, row_q, (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));  // the host vectors go out of scope at return
  const JacMat* mats = (const JacMat*)(ws + oM);
  const U1Block* blk = (const U1Block*)(ws + oB);
  {
    int64_t max_mn = 1;
    for (const auto& b : blocks) max_mn = std::max<int64_t>(max_mn, (int64_t)b.m * b.n);
    const int gx = (int)std::min<int64_t>((max_mn + 255) / 256, 1024);
    u1_gather_kernel<<<dim3(gx, nblk), 256, 0, s>>>((const double2*)theta, n, blk, (const int32_t*)(ws + oRows),
                                                   (const int32_t*)(ws + oCols), (double2*)(ws + oX));
    MPS_TRY_HIP(h, hipGetLastError());
  }
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, (JacMat*)(ws + oM), nblk, h->status_dev));
  st = run_jacobi(h, s, (JacMat*)(ws + oM), nblk, jac_nb(max_m), max_m, (int32_t*)(ws + oU), false);
  if (st != MPS_OK) return st;
  const int kmax = (int)std::min<int64_t>(chi_max, R);
  SelOut* sel = (SelOut*)(ws + oSel);
  u1_select_kernel<<<1, 256, (size_t)R * (sizeof(double) + sizeof(int)), s>>>(
      mats, blk, nblk, R, kmax, count_rule_eps(h, eps), (int32_t*)(ws + oPe), (double*)(ws + oS2), sel);
  MPS_TRY_HIP(h, hipGetLastError());
  u1_vh_kernel<<<kmax, 256, 0, s>>>(mats, blk, nblk, (const int32_t*)(ws + oCols), (const int32_t*)(ws + oPe),
                                    (const double*)(ws + oS2), sel, n, (double2*)Vh, S, q_out, k_dev, disc_dev,
                                    norm2_dev);
  MPS_TRY_HIP(h, hipGetLastError());
  {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((m * kmax + 255) / 256, 4096));
    u1_u_kernel<<<g, 256, 0, s>>>((const double2*)theta, (const double2*)Vh, S, sel, (const int32_t*)(ws + oRq),
                                  q_out, m, n, chi_max, (double2*)U);
    MPS_TRY_HIP(h, hipGetLastError());
  }
  return MPS_OK;
}
