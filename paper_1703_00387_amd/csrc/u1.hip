// U(1)-symmetric truncated SVD: the two-site tensor cut at a bond is block
// diagonal in the charge the bond carries, so the decomposition runs on every
// charge block (App. "Convenient features", symmetry conservation).  The blocks
// of one matrix are gathered into separate matrices and go through the
// batched block Jacobi together; one selection ranks the squared singular
// values of all blocks (the count rule of Sec. "Basic concepts" applied to
// their union); the kept right vectors are scattered back to the full column
// space with the charge of their block, and U = theta V / s.
#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <vector>

#include "common.h"

namespace {

// One charge block of one matrix.  Row and column lists of all matrices of a
// call are concatenated; row_off and col_off index them, the rows of matrix i
// occupy [row0_i, row0_i + R_i) of the row list.
struct U1Block {
  const double2* src;                       // the matrix the block is cut from, row-major with leading dim ld
  int64_t ld;
  int64_t x_off;                            // offset of the gathered block (complex128 elements)
  int32_t q, m, n, row_off, col_off, item;  // charge, shape, list offsets, owning matrix
};

// The blocks and rows of one matrix.
struct U1Range {
  int32_t blk0, nblk;  // its blocks: [blk0, blk0 + nblk), ascending charge
  int32_t row0, R;     // its entries of the row list
  int32_t kmax, ncols; // cap on the kept count, columns of the matrix
};

// Per bond item of a charge-carrying chain.
struct U1Item {
  int32_t* qb;         // the chain's bond charges [L+1][chi_max]
  int32_t b, chi_max, d, pad;
};

// X_b[i][j] = src[rows[i]][cols[j]], grid (chunks, blocks)
__global__ __launch_bounds__(256) void u1_gather_kernel(const U1Block* __restrict__ blk,
                                                        const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ cols, double2* __restrict__ Xw) {
  const U1Block b = blk[blockIdx.y];
  const int64_t tot = (int64_t)b.m * b.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / b.n), j = (int)(e % b.n);
    Xw[b.x_off + e] = b.src[(size_t)rows[b.row_off + i] * b.ld + cols[b.col_off + j]];
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

// One workgroup per matrix.  Entry e of the matrix's row list (blocks by
// ascending charge, rows in order) holds a squared singular value: the
// converged row norm of its block.  They are ranked descending (ties by e,
// that is by charge, then by row), the count rule is applied to the sorted
// list, and the sorted entries (as positions in the whole row list), their
// values and the selection summary are written.
__global__ __launch_bounds__(256) void u1_select_kernel(const JacMat* __restrict__ mats,
                                                        const U1Block* __restrict__ blk,
                                                        const U1Range* __restrict__ ranges, double eps,
                                                        int32_t* pe, double* s2o, SelOut* out) {
  extern __shared__ double dyn[];
  const U1Range rg = ranges[blockIdx.x];
  const int R = rg.R, kmax = rg.kmax;
  double* v = dyn;                // [R]
  int* perm = (int*)(v + R);      // [R]
  const int tid = threadIdx.x;
  const U1Block* bl = blk + rg.blk0;
  for (int e = tid; e < R; e += 256) {
    const int b = u1_block_of(bl, rg.nblk, rg.row0 + e);
    const double a = mats[rg.blk0 + b].nrm2[rg.row0 + e - bl[b].row_off];
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
    pe[rg.row0 + r] = rg.row0 + perm[r];
    s2o[rg.row0 + r] = fmax(v[perm[r]], 0.0);
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
    out[blockIdx.x] = o;
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
                                                   const U1Block* __restrict__ blk, int nblk,
                                                   const int32_t* __restrict__ cols, int64_t m, int64_t n,
                                                   int64_t chi_max, double2* U) {
  const int k = sel->k;
  const size_t total = (size_t)m * k;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx / k), j = (int)(idx % k);
    double2 acc = make_double2(0.0, 0.0);
    const int32_t q = q_out[j];
    int b = -1;
    if (rowq[i] == q)
      for (int t = 0; t < nblk; ++t)
        if (blk[t].q == q) {
          b = t;
          break;
        }
    if (b < 0) {
      U[(size_t)i * chi_max + j] = acc;
      continue;
    }
    // only the block's columns: Vh_j vanishes on the others
    const int32_t* cb = cols + blk[b].col_off;
    for (int t = 0; t < blk[b].n; ++t) {
      const int64_t c = cb[t];
      const double2 a = theta[(size_t)i * n + c], v = Vh[(size_t)j * n + c];
      acc.x += a.x * v.x + a.y * v.y;
      acc.y += a.y * v.x - a.x * v.y;
    }
    const double sj = S[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    U[(size_t)i * chi_max + j] = make_double2(acc.x * inv, acc.y * inv);
  }
}


// ---------------------------------------------------------------------------
// charge-carrying chains: one layer of bond items
// ---------------------------------------------------------------------------

// Row i of out: chi_b, chi_{b+2}, the charges of bond b (chi_max entries),
// those of bond b+2 (chi_max entries).
__global__ __launch_bounds__(256) void u1_read_kernel(const BondItem* __restrict__ items,
                                                      const U1Item* __restrict__ ui, int stride,
                                                      int32_t* __restrict__ out) {
  const BondItem it = items[blockIdx.x];
  const int cm = it.chi_max;
  const int chl = it.chi[it.b], chr = it.chi[it.b + 2];
  int32_t* o = out + (size_t)blockIdx.x * stride;
  if (threadIdx.x == 0) {
    o[0] = chl;
    o[1] = chr;
  }
  const int32_t* qb = ui[blockIdx.x].qb;
  for (int a = threadIdx.x; a < min(max(chl, 0), cm); a += 256) o[2 + a] = qb[(size_t)it.b * cm + a];
  for (int g = threadIdx.x; g < min(max(chr, 0), cm); g += 256) o[2 + cm + g] = qb[(size_t)(it.b + 2) * cm + g];
}

// grid (kept-count cap, items): kept vector j of item i.  Its block row over
// s_j is the new right site's row j (V^dag_k, zero off the block's columns),
// stored in the chain's tensor and in the item's V^dag workspace; lam_{b+1},
// the bond charge, chi_{b+1} and the discarded weight are written alongside.
template <class T>
__global__ __launch_bounds__(256) void u1_wb_kernel(const BondItem* __restrict__ items,
                                                    const U1Item* __restrict__ ui, const JacMat* __restrict__ mats,
                                                    const U1Block* __restrict__ blk,
                                                    const U1Range* __restrict__ ranges,
                                                    const int32_t* __restrict__ cols, const int32_t* __restrict__ pe,
                                                    const double* __restrict__ s2o, const SelOut* __restrict__ sel) {
  const int i = blockIdx.y, j = blockIdx.x;
  const BondItem it = items[i];
  const U1Range rg = ranges[i];
  const SelOut so = sel[i];
  const int d = it.d, cm = it.chi_max, ncols = rg.ncols, chr = ncols / d;
  if (j == 0 && threadIdx.x == 0) {
    it.chi[it.b + 1] = so.k;
    it.disc[it.b] += so.disc;
  }
  if (j >= so.k) return;
  const int e = pe[rg.row0 + j];
  const U1Block* bl = blk + rg.blk0;
  const int b = u1_block_of(bl, rg.nblk, e);
  const U1Block B = bl[b];
  const JacMat M = mats[rg.blk0 + b];
  const int r = e - B.row_off;
  const double sv = sqrt(s2o[rg.row0 + j]);
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  T* vrow = (T*)it.Vh + (size_t)j * ncols;
  T* Br = (T*)it.Br;
  T z;
  z.x = 0;
  z.y = 0;
  for (int c = threadIdx.x; c < ncols; c += 256) {
    vrow[c] = z;
    Br[((size_t)j * d + c / chr) * cm + c % chr] = z;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < B.n; c += 256) {
    const double2 x = M.X[(size_t)r * M.ld + c];
    T v;
    v.x = x.x * inv;
    v.y = x.y * inv;
    const int col = cols[B.col_off + c];
    vrow[col] = v;
    Br[((size_t)j * d + col / chr) * cm + col % chr] = v;
  }
  if (threadIdx.x == 0) {
    it.lam_m[j] = sv / so.nk;
    ui[i].qb[(size_t)(it.b + 1) * cm + j] = B.q;
  }
}

// One matrix, grid (kept-count cap): kept vector j of the matrix's blocks,
// divided by s_j, zero off its block's columns, written as row j of dst
// ([k][len]) or as column j ([len][k], col_major); its charge to q_out[j].
template <class T>
__global__ __launch_bounds__(256) void u1_rows_kernel(const JacMat* __restrict__ mats,
                                                      const U1Block* __restrict__ blk, int nblk,
                                                      const int32_t* __restrict__ cols,
                                                      const int32_t* __restrict__ pe, const double* __restrict__ s2o,
                                                      const SelOut* __restrict__ sel, T* dst, int len, int col_major,
                                                      int32_t* q_out) {
  const int k = sel->k, j = blockIdx.x;
  if (j >= k) return;
  const int e = pe[j];
  const int b = u1_block_of(blk, nblk, e);
  const U1Block B = blk[b];
  const JacMat M = mats[b];
  const int r = e - B.row_off;
  const double sv = sqrt(s2o[j]);
  const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
  T z;
  z.x = 0;
  z.y = 0;
  for (int c = threadIdx.x; c < len; c += 256) dst[col_major ? (size_t)c * k + j : (size_t)j * len + c] = z;
  __syncthreads();
  for (int c = threadIdx.x; c < B.n; c += 256) {
    const double2 x = M.X[(size_t)r * M.ld + c];
    T v;
    v.x = x.x * inv;
    v.y = x.y * inv;
    const int col = cols[B.col_off + c];
    dst[col_major ? (size_t)col * k + j : (size_t)j * len + col] = v;
  }
  if (threadIdx.x == 0) q_out[j] = B.q;
}

// Workspace of u1_layer for up to n_cap items of at most m_cap rows and columns.
struct U1Plan {
  size_t oItems, oRb, oX, oMats, oBlk, oRg, oRows, oCols, oRm, oNrm, oPe, oS2, off;
  U1Plan(int n_cap, int m_cap, int chi_cap) {
    WsPlan p;
    const size_t nm = (size_t)n_cap * m_cap;
    oItems = p.take<U1Item>(n_cap);
    oRb = p.take<int32_t>((size_t)n_cap * (2 + 2 * chi_cap) + 16);
    oX = p.take<double2>(nm * m_cap);
    oMats = p.take<JacMat>(nm);
    oBlk = p.take<U1Block>(nm);
    oRg = p.take<U1Range>(n_cap);
    oRows = p.take<int32_t>(nm);
    oCols = p.take<int32_t>(nm);
    oRm = p.take<int32_t>(nm);
    oNrm = p.take<double>(nm);
    oPe = p.take<int32_t>(nm);
    oS2 = p.take<double>(nm);
    off = p.off + 256;
  }
};

}  // namespace

size_t u1_layer_bytes(int n_cap, int m_cap, int chi_cap) { return U1Plan(n_cap, m_cap, chi_cap).off; }

mps_status u1_layer(mps_handle h, hipStream_t s, const BondItem* it_host, const BondItem* it_dev, const int* chain_of,
                    int n, const mps_u1_chain* u1c, int n_cap, int m_cap, int chi_cap, double eps, bool c128,
                    char* region, SelOut* sel, int32_t* unconv, bool fixed) {
  if (n <= 0) return MPS_OK;
  const U1Plan P(n_cap, m_cap, chi_cap);
  region = (char*)(((uintptr_t)region + 255) & ~(uintptr_t)255);
  const int stride = 2 + 2 * chi_cap;
  std::vector<U1Item> ui(n);
  for (int i = 0; i < n; ++i) ui[i].qb = u1c[chain_of[i]].qbond;
  MPS_TRY_HIP(h, hipMemcpyAsync(region + P.oItems, ui.data(), n * sizeof(U1Item), hipMemcpyHostToDevice, s));
  U1Item* dUi = (U1Item*)(region + P.oItems);
  u1_read_kernel<<<n, 256, 0, s>>>(it_dev, dUi, stride, (int32_t*)(region + P.oRb));
  MPS_TRY_HIP(h, hipGetLastError());
  std::vector<int32_t> rb((size_t)n * stride);
  MPS_TRY_HIP(h, hipMemcpyAsync(rb.data(), region + P.oRb, rb.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));
  // the charge blocks of every item, ascending charge, rows and columns in order
  std::vector<U1Block> blocks;
  std::vector<U1Range> ranges(n);
  std::vector<int32_t> rows, cols;
  std::vector<int32_t> rq, cq, keys;     // per item: row and column charges, distinct row charges
  std::vector<int> nr, nc, pr, pc;       // per charge slot: counts, then fill positions
  int64_t xw = 0, max_mn = 1;
  int max_m = 1, max_R = 1, k_cap = 1;
  for (int i = 0; i < n; ++i) {
    const BondItem& it = it_host[i];
    const int d = it.d, cm = it.chi_max;
    const int32_t* o = rb.data() + (size_t)i * stride;
    const int chl = o[0], chr = o[1];
    if (chl < 1 || chl > cm || chr < 1 || chr > cm)
      return mps_fail(h, MPS_ERR_SHAPE, "bond dimension out of range in a charge-carrying chain");
    const int32_t* qs = u1c[chain_of[i]].qsite;
    const int32_t md = u1c[chain_of[i]].modulus;  // 0: U(1); n >= 2: Z_n
    auto red = [md](int64_t v) -> int32_t { return md == 0 ? (int32_t)v : (int32_t)(((v % md) + md) % md); };
    const int M = chl * d, N = d * chr;
    rq.resize(M);
    cq.resize(N);
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int a = 0; a < chl; ++a)
      for (int s1 = 0; s1 < d; ++s1) {
        const int32_t v = red((int64_t)o[2 + a] + qs[s1]);
        rq[a * d + s1] = v;
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
    for (int s2 = 0; s2 < d; ++s2)
      for (int g = 0; g < chr; ++g) cq[s2 * chr + g] = red((int64_t)o[2 + cm + g] - qs[s2]);
    // charge slots in ascending order: offsets from the smallest row charge
    // when the rows' charges are dense, else positions among their sorted
    // distinct values; a column whose charge no row has gets no slot
    const bool direct = (int64_t)hi - lo < 4LL * (M + N);
    keys.clear();
    if (!direct) {
      keys.assign(rq.begin(), rq.end());
      std::sort(keys.begin(), keys.end());
      keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    }
    auto slot = [&](int32_t v) -> int {
      if (direct) return (v < lo || v > hi) ? -1 : (int)(v - lo);
      auto f = std::lower_bound(keys.begin(), keys.end(), v);
      return (f != keys.end() && *f == v) ? (int)(f - keys.begin()) : -1;
    };
    const int K = direct ? (int)(hi - lo + 1) : (int)keys.size();
    nr.assign(K, 0);
    nc.assign(K, 0);
    for (int r = 0; r < M; ++r) nr[slot(rq[r])]++;
    for (int c = 0; c < N; ++c) {
      const int k = slot(cq[c]);
      if (k >= 0) nc[k]++;
    }
    U1Range& rg = ranges[i];
    rg.blk0 = (int32_t)blocks.size();
    rg.row0 = (int32_t)rows.size();
    rg.ncols = N;
    pr.assign(K, -1);
    pc.assign(K, -1);
    size_t rtot = rows.size(), ctot = cols.size();
    for (int k = 0; k < K; ++k) {
      if (nr[k] == 0 || nc[k] == 0) continue;
      U1Block b;
      b.src = it.X;
      b.ld = N;
      b.q = direct ? lo + k : keys[k];
      b.m = nr[k];
      b.n = nc[k];
      b.row_off = (int32_t)rtot;
      b.col_off = (int32_t)ctot;
      b.item = i;
      b.x_off = xw;
      pr[k] = (int)rtot;
      pc[k] = (int)ctot;
      rtot += b.m;
      ctot += b.n;
      xw += (int64_t)b.m * b.n;
      max_m = std::max(max_m, b.m);
      max_mn = std::max<int64_t>(max_mn, (int64_t)b.m * b.n);
      blocks.push_back(b);
    }
    rows.resize(rtot);
    cols.resize(ctot);
    for (int r = 0; r < M; ++r) {
      const int k = slot(rq[r]);
      if (pr[k] >= 0) rows[pr[k]++] = r;
    }
    for (int c = 0; c < N; ++c) {
      const int k = slot(cq[c]);
      if (k >= 0 && pc[k] >= 0) cols[pc[k]++] = c;
    }
    rg.nblk = (int32_t)blocks.size() - rg.blk0;
    rg.R = (int32_t)rows.size() - rg.row0;
    if (rg.nblk == 0)
      return mps_fail(h, MPS_ERR_SHAPE, "no charge is shared across a bond of a charge-carrying chain");
    rg.kmax = std::min(cm, rg.R);
    max_R = std::max(max_R, rg.R);
    k_cap = std::max(k_cap, rg.kmax);
  }
  const int nblk = (int)blocks.size();
  if (nblk > 65535) return mps_fail(h, MPS_ERR_CAPACITY, "more than 65535 charge blocks in one layer");
  if ((int64_t)xw > (int64_t)n_cap * m_cap * m_cap || (int64_t)nblk > (int64_t)n_cap * m_cap ||
      (int64_t)rows.size() > (int64_t)n_cap * m_cap || (int64_t)cols.size() > (int64_t)n_cap * m_cap)
    return mps_fail(h, MPS_ERR_CAPACITY, "charge blocks exceed the layer workspace");
  char* const ws = region;
  std::vector<JacMat> hm(nblk);
  for (int i = 0; i < nblk; ++i) {
    std::memset(&hm[i], 0, sizeof(JacMat));
    hm[i].X = (double2*)(ws + P.oX) + blocks[i].x_off;
    hm[i].rowmap = (int32_t*)(ws + P.oRm) + blocks[i].row_off;
    hm[i].nrm2 = (double*)(ws + P.oNrm) + blocks[i].row_off;
    hm[i].m = blocks[i].m;
    hm[i].n = blocks[i].n;
    hm[i].ld = blocks[i].n;
    hm[i].nb = jac_nb(blocks[i].m);
    hm[i].kmax = blocks[i].m;
  }
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oMats, hm.data(), nblk * sizeof(JacMat), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oBlk, blocks.data(), nblk * sizeof(U1Block), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oRg, ranges.data(), n * sizeof(U1Range), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oRows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oCols, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  JacMat* mats = (JacMat*)(ws + P.oMats);
  const U1Block* blk = (const U1Block*)(ws + P.oBlk);
  const U1Range* rgd = (const U1Range*)(ws + P.oRg);
  const int gx = (int)std::min<int64_t>((max_mn + 255) / 256, 1024);
  u1_gather_kernel<<<dim3(gx, nblk), 256, 0, s>>>(blk, (const int32_t*)(ws + P.oRows), (const int32_t*)(ws + P.oCols),
                                                 (double2*)(ws + P.oX));
  MPS_TRY_HIP(h, hipGetLastError());
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, mats, nblk, h->status_dev));
  mps_status st = run_jacobi(h, s, mats, nblk, jac_nb(max_m), max_m, unconv, fixed);
  if (st != MPS_OK) return st;
  int32_t* pe = (int32_t*)(ws + P.oPe);
  double* s2o = (double*)(ws + P.oS2);
  u1_select_kernel<<<n, 256, (size_t)max_R * (sizeof(double) + sizeof(int)), s>>>(mats, blk, rgd,
                                                                                   count_rule_eps(h, eps), pe, s2o, sel);
  MPS_TRY_HIP(h, hipGetLastError());
  const int32_t* dcols = (const int32_t*)(ws + P.oCols);
  if (c128)
    u1_wb_kernel<double2><<<dim3(k_cap, n), 256, 0, s>>>(it_dev, dUi, mats, blk, rgd, dcols, pe, s2o, sel);
  else
    u1_wb_kernel<float2><<<dim3(k_cap, n), 256, 0, s>>>(it_dev, dUi, mats, blk, rgd, dcols, pe, s2o, sel);
  MPS_TRY_HIP(h, hipGetLastError());
  MPS_TRY_HIP(h, hipStreamSynchronize(s));  // the host vectors go out of scope at return
  return MPS_OK;
}

mps_status u1_split_one(mps_handle h, hipStream_t s, const double2* X, int m, int n, const int32_t* row_q,
                        const int32_t* col_q, int kmax, double eps, char* region, int m_cap, int chi_cap,
                        SelOut* sel, void* dst, int col_major, bool c128, int* k_out, double* disc_out,
                        int32_t* q_out) {
  if (m < 1 || n < 1 || m > m_cap || n > m_cap) return mps_fail(h, MPS_ERR_CAPACITY, "split larger than its workspace");
  const U1Plan P(1, m_cap, chi_cap);
  region = (char*)(((uintptr_t)region + 255) & ~(uintptr_t)255);
  char* const ws = region;
  std::map<int32_t, std::pair<std::vector<int32_t>, std::vector<int32_t>>> sec;
  for (int r = 0; r < m; ++r) sec[row_q[r]].first.push_back(r);
  for (int c = 0; c < n; ++c) sec[col_q[c]].second.push_back(c);
  std::vector<U1Block> blocks;
  std::vector<int32_t> rows, cols;
  int64_t xw = 0, max_mn = 1;
  int max_m = 1;
  for (auto& kv : sec) {
    const auto& rr = kv.second.first;
    const auto& cc = kv.second.second;
    if (rr.empty() || cc.empty()) continue;
    U1Block b;
    b.src = X;
    b.ld = n;
    b.q = kv.first;
    b.m = (int32_t)rr.size();
    b.n = (int32_t)cc.size();
    b.row_off = (int32_t)rows.size();
    b.col_off = (int32_t)cols.size();
    b.item = 0;
    b.x_off = xw;
    xw += (int64_t)b.m * b.n;
    max_m = std::max(max_m, b.m);
    max_mn = std::max<int64_t>(max_mn, (int64_t)b.m * b.n);
    rows.insert(rows.end(), rr.begin(), rr.end());
    cols.insert(cols.end(), cc.begin(), cc.end());
    blocks.push_back(b);
  }
  const int nblk = (int)blocks.size();
  if (nblk == 0) return mps_fail(h, MPS_ERR_SHAPE, "no charge is shared across a bond of a charge-carrying chain");
  const int R = (int)rows.size();
  const U1Range rg{0, nblk, 0, R, std::min(kmax, R), n};
  std::vector<JacMat> hm(nblk);
  for (int i = 0; i < nblk; ++i) {
    std::memset(&hm[i], 0, sizeof(JacMat));
    hm[i].X = (double2*)(ws + P.oX) + blocks[i].x_off;
    hm[i].rowmap = (int32_t*)(ws + P.oRm) + blocks[i].row_off;
    hm[i].nrm2 = (double*)(ws + P.oNrm) + blocks[i].row_off;
    hm[i].m = blocks[i].m;
    hm[i].n = blocks[i].n;
    hm[i].ld = blocks[i].n;
    hm[i].nb = jac_nb(blocks[i].m);
    hm[i].kmax = blocks[i].m;
  }
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oMats, hm.data(), nblk * sizeof(JacMat), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oBlk, blocks.data(), nblk * sizeof(U1Block), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oRg, &rg, sizeof(U1Range), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oRows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + P.oCols, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  JacMat* mats = (JacMat*)(ws + P.oMats);
  const U1Block* blk = (const U1Block*)(ws + P.oBlk);
  const int gx = (int)std::min<int64_t>((max_mn + 255) / 256, 1024);
  u1_gather_kernel<<<dim3(gx, nblk), 256, 0, s>>>(blk, (const int32_t*)(ws + P.oRows), (const int32_t*)(ws + P.oCols),
                                                 (double2*)(ws + P.oX));
  MPS_TRY_HIP(h, hipGetLastError());
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, mats, nblk, h->status_dev));
  mps_status st = run_jacobi(h, s, mats, nblk, jac_nb(max_m), max_m, (int32_t*)(ws + P.oRb), false);
  if (st != MPS_OK) return st;
  int32_t* pe = (int32_t*)(ws + P.oPe);
  double* s2o = (double*)(ws + P.oS2);
  u1_select_kernel<<<1, 256, (size_t)R * (sizeof(double) + sizeof(int)), s>>>(
      mats, blk, (const U1Range*)(ws + P.oRg), count_rule_eps(h, eps), pe, s2o, sel);
  MPS_TRY_HIP(h, hipGetLastError());
  int32_t* qd = (int32_t*)(ws + P.oRb) + 8;   // after the Jacobi's counters
  const int32_t* dcols = (const int32_t*)(ws + P.oCols);
  if (c128)
    u1_rows_kernel<double2><<<rg.kmax, 256, 0, s>>>(mats, blk, nblk, dcols, pe, s2o, sel, (double2*)dst, n,
                                                    col_major, qd);
  else
    u1_rows_kernel<float2><<<rg.kmax, 256, 0, s>>>(mats, blk, nblk, dcols, pe, s2o, sel, (float2*)dst, n,
                                                   col_major, qd);
  MPS_TRY_HIP(h, hipGetLastError());
  SelOut so;
  MPS_TRY_HIP(h, hipMemcpyAsync(&so, sel, sizeof(so), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipMemcpyAsync(q_out, qd, rg.kmax * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));  // the host vectors go out of scope at return
  *k_out = so.k;
  *disc_out = so.disc;
  return MPS_OK;
}

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
    b.src = (const double2*)theta;
    b.ld = n;
    b.q = kv.first;
    b.m = (int32_t)rr.size();
    b.n = (int32_t)cc.size();
    b.row_off = (int32_t)rows.size();
    b.col_off = (int32_t)cols.size();
    b.item = 0;
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
  const size_t oRg = p.take<U1Range>(1);
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
  const int kmax = (int)std::min<int64_t>(chi_max, R);
  const U1Range rg{0, nblk, 0, R, kmax, (int32_t)n};
  MPS_TRY_HIP(h, hipMemcpyAsync(ws + oRg, &rg, sizeof(U1Range), hipMemcpyHostToDevice, s));
  MPS_TRY_HIP(h, hipStreamSynchronize(s));  // the host vectors go out of scope at return
  const JacMat* mats = (const JacMat*)(ws + oM);
  const U1Block* blk = (const U1Block*)(ws + oB);
  {
    int64_t max_mn = 1;
    for (const auto& b : blocks) max_mn = std::max<int64_t>(max_mn, (int64_t)b.m * b.n);
    const int gx = (int)std::min<int64_t>((max_mn + 255) / 256, 1024);
    u1_gather_kernel<<<dim3(gx, nblk), 256, 0, s>>>(blk, (const int32_t*)(ws + oRows), (const int32_t*)(ws + oCols),
                                                   (double2*)(ws + oX));
    MPS_TRY_HIP(h, hipGetLastError());
  }
  MPS_TRY_HIP(h, launch_jac_prep_plain(s, (JacMat*)(ws + oM), nblk, h->status_dev));
  st = run_jacobi(h, s, (JacMat*)(ws + oM), nblk, jac_nb(max_m), max_m, (int32_t*)(ws + oU), false);
  if (st != MPS_OK) return st;
  SelOut* sel = (SelOut*)(ws + oSel);
  u1_select_kernel<<<1, 256, (size_t)R * (sizeof(double) + sizeof(int)), s>>>(
      mats, blk, (const U1Range*)(ws + oRg), count_rule_eps(h, eps), (int32_t*)(ws + oPe), (double*)(ws + oS2), sel);
  MPS_TRY_HIP(h, hipGetLastError());
  u1_vh_kernel<<<kmax, 256, 0, s>>>(mats, blk, nblk, (const int32_t*)(ws + oCols), (const int32_t*)(ws + oPe),
                                    (const double*)(ws + oS2), sel, n, (double2*)Vh, S, q_out, k_dev, disc_dev,
                                    norm2_dev);
  MPS_TRY_HIP(h, hipGetLastError());
  {
    const int g = (int)std::max<int64_t>(1, std::min<int64_t>((m * kmax + 255) / 256, 4096));
    u1_u_kernel<<<g, 256, 0, s>>>((const double2*)theta, (const double2*)Vh, S, sel, (const int32_t*)(ws + oRq),
                                  q_out, blk, nblk, (const int32_t*)(ws + oCols), m, n, chi_max, (double2*)U);
    MPS_TRY_HIP(h, hipGetLastError());
  }
  return MPS_OK;
}
