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
  if (tid == 0 && R == 0) {
    // no block (a bond without a shared charge): nothing is kept, the update
    // is skipped
    SelOut o;
    o.k = 0;
    o.m = 0;
    o.disc = 0.0;
    o.norm2 = 0.0;
    o.nk = 1.0;
    out[blockIdx.x] = o;
  } else if (tid == 0) {
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
  if (so.k == 0) return;  // no block: the bond keeps its tensors
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

// Row blocks of a Jacobi matrix of m rows (32-row blocks, an even count >= 2).
__device__ __forceinline__ int u1_nb(int m) {
  int nb = (m + 31) / 32;
  if (nb < 2) nb = 2;
  return nb + (nb & 1);
}

// Largest charge-block row count per item of the device plan, and the most
// rows (or columns) of the matrix one thread of u1_plan_kernel holds.
constexpr int kU1PlanCap = 2048;
constexpr int kU1PerThread = kU1PlanCap / 256;

// Index of v in the ascending keys[0, K), -1 if absent.
__device__ __forceinline__ int u1_find(const int* keys, int K, int v) {
  int lo = 0, hi = K - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int x = keys[mid];
    if (x == v) return mid;
    if (x < v) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// One workgroup per bond item: the charge blocks of theta' = (rows a s,
// columns t g) built on the device from the chain's bond charges.  Row (a, s)
// carries q_b(a) + q(s), column (t, g) carries q_{b+2}(g) - q(t) (reduced
// modulo n for Z_n); a block is a charge both carry, its rows and columns in
// their order.  The item's blocks take slots [i m_cap, i m_cap + nblk) of
// blk and mats (ascending charge), its rows and columns the same range of
// the row and column lists, its gathered blocks [i m_cap^2, ...) of Xw; the
// slots after its blocks are empty, already converged matrices.  A bond
// dimension out of range or no shared charge gives no block and sets
// MPS_DEV_CHARGE.  Dynamic LDS: 21 m_cap bytes.
__global__ __launch_bounds__(256) void u1_plan_kernel(const BondItem* __restrict__ items,
                                                      const U1Item* __restrict__ ui, int m_cap, double2* Xw,
                                                      int32_t* rmap, double* nrm, U1Block* blk, U1Range* rgs,
                                                      int32_t* rows, int32_t* cols, JacMat* mats, uint32_t* status) {
  extern __shared__ int u1_dyn[];
  int* rq = u1_dyn;          // [m_cap] row charges, then row slots
  int* cq = rq + m_cap;      // [m_cap] column charges, then column slots (-1: no row has it)
  int* keys = cq + m_cap;    // [m_cap] distinct row charges ascending, then block index or -1
  int* nr = keys + m_cap;    // [m_cap] rows per slot, then the block's first row
  int* nc = nr + m_cap;      // [m_cap] columns per slot, then the block's first column
  unsigned char* fq = (unsigned char*)(nc + m_cap);  // [m_cap] first row of its charge
  __shared__ int K_s, nblk_s;
  const int i = blockIdx.x, tid = threadIdx.x;
  const BondItem it = items[i];
  const U1Item u = ui[i];
  const int d = it.d, cm = it.chi_max;
  const int chl = it.chi[it.b], chr = it.chi[it.b + 2];
  const bool bad = chl < 1 || chl > cm || chr < 1 || chr > cm || chl * d > m_cap || chr * d > m_cap;
  const int M = bad ? 0 : chl * d, N = bad ? 0 : d * chr;
  const int kb0 = i * m_cap;
  const size_t x0 = (size_t)i * m_cap * m_cap;
  const int md = u.modulus;
  auto red = [md](long long v) -> int { return md == 0 ? (int)v : (int)(((v % md) + md) % md); };
  for (int r = tid; r < M; r += 256)
    rq[r] = red((long long)u.qb[(size_t)it.b * cm + r / d] + u.qsite[r % d]);
  for (int c = tid; c < N; c += 256)
    cq[c] = red((long long)u.qb[(size_t)(it.b + 2) * cm + c % chr] - u.qsite[c / chr]);
  if (tid == 0) K_s = 0;
  __syncthreads();
  // distinct row charges: the first row of each, ranked by charge
  for (int r = tid; r < M; r += 256) {
    const int v = rq[r];
    bool first = true;
    for (int t = 0; t < r && first; ++t) first = rq[t] != v;
    fq[r] = first ? 1 : 0;
  }
  __syncthreads();
  for (int r = tid; r < M; r += 256)
    if (fq[r]) {
      const int v = rq[r];
      int rank = 0;
      for (int t = 0; t < M; ++t) rank += (fq[t] && rq[t] < v) ? 1 : 0;
      keys[rank] = v;
      atomicAdd(&K_s, 1);
    }
  __syncthreads();
  const int K = K_s;
  // the slot of every row and column, and the counts per slot
  int kr[kU1PerThread], kc[kU1PerThread];
#pragma unroll
  for (int e = 0; e < kU1PerThread; ++e) {
    const int x = tid + e * 256;
    kr[e] = x < M ? u1_find(keys, K, rq[x]) : -1;
    kc[e] = x < N ? u1_find(keys, K, cq[x]) : -1;
  }
  for (int k = tid; k < K; k += 256) {
    nr[k] = 0;
    nc[k] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kU1PerThread; ++e) {
    const int x = tid + e * 256;
    if (x < M) {
      rq[x] = kr[e];
      atomicAdd(&nr[kr[e]], 1);
    }
    if (x < N) {
      cq[x] = kc[e];
      if (kc[e] >= 0) atomicAdd(&nc[kc[e]], 1);
    }
  }
  __syncthreads();
  // the blocks in ascending charge: descriptors, then first row and column
  if (tid == 0) {
    int nb = 0, ro = 0, co = 0;
    size_t xo = 0;
    for (int k = 0; k < K; ++k) {
      const int m = nr[k], n = nc[k];
      if (m > 0 && n > 0) {
        U1Block B;
        B.src = it.X;
        B.ld = N;
        B.x_off = (int64_t)(x0 + xo);
        B.q = keys[k];
        B.m = m;
        B.n = n;
        B.row_off = kb0 + ro;
        B.col_off = kb0 + co;
        B.item = i;
        blk[kb0 + nb] = B;
        JacMat J;
        J.X = Xw + x0 + xo;
        J.rowmap = rmap + kb0 + ro;
        J.nrm2 = nrm + kb0 + ro;
        J.m = m;
        J.n = n;
        J.ld = n;
        J.nb = u1_nb(m);
        J.conv = 0;
        J.rot = 0;
        J.kmax = m;
        J.pad = 0;
        J.fro2 = 0.0;
        mats[kb0 + nb] = J;
        nr[k] = ro;
        nc[k] = co;
        keys[k] = nb;
        ro += m;
        co += n;
        xo += (size_t)m * n;
        ++nb;
      } else {
        keys[k] = -1;
      }
    }
    nblk_s = nb;
    U1Range rg;
    rg.blk0 = kb0;
    rg.nblk = nb;
    rg.row0 = kb0;
    rg.R = ro;
    rg.kmax = min(cm, ro);
    rg.ncols = N;
    rgs[i] = rg;
    if (nb == 0) atomicOr(status, MPS_DEV_CHARGE);
  }
  __syncthreads();
  for (int j = nblk_s + tid; j < m_cap; j += 256) {
    JacMat J;
    J.X = Xw + x0;
    J.rowmap = rmap + kb0;
    J.nrm2 = nrm + kb0;
    J.m = 0;
    J.n = 0;
    J.ld = 1;
    J.nb = 2;
    J.conv = 1;
    J.rot = 0;
    J.kmax = 0;
    J.pad = 0;
    J.fro2 = 0.0;
    mats[kb0 + j] = J;
  }
  // a row's place: its block's first row plus the rows of its slot before it
  for (int r = tid; r < M; r += 256) {
    const int k = rq[r];
    if (keys[k] < 0) continue;
    int before = 0;
    for (int t = 0; t < r; ++t) before += rq[t] == k ? 1 : 0;
    rows[kb0 + nr[k] + before] = r;
  }
  for (int c = tid; c < N; c += 256) {
    const int k = cq[c];
    if (k < 0 || keys[k] < 0) continue;
    int before = 0;
    for (int t = 0; t < c; ++t) before += cq[t] == k ? 1 : 0;
    cols[kb0 + nc[k] + before] = c;
  }
}

// grid (chunks, items): the blocks of item blockIdx.y gathered,
// X_b[i][j] = src[rows[i]][cols[j]]
__global__ __launch_bounds__(256) void u1_gather_items_kernel(const U1Range* __restrict__ rgs,
                                                              const U1Block* __restrict__ blk,
                                                              const int32_t* __restrict__ rows,
                                                              const int32_t* __restrict__ cols,
                                                              double2* __restrict__ Xw) {
  const U1Range rg = rgs[blockIdx.y];
  for (int b = rg.blk0; b < rg.blk0 + rg.nblk; ++b) {
    const U1Block B = blk[b];
    const int64_t tot = (int64_t)B.m * B.n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
      const int r = (int)(e / B.n), c = (int)(e % B.n);
      Xw[B.x_off + e] = B.src[(size_t)rows[B.row_off + r] * B.ld + cols[B.col_off + c]];
    }
  }
}

// grid (items, 16): squared row norms of the item's blocks
__global__ __launch_bounds__(256) void u1_norms_kernel(const U1Range* __restrict__ rgs,
                                                       const JacMat* __restrict__ mats) {
  const U1Range rg = rgs[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int b = rg.blk0; b < rg.blk0 + rg.nblk; ++b) {
    const JacMat& M = mats[b];
    for (int r = blockIdx.y * 4 + wave; r < M.m; r += 4 * gridDim.y) {
      const double2* xr = M.X + (size_t)r * M.ld;
      double a = 0.0;
      for (int c = lane; c < M.n; c += 64) {
        const double2 v = xr[c];
        a += v.x * v.x + v.y * v.y;
      }
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
      if (lane == 0) M.nrm2[r] = a;
    }
  }
}

// grid (items): |X|_F^2 of every block, the natural row order, the flags
__global__ __launch_bounds__(256) void u1_fro_kernel(const U1Range* __restrict__ rgs, JacMat* __restrict__ mats,
                                                     uint32_t* status) {
  __shared__ double red[256];
  const U1Range rg = rgs[blockIdx.x];
  const int tid = threadIdx.x;
  for (int b = rg.blk0; b < rg.blk0 + rg.nblk; ++b) {
    JacMat* M = mats + b;
    const int m = M->m;
    double a = 0.0;
    for (int r = tid; r < m; r += 256) a += M->nrm2[r];
    red[tid] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    const double f2 = red[0];
    __syncthreads();
    for (int g = tid; g < m; g += 256) M->rowmap[g] = g;
    if (tid == 0) {
      M->fro2 = f2;
      M->rot = 0;
      M->conv = (f2 == f2 && f2 < 1e300) ? 0 : 1;
      if (M->conv) atomicOr(status, MPS_DEV_NONFINITE);
    }
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
  size_t oItems, oRb, oX, oMats, oBlk, oRg, oRows, oCols, oRm, oNrm, oPe, oS2, oList, oCnt, off;
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
    oList = p.take<int32_t>(nm);
    oCnt = p.take<int32_t>(4);
    off = p.off + 256;
  }
};

}  // namespace

size_t u1_layer_bytes(int n_cap, int m_cap, int chi_cap) { return U1Plan(n_cap, m_cap, chi_cap).off; }

mps_status u1_layer(mps_handle h, hipStream_t s, const BondItem* it_dev, const U1Item* ui_dev, int n, int n_cap,
                    int m_cap, int chi_cap, double eps, bool c128, char* region, SelOut* sel, int32_t* unconv) {
  if (n <= 0) return MPS_OK;
  if (n > n_cap || m_cap > kU1PlanCap || (int64_t)n_cap * m_cap > kSchedCap)
    return mps_fail(h, MPS_ERR_CAPACITY, "charge blocks exceed the layer workspace");
  const U1Plan P(n_cap, m_cap, chi_cap);
  char* const ws = (char*)(((uintptr_t)region + 255) & ~(uintptr_t)255);
  double2* Xw = (double2*)(ws + P.oX);
  JacMat* mats = (JacMat*)(ws + P.oMats);
  U1Block* blk = (U1Block*)(ws + P.oBlk);
  U1Range* rgd = (U1Range*)(ws + P.oRg);
  int32_t* rows = (int32_t*)(ws + P.oRows);
  int32_t* cols = (int32_t*)(ws + P.oCols);
  // the blocks, their rows and columns from the bond charges on the device:
  // no launch below depends on their number or shapes on the host
  u1_plan_kernel<<<n, 256, (size_t)m_cap * (5 * sizeof(int) + 1), s>>>(
      it_dev, ui_dev, m_cap, Xw, (int32_t*)(ws + P.oRm), (double*)(ws + P.oNrm), blk, rgd, rows, cols, mats,
      h->status_dev);
  MPS_TRY_HIP(h, hipGetLastError());
  const int gx = std::max(1, std::min(64, m_cap * m_cap / 4096));
  u1_gather_items_kernel<<<dim3(gx, n), 256, 0, s>>>(rgd, blk, rows, cols, Xw);
  MPS_TRY_HIP(h, hipGetLastError());
  u1_norms_kernel<<<dim3(n, 16), 256, 0, s>>>(rgd, mats);
  MPS_TRY_HIP(h, hipGetLastError());
  u1_fro_kernel<<<n, 256, 0, s>>>(rgd, mats, h->status_dev);
  MPS_TRY_HIP(h, hipGetLastError());
  mps_status st = run_jacobi_slots(h, s, mats, n * m_cap, jac_nb(m_cap), unconv, (int32_t*)(ws + P.oList),
                                   (int32_t*)(ws + P.oCnt));
  if (st != MPS_OK) return st;
  int32_t* pe = (int32_t*)(ws + P.oPe);
  double* s2o = (double*)(ws + P.oS2);
  u1_select_kernel<<<n, 256, (size_t)m_cap * (sizeof(double) + sizeof(int)), s>>>(mats, blk, rgd,
                                                                                 count_rule_eps(h, eps), pe, s2o, sel);
  MPS_TRY_HIP(h, hipGetLastError());
  if (c128)
    u1_wb_kernel<double2><<<dim3(chi_cap, n), 256, 0, s>>>(it_dev, ui_dev, mats, blk, rgd, cols, pe, s2o, sel);
  else
    u1_wb_kernel<float2><<<dim3(chi_cap, n), 256, 0, s>>>(it_dev, ui_dev, mats, blk, rgd, cols, pe, s2o, sel);
  MPS_TRY_HIP(h, hipGetLastError());
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
