// 64x64 complex output tile on MFMA, one 256-thread workgroup = 4 waves,
// each wave a 32x32 quarter made of 2x2 16x16 MFMA tiles.  Two precisions:
//   complex64  : v_mfma_f32_16x16x4f32, FP32 accumulation
//   complex128 : v_mfma_f64_16x16x4f64, FP64 accumulation
// A complex product is four real products:
//   C_re += A_re B_re - A_im B_im,   C_im += A_re B_im + A_im B_re.
// Operands are staged in LDS as As[k][row] and Bs[k][col], a K-chunk of 16 at
// a time.  Lane layout of the 16x16x4 instructions (both precisions): lane l
// supplies A[l%16][l/16] and B[l/16][l%16].  Accumulator entry r of lane l is
// C[4*(l/16)+r][l%16] for f32 but C[l/16+4r][l%16] for f64 (measured on
// gfx950 with an in-bounds probe); acc_row() gives the row.
#pragma once
#include "common.h"

#define TBM 64
#define TBN 64
#define TBK 16
#define TLD 68   // LDS row pitch (complex elements) of the staged operands

typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T>
struct Cx;
template <>
struct Cx<float2> {
  typedef float R;
  typedef floatx4 V4;
  static __device__ __forceinline__ V4 mfma(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ float2 make(double re, double im) { return make_float2((float)re, (float)im); }
  static __device__ __forceinline__ int acc_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Cx<double2> {
  typedef double R;
  typedef doublex4 V4;
  static __device__ __forceinline__ V4 mfma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ double2 make(double re, double im) { return make_double2(re, im); }
  static __device__ __forceinline__ int acc_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <class T>
struct AccTile {
  typename Cx<T>::V4 re[2][2];
  typename Cx<T>::V4 im[2][2];
};

template <class T>
__device__ __forceinline__ void acc_zero(AccTile<T>& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a.re[i][j][r] = 0;
        a.im[i][j][r] = 0;
      }
}

// One staged K-chunk: As[TBK][TLD], Bs[TBK][TLD].
template <class T>
__device__ __forceinline__ void mma_chunk(const T* __restrict__ As, const T* __restrict__ Bs, AccTile<T>& acc,
                                          int wm, int wn, int lane) {
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    T a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = As[kr * TLD + wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Bs[kr * TLD + wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc.re[i][j] = Cx<T>::mfma(a[i].x, b[j].x, acc.re[i][j]);
        acc.re[i][j] = Cx<T>::mfma(-a[i].y, b[j].y, acc.re[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].x, b[j].y, acc.im[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].y, b[j].x, acc.im[i][j]);
      }
  }
}

// Same with the A operand read in place from a tile of pitch lda: A(k, m) = Al[k * lda + m].
template <class T>
__device__ __forceinline__ void mma_chunk_lda(const T* __restrict__ Al, int lda, const T* __restrict__ Bs,
                                              AccTile<T>& acc, int wm, int wn, int lane) {
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    T a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = Al[kr * lda + wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = Bs[kr * TLD + wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc.re[i][j] = Cx<T>::mfma(a[i].x, b[j].x, acc.re[i][j]);
        acc.re[i][j] = Cx<T>::mfma(-a[i].y, b[j].y, acc.re[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].x, b[j].y, acc.im[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].y, b[j].x, acc.im[i][j]);
      }
  }
}

// Write the accumulators into an LDS tile Cs[TBM][ldc].
template <class T>
__device__ __forceinline__ void acc_to_lds(const AccTile<T>& acc, T* Cs, int ldc, int wm, int wn, int lane) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = wm + i * 16 + Cx<T>::acc_row(lane, r);
        int col = wn + j * 16 + (lane & 15);
        T v;
        v.x = acc.re[i][j][r];
        v.y = acc.im[i][j][r];
        Cs[row * ldc + col] = v;
      }
}

// ---------------------------------------------------------------------------
// Tile shapes for the tuned GEMMs: 2 x 2 waves, each wave MI x NJ MFMA tiles
// of 16 x 16, so a workgroup tile is (32 MI) x (32 NJ); MI = NJ = 2 is the
// 64 x 64 tile above.  The staged chunks have pitches BM + 4 and BN + 4.
// ---------------------------------------------------------------------------
template <class T, int MI, int NJ>
struct AccTileT {
  typename Cx<T>::V4 re[MI][NJ];
  typename Cx<T>::V4 im[MI][NJ];
};

template <class T, int MI, int NJ>
__device__ __forceinline__ void acc_zero_t(AccTileT<T, MI, NJ>& a) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a.re[i][j][r] = 0;
        a.im[i][j][r] = 0;
      }
}

// One staged K-chunk: As[TBK][lda] (rows of the tile), Bs[TBK][ldb] (columns).
template <class T, int MI, int NJ>
__device__ __forceinline__ void mma_chunk_t(const T* __restrict__ As, int lda, const T* __restrict__ Bs, int ldb,
                                            AccTileT<T, MI, NJ>& acc, int wm, int wn, int lane) {
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    T a[MI], b[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) a[i] = As[kr * lda + wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = Bs[kr * ldb + wn + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        acc.re[i][j] = Cx<T>::mfma(a[i].x, b[j].x, acc.re[i][j]);
        acc.re[i][j] = Cx<T>::mfma(-a[i].y, b[j].y, acc.re[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].x, b[j].y, acc.im[i][j]);
        acc.im[i][j] = Cx<T>::mfma(a[i].y, b[j].x, acc.im[i][j]);
      }
  }
}

// The tile shapes the GEMM autotuner chooses from: (MI, NJ) of candidate c.
constexpr int kGemmCands = 6;
__host__ __device__ constexpr int gemm_cand_mi(int c) { return c == 1 ? 4 : (c == 3 || c == 5) ? 1 : 2; }
__host__ __device__ constexpr int gemm_cand_nj(int c) { return c == 2 ? 4 : (c == 4 || c == 5) ? 1 : 2; }
