// Complex products on MFMA with three real products each (Gauss's form):
//   t1 = A_re B_re,  t2 = A_im B_im,  t3 = (A_re + A_im)(B_re + B_im),
//   C_re = t1 - t2,  C_im = t3 - t1 - t2,
// three matrix instructions per complex product instead of four.  The operand
// sums are formed in registers from the staged fragments; the lane layout is
// that of mfma_tile.h (2 x 2 waves, each MI x NJ tiles of 16 x 16).  The
// rounding error of C_im grows from about 2 to about 4 units of |A||B| (C_im
// is a difference of the three sums), in either precision.
#pragma once
#include "mfma_tile.h"

template <class T, int MI, int NJ>
struct Acc3 {
  typename Cx<T>::V4 t1[MI][NJ];
  typename Cx<T>::V4 t2[MI][NJ];
  typename Cx<T>::V4 t3[MI][NJ];
};

template <class T, int MI, int NJ>
__device__ __forceinline__ void acc3_zero(Acc3<T, MI, NJ>& a) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a.t1[i][j][r] = 0;
        a.t2[i][j][r] = 0;
        a.t3[i][j][r] = 0;
      }
}

// One staged K-chunk: As[TBK][lda] (rows of the tile), Bs[TBK][ldb] (columns).
template <class T, int MI, int NJ>
__device__ __forceinline__ void mma3_chunk(const T* __restrict__ As, int lda, const T* __restrict__ Bs, int ldb,
                                           Acc3<T, MI, NJ>& acc, int wm, int wn, int lane) {
  typedef typename Cx<T>::R R;
#pragma unroll
  for (int kk = 0; kk < TBK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    T a[MI], b[NJ];
    R as[MI], bs[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      a[i] = As[kr * lda + wm + i * 16 + (lane & 15)];
      as[i] = a[i].x + a[i].y;
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      b[j] = Bs[kr * ldb + wn + j * 16 + (lane & 15)];
      bs[j] = b[j].x + b[j].y;
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        acc.t1[i][j] = Cx<T>::mfma(a[i].x, b[j].x, acc.t1[i][j]);
        acc.t2[i][j] = Cx<T>::mfma(a[i].y, b[j].y, acc.t2[i][j]);
        acc.t3[i][j] = Cx<T>::mfma(as[i], bs[j], acc.t3[i][j]);
      }
  }
}

// Entry r of accumulator tile (i, j) as a complex number.
template <class T, int MI, int NJ>
__device__ __forceinline__ T acc3_get(const Acc3<T, MI, NJ>& acc, int i, int j, int r) {
  T v;
  v.x = acc.t1[i][j][r] - acc.t2[i][j][r];
  v.y = acc.t3[i][j][r] - acc.t1[i][j][r] - acc.t2[i][j][r];
  return v;
}

// One interface over both accumulator forms, for kernels that pick the form
// per precision: Acc3 (three products) or AccTileT (four).
template <class T, int MI, int NJ>
__device__ __forceinline__ void acc_clear(Acc3<T, MI, NJ>& a) { acc3_zero<T, MI, NJ>(a); }
template <class T, int MI, int NJ>
__device__ __forceinline__ void acc_clear(AccTileT<T, MI, NJ>& a) { acc_zero_t<T, MI, NJ>(a); }
template <class T, int MI, int NJ>
__device__ __forceinline__ void acc_chunk(const T* As, int lda, const T* Bs, int ldb, Acc3<T, MI, NJ>& a, int wm,
                                          int wn, int lane) {
  mma3_chunk<T, MI, NJ>(As, lda, Bs, ldb, a, wm, wn, lane);
}
template <class T, int MI, int NJ>
__device__ __forceinline__ void acc_chunk(const T* As, int lda, const T* Bs, int ldb, AccTileT<T, MI, NJ>& a, int wm,
                                          int wn, int lane) {
  mma_chunk_t<T, MI, NJ>(As, lda, Bs, ldb, a, wm, wn, lane);
}
template <class T, int MI, int NJ>
__device__ __forceinline__ T acc_value(const Acc3<T, MI, NJ>& a, int i, int j, int r) {
  return acc3_get<T, MI, NJ>(a, i, j, r);
}
template <class T, int MI, int NJ>
__device__ __forceinline__ T acc_value(const AccTileT<T, MI, NJ>& a, int i, int j, int r) {
  T v;
  v.x = a.re[i][j][r];
  v.y = a.im[i][j][r];
  return v;
}
