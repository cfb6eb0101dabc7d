// Three-level pivot (paper, Section 5 and Algorithm 5.1): a pivot of two
// blocks of up to 64 columns each (block width 64, up to 128 columns) is
// "shortened" to the Cholesky factor R of its Gram block A_P = R^* R (order up
// to 128), and R is then orthogonalised by the blocked block-oriented method
// with inner blocks of half the outer width, whose inner partition respects
// the boundary between the two outer blocks (Algorithm 5.1).  The inner
// steps run on the existing kernels (Gram of R's columns, pivot solve, update)
// and each inner transformation is applied to R and to the corresponding
// columns of G (the accumulated transformation W = W_1 W_2 ... applied factor
// by factor, which needs no 128-column update).
//
// This file holds the one new kernel of that path: k_chol128 sums the Gram
// partials of the six 64-column sub-pivots that cover the upper triangle of
// A_P (the diagonal blocks A_II, A_JJ and the four quarter blocks of A_IJ),
// factors A_P = R^* R in LDS (packed upper triangle: 128 x 129 / 2 entries),
// and writes R (zero below the diagonal and beyond the pivot's order) to the
// pair's 128 x 128 slot of the R workspace.
#include "jj_device.h"

#include <math.h>

namespace jj {

typedef double dv2c __attribute__((ext_vector_type(2)));

constexpr int kP3 = kMaxPivot3;                 // largest three-level pivot: 128 columns
constexpr int kP3Packed = kP3 * (kP3 + 1) / 2;  // entries of its packed upper triangle
constexpr int kChol3Threads = 512;

__device__ __forceinline__ int pk(int i, int j) { return j * (j + 1) / 2 + i; }  // (i <= j)

template <bool CPLX>
struct C3;
template <>
struct C3<false> {
  typedef double T;
  static __device__ __forceinline__ T zero() { return 0.0; }
  static __device__ __forceinline__ T add(T a, T b) { return a + b; }
  static __device__ __forceinline__ double re(T a) { return a; }
  static __device__ __forceinline__ double abs2(T a) { return a * a; }
  static __device__ __forceinline__ T scale(T a, double s) { return a * s; }
  // a - conj(u) v
  static __device__ __forceinline__ T sub_cprod(T a, T u, T v) { return a - u * v; }
  static __device__ __forceinline__ bool finite(T a) { return isfinite(a); }
};
template <>
struct C3<true> {
  typedef dv2c T;
  static __device__ __forceinline__ T zero() { return T{0.0, 0.0}; }
  static __device__ __forceinline__ T add(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
  static __device__ __forceinline__ double re(T a) { return a.x; }
  static __device__ __forceinline__ double abs2(T a) { return a.x * a.x + a.y * a.y; }
  static __device__ __forceinline__ T scale(T a, double s) { return T{a.x * s, a.y * s}; }
  static __device__ __forceinline__ T sub_cprod(T a, T u, T v) {
    return T{a.x - (u.x * v.x + u.y * v.y), a.y - (u.x * v.y - u.y * v.x)};
  }
  static __device__ __forceinline__ bool finite(T a) { return isfinite(a.x) && isfinite(a.y); }
};

// One workgroup per pair.  part: the six sub-pivot partial sets of pair p at
// part + (6p + v) * nch * 64 * 64 (scalars), v = 0: I, 1: J, 2: I1 J1,
// 3: I1 J2, 4: I2 J1, 5: I2 J2 (I = I1 I2 and J = J1 J2 the halves of the
// uniform inner partition).  n1[p], n2[p]: the sizes of I and J.  R: the pair's
// 128 x 128 slot at R + p * 128 * ldr (scalars), ldr >= 128 rows.
template <bool CPLX>
__global__ __launch_bounds__(kChol3Threads) void k_chol128(const double* __restrict__ part, int nch, int nrows,
                                                           int rows_per_chunk, const int* __restrict__ n1s,
                                                           const int* __restrict__ n2s, int count,
                                                           double* __restrict__ Rout, int ldr, int first,
                                                           SweepStats* st) {
  typedef typename C3<CPLX>::T T;
  __shared__ T A[kP3Packed];
  __shared__ double s_dinv[kP3];
  __shared__ double redv[kChol3Threads / 64];
  __shared__ int s_bad;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (p >= count) return;
  const int nI = n1s[p], nJ = n2s[p], m = nI + nJ;
  const int a1 = (nI + 1) / 2, b1 = (nJ + 1) / 2;
  const int nchp = min(nch, (nrows + rows_per_chunk - 1) / rows_per_chunk);
  const T* P = reinterpret_cast<const T*>(part);
  if (tid == 0) s_bad = 0;
  // ---- A_P from the six sub-pivots (entries with i <= j only) ----
  for (int e = tid; e < kP3Packed; e += kChol3Threads) {
    // packed index -> (i, j), column by column
    int j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > e) j--;
    while ((j + 1) * (j + 2) / 2 <= e) j++;
    const int i = e - j * (j + 1) / 2;
    T v = C3<CPLX>::zero();
    if (j < m) {
      int sub, r, c;  // sub-pivot and its (row, column)
      if (j < nI) {
        sub = 0, r = i, c = j;
      } else if (i >= nI) {
        sub = 1, r = i - nI, c = j - nI;
      } else {
        const int jj = j - nI;
        const bool iu = i < a1, ju = jj < b1;
        sub = iu ? (ju ? 2 : 3) : (ju ? 4 : 5);
        const int nfi = iu ? a1 : nI - a1;  // first-block size of that sub-pivot
        r = iu ? i : i - a1;
        c = nfi + (ju ? jj : jj - b1);
      }
      const T* src = P + ((size_t)(6 * p + sub) * nch) * (kMaxPivot * kMaxPivot) + r * kMaxPivot + c;
      v = src[0];
      for (int k = 1; k < nchp; k++) v = C3<CPLX>::add(v, src[(size_t)k * (kMaxPivot * kMaxPivot)]);
    }
    A[e] = v;
  }
  __syncthreads();
  // ---- scaled off-diagonal of the part the steps annihilate (all of A_P in
  // the first step of a sweep, A_IJ otherwise), for the sweep's statistics ----
  if (tid < kP3) {
    const double d = tid < m ? C3<CPLX>::re(A[pk(tid, tid)]) : 1.0;
    s_dinv[tid] = (d > 0.0 && isfinite(d)) ? 1.0 / sqrt(d) : 0.0;
    if (tid < m && !(d > 0.0 && isfinite(d))) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  double off = 0.0;
  for (int e = tid; e < kP3Packed; e += kChol3Threads) {
    int j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > e) j--;
    while ((j + 1) * (j + 2) / 2 <= e) j++;
    const int i = e - j * (j + 1) / 2;
    if (i < j && j < m && (first || (i < nI && j >= nI))) {
      const double f = s_dinv[i] * s_dinv[j];
      off = fmax(off, sqrt(C3<CPLX>::abs2(A[e])) * f);
    }
  }
#pragma unroll
  for (int msk = 32; msk > 0; msk >>= 1) off = fmax(off, __shfl_xor(off, msk));
  if ((tid & 63) == 0) redv[tid >> 6] = off;
  __syncthreads();
  if (tid == 0) {
    double o = redv[0];
    for (int w = 1; w < kChol3Threads / 64; w++) o = fmax(o, redv[w]);
    atomicMax(&st->max_off_bits, (unsigned long long)__double_as_longlong(isfinite(o) ? o : 1.0e300));
  }
  // ---- Cholesky A_P = R^* R, row by row: r_kk = sqrt(a_kk), r_kj = a_kj / r_kk,
  // then a_ij -= conj(r_ki) r_kj for k < i <= j ----
  for (int k = 0; k < m && !s_bad; k++) {
    const double d = C3<CPLX>::re(A[pk(k, k)]);
    __syncthreads();  // every thread has read a_kk
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) s_bad = 1;
      __syncthreads();
      break;
    }
    const double rkk = sqrt(d), rinv = 1.0 / rkk;
    for (int j = k + 1 + tid; j < m; j += kChol3Threads) A[pk(k, j)] = C3<CPLX>::scale(A[pk(k, j)], rinv);
    if (tid == 0) {
      T dk = C3<CPLX>::zero();
      if constexpr (CPLX) dk.x = rkk; else dk = rkk;
      A[pk(k, k)] = dk;
    }
    __syncthreads();
    // trailing update: 4 threads per column j, rows i = k+1 .. j
    for (int j = k + 1 + (tid >> 2); j < m; j += kChol3Threads / 4) {
      const T rkj = A[pk(k, j)];
      for (int i = k + 1 + (tid & 3); i <= j; i += 4) A[pk(i, j)] = C3<CPLX>::sub_cprod(A[pk(i, j)], A[pk(k, i)], rkj);
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicOr(&st->breakdown, 1);
    return;
  }
  // ---- R (zero below the diagonal and outside m x m) to the pair's slot ----
  T* Rp = reinterpret_cast<T*>(Rout) + (size_t)p * kP3 * ldr;
  for (int e = tid; e < kP3 * kP3; e += kChol3Threads) {
    const int r = e % kP3, c = e / kP3;
    Rp[(size_t)c * ldr + r] = (r <= c && c < m) ? A[pk(r, c)] : C3<CPLX>::zero();
  }
}

void launch_chol128(bool cplx, const double* part, int nch, int nrows, int rows_per_chunk, const int* n1s,
                    const int* n2s, int count, double* R, int ldr, int first, SweepStats* st, hipStream_t stream) {
  if (cplx)
    launch(k_chol128<true>, dim3(count), dim3(kChol3Threads), 0, stream, part, nch, nrows, rows_per_chunk, n1s, n2s,
           count, R, ldr, first, st);
  else
    launch(k_chol128<false>, dim3(count), dim3(kChol3Threads), 0, stream, part, nch, nrows, rows_per_chunk, n1s,
           n2s, count, R, ldr, first, st);
}

}  // namespace jj
