// Gram partials on FP32 MFMA for the mixed-precision pre-sweeps.
//
// The factor G stays FP64 in HBM; each lane converts the values it loads to
// FP32 and the products are accumulated by v_mfma_f32_16x16x4f32 (twice the
// FP64 matrix rate).  Only the Gram block A_P = [G_i G_j]^* [G_i G_j] (eq. 3.6)
// is formed this way: the pivot solver factors it and computes every rotation
// in FP64 and accumulates W_P in FP64, and the update of G stays FP64, so each
// applied transformation is J-unitary to FP64 working precision (the
// robustness remark (a) of Section 2.3: inaccurate rotation parameters do not
// harm the one-sided process as long as the transformation applied to G is
// numerically J-unitary).
//
// Lane layout of v_mfma_f32_16x16x4f32 (measured on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16] and receives D[4*(l/16) + v][l%16] in
// element v (note: not the layout of the FP64 instruction).
#include "jj_device.h"

namespace jj {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4m __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16f(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Real: same grid, row grouping and output format as the FP64 Gram kernel.
__global__ __launch_bounds__(256) void k_gram_f32mix(const double* __restrict__ G0, int ldg0, int n0,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     int rows_per_chunk, double* __restrict__ part, Batch bt) {
  __shared__ d4m red[10][64];
  const int nch = gridDim.x;
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = const_cast<double*>(G0);
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (ch > 0 && ch * rows_per_chunk >= n) return;  // chunk beyond this problem's rows
  const gdbl* G = as_global(Gm);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const gdbl* cp[4];
#pragma unroll
  for (int J = 0; J < 4; J++) {
    int c = J * 16 + c16;
    int pc = (c < m) ? cols[p * kMaxPivot + c] : -1;
    cp[J] = (pc >= 0) ? G + (size_t)pc * ldg : nullptr;
  }
  f4 acc[10];
#pragma unroll
  for (int t = 0; t < 10; t++) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  float x[4][4], xn[4][4];
  int base = r0 + wave * 16;
#pragma unroll
  for (int J = 0; J < 4; J++)
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      int row = base + 4 * g + kk;
      x[J][kk] = (cp[J] != nullptr && row < r1) ? (float)cp[J][row] : 0.f;
    }
  for (; base < r1; base += 64) {
    const int nb = base + 64;
#pragma unroll
    for (int J = 0; J < 4; J++)
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        int row = nb + 4 * g + kk;
        xn[J][kk] = (cp[J] != nullptr && row < r1) ? (float)cp[J][row] : 0.f;
      }
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      int t = 0;
#pragma unroll
      for (int I = 0; I < 4; I++)
#pragma unroll
        for (int J = I; J < 4; J++) {
          if (J < nt) acc[t] = mfma16f(x[I][kk], x[J][kk], acc[t]);
          t++;
        }
    }
#pragma unroll
    for (int J = 0; J < 4; J++)
#pragma unroll
      for (int kk = 0; kk < 4; kk++) x[J][kk] = xn[J][kk];
  }
  // waves reduced in FP64, fixed order ((w3 + w2) + w1) + w0
  d4m accd[10];
#pragma unroll
  for (int t = 0; t < 10; t++)
    accd[t] = d4m{(double)acc[t][0], (double)acc[t][1], (double)acc[t][2], (double)acc[t][3]};
  for (int w = 3; w >= 1; w--) {
    if (wave == w)
      for (int t = 0; t < 10; t++) red[t][lane] = accd[t];
    __syncthreads();
    if (wave == w - 1)
      for (int t = 0; t < 10; t++) accd[t] = red[t][lane] + accd[t];
    __syncthreads();
  }
  if (wave == 0) {
    double* out = part + ((size_t)slot * nch + ch) * (kMaxPivot * kMaxPivot);
    int t = 0;
#pragma unroll
    for (int I = 0; I < 4; I++)
#pragma unroll
      for (int J = I; J < 4; J++) {
        if (J < nt) {
#pragma unroll
          for (int v = 0; v < 4; v++) out[(16 * I + 4 * g + v) * kMaxPivot + 16 * J + c16] = accd[t][v];
        }
        t++;
      }
  }
}

// Complex: Re A = Xr^T Xr + Xi^T Xi, Im A = Xr^T Xi - Xi^T Xr on FP32 MFMA.
__global__ __launch_bounds__(256, 2) void k_gram_c64mix(const double* __restrict__ G0, int ldg0, int n0,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     int rows_per_chunk, double* __restrict__ part, Batch bt) {
  __shared__ d4m red[10][2][64];
  const int nch = gridDim.x;
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = const_cast<double*>(G0);
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (ch > 0 && ch * rows_per_chunk >= n) return;  // chunk beyond this problem's rows
  const gdbl2* G = as_global2(Gm);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const gdbl2* cp[4];
#pragma unroll
  for (int J = 0; J < 4; J++) {
    int c = J * 16 + c16;
    int pc = (c < m) ? cols[p * kMaxPivot + c] : -1;
    cp[J] = (pc >= 0) ? G + (size_t)pc * ldg : nullptr;
  }
  f4 are[10], aim[10];
#pragma unroll
  for (int t = 0; t < 10; t++) {
    are[t] = f4{0.f, 0.f, 0.f, 0.f};
    aim[t] = f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int base = r0 + wave * 16; base < r1; base += 64) {
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      const int row = base + 4 * g + kk;
      float xr[4], xi[4];
#pragma unroll
      for (int J = 0; J < 4; J++) {
        const dv2 v = (cp[J] != nullptr && row < r1) ? cp[J][row] : dv2{0.0, 0.0};
        xr[J] = (float)v.x;
        xi[J] = (float)v.y;
      }
      int t = 0;
#pragma unroll
      for (int I = 0; I < 4; I++)
#pragma unroll
        for (int J = I; J < 4; J++) {
          if (J < nt) {
            are[t] = mfma16f(xr[I], xr[J], are[t]);
            are[t] = mfma16f(xi[I], xi[J], are[t]);
            aim[t] = mfma16f(xr[I], xi[J], aim[t]);
            aim[t] = mfma16f(-xi[I], xr[J], aim[t]);
          }
          t++;
        }
    }
  }
  d4m dre[10], dim[10];
#pragma unroll
  for (int t = 0; t < 10; t++) {
    dre[t] = d4m{(double)are[t][0], (double)are[t][1], (double)are[t][2], (double)are[t][3]};
    dim[t] = d4m{(double)aim[t][0], (double)aim[t][1], (double)aim[t][2], (double)aim[t][3]};
  }
  for (int w = 3; w >= 1; w--) {
    if (wave == w)
      for (int t = 0; t < 10; t++) {
        red[t][0][lane] = dre[t];
        red[t][1][lane] = dim[t];
      }
    __syncthreads();
    if (wave == w - 1)
      for (int t = 0; t < 10; t++) {
        dre[t] = red[t][0][lane] + dre[t];
        dim[t] = red[t][1][lane] + dim[t];
      }
    __syncthreads();
  }
  if (wave == 0) {
    double* out = part + ((size_t)slot * nch + ch) * (2 * kMaxPivot * kMaxPivot);
    int t = 0;
#pragma unroll
    for (int I = 0; I < 4; I++)
#pragma unroll
      for (int J = I; J < 4; J++) {
        if (J < nt) {
#pragma unroll
          for (int v = 0; v < 4; v++) {
            size_t e = (size_t)(16 * I + 4 * g + v) * kMaxPivot + 16 * J + c16;
            out[2 * e] = dre[t][v];
            out[2 * e + 1] = dim[t][v];
          }
        }
        t++;
      }
  }
}

void launch_gram_f32mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b) {
  launch(k_gram_f32mix, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part, b);
}

void launch_gram_c64mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b) {
  launch(k_gram_c64mix, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part, b);
}

}  // namespace jj
