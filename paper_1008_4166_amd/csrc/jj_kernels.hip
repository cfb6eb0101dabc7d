// gfx950 kernels of the blocked one-sided hyperbolic J-Jacobi sweep (real FP64).
//
// One block step on a pair of block-columns (paper, Section 5.3, steps 1-4):
//   k_gram_f64    A_P = [G_i G_j]^T [G_i G_j]                      (eq. 3.6)
//   k_pivot_f64   Cholesky A_P = R^T R (eq. 3.8), one-sided J-Jacobi on the
//                 columns of R accumulating W_P (eq. 3.12, Algorithms 3.1/3.2)
//   k_update_f64  [G_i G_j] <- [G_i G_j] W_P                        (eq. 3.4)
// and the finalisation lambda_i = j_i ||g_i||^2, v_i = g_i/||g_i|| (eq. 2.10).
//
// MFMA: v_mfma_f64_16x16x4f64.  Lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[4v + l/16][l%16] in element v of its 4-double accumulator.
#include "jj_device.h"

#include <math.h>

namespace jj {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Gram partials.  Grid (nch, P), 256 threads.  Chunk ch covers rows
// [ch*rows_per_chunk, min(n, (ch+1)*rows_per_chunk)).  Each wave takes 16-row
// groups; within a group lane l (column c16 = l%16 of each 16-column tile,
// row quarter g = l/16) holds rows 4g..4g+3, so the four k-steps of the group
// are rows {4g + kk}.  All upper tiles (I <= J) of the 64x64 partial are
// accumulated; the four waves are reduced through LDS in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_f64(const double* __restrict__ G, int ldg, int n,
                                                  const int* __restrict__ cols, const int* __restrict__ mlist,
                                                  int rows_per_chunk, double* __restrict__ part) {
  __shared__ d4 red[2][10][64];
  const int p = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);

  const double* cp[4];
#pragma unroll
  for (int J = 0; J < 4; J++) {
    int c = J * 16 + c16;
    int pc = (c < m) ? cols[p * kMaxPivot + c] : -1;
    cp[J] = (pc >= 0) ? G + (size_t)pc * ldg : nullptr;
  }
  d4 acc[10];
#pragma unroll
  for (int t = 0; t < 10; t++) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (int base = r0 + wave * 16; base < r1; base += 64) {
    double x[4][4];
#pragma unroll
    for (int J = 0; J < 4; J++)
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        int row = base + 4 * g + kk;
        x[J][kk] = (cp[J] != nullptr && row < r1) ? cp[J][row] : 0.0;
      }
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      int t = 0;
#pragma unroll
      for (int I = 0; I < 4; I++)
#pragma unroll
        for (int J = I; J < 4; J++) {
          if (J < nt) acc[t] = mfma16(x[I][kk], x[J][kk], acc[t]);
          t++;
        }
    }
  }
  // fixed-order reduction of the four waves: (w0 + w2) + (w1 + w3)
  if (wave >= 2)
    for (int t = 0; t < 10; t++) red[wave - 2][t][lane] = acc[t];
  __syncthreads();
  if (wave < 2)
    for (int t = 0; t < 10; t++) acc[t] += red[wave][t][lane];
  __syncthreads();
  if (wave == 1)
    for (int t = 0; t < 10; t++) red[0][t][lane] = acc[t];
  __syncthreads();
  if (wave == 0) {
    double* out = part + ((size_t)p * nch + ch) * (kMaxPivot * kMaxPivot);
    int t = 0;
#pragma unroll
    for (int I = 0; I < 4; I++)
#pragma unroll
      for (int J = I; J < 4; J++) {
        d4 s = acc[t] + red[0][t][lane];
        if (J < nt) {
#pragma unroll
          for (int v = 0; v < 4; v++) out[(16 * I + 4 * v + g) * kMaxPivot + 16 * J + c16] = s[v];
        }
        t++;
      }
  }
}

// ---------------------------------------------------------------------------
// Rotation parameters (paper, Algorithm 3.1 with sigma = +j_r j_s; real case
// eta = a_rs).  Returns 0: no rotation needed, 1: rotation (cs, sn) computed,
// -1: hyperbolic rotation does not exist (|theta| <= 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rot_params(double arr, double ass, double ars, double sigma, double tol,
                                          double* cs, double* sn) {
  if (!(fabs(ars) > tol * sqrt(arr) * sqrt(ass))) return 0;
  double theta = sigma * (ass - sigma * arr) / (2.0 * ars);
  double at = fabs(theta);
  if (sigma < 0.0 && at <= 1.0) return -1;
  double sg = theta < 0.0 ? -1.0 : 1.0;
  double t;
  if (at > 1.0)
    t = sg / (at * (1.0 + sqrt(1.0 + sigma / (theta * theta))));
  else
    t = sg / (at + sqrt(theta * theta + sigma));
  double c;
  if (sigma > 0.0)
    c = 1.0 / sqrt(1.0 + t * t);
  else
    c = 1.0 / sqrt((1.0 - fabs(t)) * (1.0 + fabs(t)));
  *cs = c;
  *sn = c * t;
  return 1;
}

// ---------------------------------------------------------------------------
// Pivot solve.  Grid P, 256 threads.  LDS holds R and W_P column-major with
// leading dimension 65.  Inner ordering: circle round-robin on the m' = m
// rounded up to even columns (column 0 fixed, the rest rotate), m'/2 disjoint
// column pairs per round handled by groups of 8 lanes.
// inner_mode 0: full diagonalisation (repeat inner sweeps until one applies no
// rotation, at most inner_max).  inner_mode 1: a single pass over the pairs
// (r in the first block, s in the second) of the off-diagonal block.
// ---------------------------------------------------------------------------
constexpr int LDR = kMaxPivot + 1;

__global__ __launch_bounds__(256) void k_pivot_f64(const double* __restrict__ part, int nch,
                                                   const int* __restrict__ mlist, const int* __restrict__ nfirst,
                                                   const signed char* __restrict__ sgl, double tol, int inner_max,
                                                   int inner_mode, double* __restrict__ Wout,
                                                   int* __restrict__ rotflag, SweepStats* st) {
  __shared__ double R[kMaxPivot * LDR];
  __shared__ double W[kMaxPivot * LDR];
  __shared__ double redv[256];
  __shared__ int s_cnt, s_bad, s_total, s_sweeps;
  __shared__ double s_piv;
  const int p = blockIdx.x, tid = threadIdx.x;
  const int m = mlist[p];
  const signed char* sg = sgl + p * kMaxPivot;

  // 1. A_P = sum of the chunk partials (upper tiles), mirrored
  const double* P = part + (size_t)p * nch * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && (r >> 4) <= (c >> 4)) {
      double s = 0.0;
      for (int k = 0; k < nch; k++) s += P[(size_t)k * (kMaxPivot * kMaxPivot) + e];
      R[c * LDR + r] = s;
    }
  }
  if (tid == 0) {
    s_bad = 0;
    s_total = 0;
    s_sweeps = 0;
  }
  __syncthreads();
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r > c) R[c * LDR + r] = R[r * LDR + c];
  }
  __syncthreads();

  // 2. convergence test on the scaled off-diagonal, and zero / non-finite diagonal
  double off = 0.0;
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r < c) {
      double v = fabs(R[c * LDR + r]) / (sqrt(R[r * LDR + r]) * sqrt(R[c * LDR + c]));
      off = fmax(off, v);
    }
  }
  for (int k = tid; k < m; k += 256) {
    double d = R[k * LDR + k];
    if (!(d > 0.0) || !isfinite(d)) atomicOr(&s_bad, 1);
  }
  redv[tid] = off;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) redv[tid] = fmax(redv[tid], redv[tid + s]);
    __syncthreads();
  }
  off = redv[0];
  if (tid == 0) atomic_max_nonneg(&st->max_off_bits, isfinite(off) ? off : 1.0e300);
  if (s_bad) {
    if (tid == 0) {
      rotflag[p] = 0;
      atomicOr(&st->breakdown, 1);
    }
    return;
  }
  if (off <= tol) {
    if (tid == 0) rotflag[p] = 0;
    return;
  }

  // 3. Cholesky A_P = R^T R (upper R), right-looking
  for (int k = 0; k < m; k++) {
    if (tid == 0) {
      double d = R[k * LDR + k];
      if (d > 0.0 && isfinite(d)) {
        s_piv = sqrt(d);
      } else {
        s_piv = 0.0;
        s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const double piv = s_piv;
    for (int c = k + 1 + tid; c < m; c += 256) R[c * LDR + k] /= piv;
    if (tid == 0) R[k * LDR + k] = piv;
    __syncthreads();
    const int L = m - k - 1;
    for (int e = tid; e < L * L; e += 256) {
      int r = k + 1 + e / L, c = k + 1 + e % L;
      if (r <= c) R[c * LDR + r] -= R[r * LDR + k] * R[c * LDR + k];
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) {
      rotflag[p] = 0;
      atomicOr(&st->breakdown, 1);
    }
    return;
  }
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m) {
      if (r > c) R[c * LDR + r] = 0.0;
      W[c * LDR + r] = (r == c) ? 1.0 : 0.0;
    }
  }
  __syncthreads();

  // 4. inner one-sided J-Jacobi on the columns of R, accumulating W_P
  const int slot = tid >> 3, sub = tid & 7;
  const int mp = m + (m & 1);
  const int n1 = nfirst[p], n2 = m - n1;
  const int L = max(n1, n2);
  const int nsweeps = inner_mode == 0 ? inner_max : 1;
  const int nrounds = inner_mode == 0 ? mp - 1 : L;
  for (int it = 0; it < nsweeps; it++) {
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for (int q = 0; q < nrounds; q++) {
      int r = -1, s = -1;
      if (inner_mode == 0) {
        if (slot < mp / 2) {
          int a = slot == 0 ? 0 : ((slot - 1 + q) % (mp - 1)) + 1;
          int b = ((mp - 1 - slot - 1 + q) % (mp - 1)) + 1;
          r = min(a, b);
          s = max(a, b);
        }
      } else if (slot < L) {
        int k2 = (slot + q) % L;
        if (slot < n1 && k2 < n2) {
          r = slot;
          s = n1 + k2;
        }
      }
      if (r >= 0 && s < m) {
        double* Rr = R + r * LDR;
        double* Rs = R + s * LDR;
        double arr = 0.0, ass = 0.0, ars = 0.0;
        for (int i = sub; i < m; i += 8) {
          double x = Rr[i], y = Rs[i];
          arr += x * x;
          ass += y * y;
          ars += x * y;
        }
#pragma unroll
        for (int msk = 1; msk < 8; msk <<= 1) {
          arr += __shfl_xor(arr, msk);
          ass += __shfl_xor(ass, msk);
          ars += __shfl_xor(ars, msk);
        }
        double sigma = (double)(sg[r] * sg[s]);
        double cs = 1.0, sn = 0.0;
        int rc = rot_params(arr, ass, ars, sigma, tol, &cs, &sn);
        if (rc > 0) {
          double* Wr = W + r * LDR;
          double* Ws = W + s * LDR;
          for (int i = sub; i < m; i += 8) {
            double x = Rr[i], y = Rs[i];
            Rr[i] = cs * x - sigma * sn * y;
            Rs[i] = sn * x + cs * y;
            double u = Wr[i], w = Ws[i];
            Wr[i] = cs * u - sigma * sn * w;
            Ws[i] = sn * u + cs * w;
          }
          if (sub == 0) atomicAdd(&s_cnt, 1);
        } else if (rc < 0 && sub == 0) {
          atomicOr(&s_bad, 1);
        }
      }
      __syncthreads();
    }
    const int cnt = s_cnt;
    if (tid == 0) {
      s_total += cnt;
      s_sweeps++;
    }
    __syncthreads();
    if (cnt == 0) break;
  }
  if (tid == 0) {
    atomicAdd(&st->rotations, (unsigned long long)s_total);
    atomicAdd(&st->inner_sweeps, (unsigned long long)s_sweeps);
    atomicAdd(&st->pivot_cols, (unsigned long long)m);
    atomicAdd(&st->pivot_cols3, (unsigned long long)m * m * m);
  }
  if (s_bad && tid == 0) atomicOr(&st->breakdown, 1);

  // 5. W_P out
  const int rotated = s_total > 0;
  if (rotated) {
    double* Wo = Wout + (size_t)p * (kMaxPivot * kMaxPivot);
    for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
      int c = e >> 6, r = e & 63;
      if (r < m && c < m) Wo[c * kMaxPivot + r] = W[c * LDR + r];
    }
  }
  if (tid == 0) {
    rotflag[p] = rotated;
    if (rotated) atomicAdd(&st->pivots_rotated, 1);
  }
}

// ---------------------------------------------------------------------------
// Update [G_i G_j] <- [G_i G_j] W_P in place.  Grid (nch, P), 256 threads.
// Computed transposed, D^T = W_P^T X^T, so that each lane's results are
// consecutive rows of one column (coalesced stores).  A wave loads its whole
// 16-row strip (all m columns) before writing any of it.
// ---------------------------------------------------------------------------
constexpr int LDW = kMaxPivot + 1;

__global__ __launch_bounds__(256) void k_update_f64(double* __restrict__ G, int ldg, int n,
                                                    const int* __restrict__ cols, const int* __restrict__ mlist,
                                                    const double* __restrict__ Wg, const int* __restrict__ rotflag,
                                                    int rows_per_chunk) {
  const int p = blockIdx.y, ch = blockIdx.x;
  if (!rotflag[p]) return;
  __shared__ double Ws[kMaxPivot * LDW];
  __shared__ int scol[kMaxPivot];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;   // output column tiles
  const int ks = (m + 3) >> 2;    // k-steps of 4 columns
  const double* Wp = Wg + (size_t)p * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int c = e >> 6, r = e & 63;
    Ws[c * LDW + r] = (r < m && c < m) ? Wp[c * kMaxPivot + r] : 0.0;
  }
  if (tid < kMaxPivot) scol[tid] = (tid < m) ? cols[p * kMaxPivot + tid] : -1;
  __syncthreads();

  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  for (int row0 = r0 + wave * 16; row0 < r1; row0 += 64) {
    const int row = row0 + c16;
    double x[16];
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      int c = 4 * kk + g;
      int pc = scol[c];
      x[kk] = (kk < ks && pc >= 0 && row < r1) ? G[(size_t)pc * ldg + row] : 0.0;
    }
#pragma unroll
    for (int I = 0; I < 4; I++) {
      if (I < nt) {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk++)
          if (kk < ks) acc = mfma16(Ws[(16 * I + c16) * LDW + 4 * kk + g], x[kk], acc);
#pragma unroll
        for (int v = 0; v < 4; v++) {
          int oc = 16 * I + 4 * v + g;
          int pc = scol[oc];
          if (oc < m && row < r1) G[(size_t)pc * ldg + row] = acc[v];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Complex Hermitian (complex128, interleaved).  A = X^H X is formed from real
// MFMA products: Re A = Xr^T Xr + Xi^T Xi, Im A = Xr^T Xi - Xi^T Xr.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gram_c128(const double* __restrict__ G, int ldg, int n,
                                                   const int* __restrict__ cols, const int* __restrict__ mlist,
                                                   int rows_per_chunk, double* __restrict__ part) {
  __shared__ d4 red[10][2][64];
  const int p = blockIdx.y, ch = blockIdx.x, nch = gridDim.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const double2* cp[4];
#pragma unroll
  for (int J = 0; J < 4; J++) {
    int c = J * 16 + c16;
    int pc = (c < m) ? cols[p * kMaxPivot + c] : -1;
    cp[J] = (pc >= 0) ? reinterpret_cast<const double2*>(G) + (size_t)pc * ldg : nullptr;
  }
  d4 are[10], aim[10];
#pragma unroll
  for (int t = 0; t < 10; t++) {
    are[t] = d4{0.0, 0.0, 0.0, 0.0};
    aim[t] = d4{0.0, 0.0, 0.0, 0.0};
  }
  for (int base = r0 + wave * 16; base < r1; base += 64) {
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      const int row = base + 4 * g + kk;
      double xr[4], xi[4];
#pragma unroll
      for (int J = 0; J < 4; J++) {
        double2 v = (cp[J] != nullptr && row < r1) ? cp[J][row] : double2{0.0, 0.0};
        xr[J] = v.x;
        xi[J] = v.y;
      }
      int t = 0;
#pragma unroll
      for (int I = 0; I < 4; I++)
#pragma unroll
        for (int J = I; J < 4; J++) {
          if (J < nt) {
            are[t] = mfma16(xr[I], xr[J], are[t]);
            are[t] = mfma16(xi[I], xi[J], are[t]);
            aim[t] = mfma16(xr[I], xi[J], aim[t]);
            aim[t] = mfma16(-xi[I], xr[J], aim[t]);
          }
          t++;
        }
    }
  }
  // fixed-order reduction: ((w3 + w2) + w1) + w0
  for (int w = 3; w >= 1; w--) {
    if (wave == w)
      for (int t = 0; t < 10; t++) {
        red[t][0][lane] = are[t];
        red[t][1][lane] = aim[t];
      }
    __syncthreads();
    if (wave == w - 1)
      for (int t = 0; t < 10; t++) {
        are[t] = red[t][0][lane] + are[t];
        aim[t] = red[t][1][lane] + aim[t];
      }
    __syncthreads();
  }
  if (wave == 0) {
    double* out = part + ((size_t)p * nch + ch) * (2 * kMaxPivot * kMaxPivot);
    int t = 0;
#pragma unroll
    for (int I = 0; I < 4; I++)
#pragma unroll
      for (int J = I; J < 4; J++) {
        if (J < nt) {
#pragma unroll
          for (int v = 0; v < 4; v++) {
            size_t e = (size_t)(16 * I + 4 * v + g) * kMaxPivot + 16 * J + c16;
            out[2 * e] = are[t][v];
            out[2 * e + 1] = aim[t][v];
          }
        }
        t++;
      }
  }
}

// Pivot solve, complex.  R and W_P in LDS as interleaved complex, leading
// dimension 65.  The rotation carries the phase e^{i alpha} = a_rs / eta on
// column r (the modified rotation of eq. 2.3 used by Algorithm 3.1).
__global__ __launch_bounds__(256) void k_pivot_c128(const double* __restrict__ part, int nch,
                                                    const int* __restrict__ mlist, const int* __restrict__ nfirst,
                                                    const signed char* __restrict__ sgl, double tol, int inner_max,
                                                    int inner_mode, double* __restrict__ Wout,
                                                    int* __restrict__ rotflag, SweepStats* st) {
  __shared__ double2 R[kMaxPivot * LDR];
  __shared__ double2 W[kMaxPivot * LDR];
  __shared__ double redv[256];
  __shared__ int s_cnt, s_bad, s_total, s_sweeps;
  __shared__ double s_piv;
  const int p = blockIdx.x, tid = threadIdx.x;
  const int m = mlist[p];
  const signed char* sg = sgl + p * kMaxPivot;

  const double2* P = reinterpret_cast<const double2*>(part) + (size_t)p * nch * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && (r >> 4) <= (c >> 4)) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < nch; k++) {
        double2 v = P[(size_t)k * (kMaxPivot * kMaxPivot) + e];
        sr += v.x;
        si += v.y;
      }
      R[c * LDR + r] = double2{sr, si};
    }
  }
  if (tid == 0) {
    s_bad = 0;
    s_total = 0;
    s_sweeps = 0;
  }
  __syncthreads();
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r > c) {
      double2 u = R[r * LDR + c];
      R[c * LDR + r] = double2{u.x, -u.y};
    }
  }
  __syncthreads();
  // the diagonal of a Hermitian matrix is real
  for (int k = tid; k < m; k += 256) R[k * LDR + k].y = 0.0;
  __syncthreads();

  double off = 0.0;
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r < c) {
      double2 a = R[c * LDR + r];
      double v = hypot(a.x, a.y) / (sqrt(R[r * LDR + r].x) * sqrt(R[c * LDR + c].x));
      off = fmax(off, v);
    }
  }
  for (int k = tid; k < m; k += 256) {
    double d = R[k * LDR + k].x;
    if (!(d > 0.0) || !isfinite(d)) atomicOr(&s_bad, 1);
  }
  redv[tid] = off;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) redv[tid] = fmax(redv[tid], redv[tid + s]);
    __syncthreads();
  }
  off = redv[0];
  if (tid == 0) atomic_max_nonneg(&st->max_off_bits, isfinite(off) ? off : 1.0e300);
  if (s_bad) {
    if (tid == 0) {
      rotflag[p] = 0;
      atomicOr(&st->breakdown, 1);
    }
    return;
  }
  if (off <= tol) {
    if (tid == 0) rotflag[p] = 0;
    return;
  }

  // Cholesky A_P = R^H R
  for (int k = 0; k < m; k++) {
    if (tid == 0) {
      double d = R[k * LDR + k].x;
      if (d > 0.0 && isfinite(d)) {
        s_piv = sqrt(d);
      } else {
        s_piv = 0.0;
        s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const double piv = s_piv;
    for (int c = k + 1 + tid; c < m; c += 256) {
      double2 a = R[c * LDR + k];
      R[c * LDR + k] = double2{a.x / piv, a.y / piv};
    }
    if (tid == 0) R[k * LDR + k] = double2{piv, 0.0};
    __syncthreads();
    const int L = m - k - 1;
    for (int e = tid; e < L * L; e += 256) {
      int r = k + 1 + e / L, c = k + 1 + e % L;
      if (r <= c) {
        double2 u = R[r * LDR + k], v = R[c * LDR + k], a = R[c * LDR + r];
        // a -= conj(u) v
        a.x -= u.x * v.x + u.y * v.y;
        a.y -= u.x * v.y - u.y * v.x;
        R[c * LDR + r] = a;
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) {
      rotflag[p] = 0;
      atomicOr(&st->breakdown, 1);
    }
    return;
  }
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m) {
      if (r > c) R[c * LDR + r] = double2{0.0, 0.0};
      W[c * LDR + r] = double2{(r == c) ? 1.0 : 0.0, 0.0};
    }
  }
  __syncthreads();

  const int slot = tid >> 3, sub = tid & 7;
  const int mp = m + (m & 1);
  const int n1 = nfirst[p], n2 = m - n1;
  const int L = max(n1, n2);
  const int nsweeps = inner_mode == 0 ? inner_max : 1;
  const int nrounds = inner_mode == 0 ? mp - 1 : L;
  for (int it = 0; it < nsweeps; it++) {
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for (int q = 0; q < nrounds; q++) {
      int r = -1, s = -1;
      if (inner_mode == 0) {
        if (slot < mp / 2) {
          int a = slot == 0 ? 0 : ((slot - 1 + q) % (mp - 1)) + 1;
          int b = ((mp - 1 - slot - 1 + q) % (mp - 1)) + 1;
          r = min(a, b);
          s = max(a, b);
        }
      } else if (slot < L) {
        int k2 = (slot + q) % L;
        if (slot < n1 && k2 < n2) {
          r = slot;
          s = n1 + k2;
        }
      }
      if (r >= 0 && s < m) {
        double2* Rr = R + r * LDR;
        double2* Rs = R + s * LDR;
        double arr = 0.0, ass = 0.0, are = 0.0, aim = 0.0;
        for (int i = sub; i < m; i += 8) {
          double2 x = Rr[i], y = Rs[i];
          arr += x.x * x.x + x.y * x.y;
          ass += y.x * y.x + y.y * y.y;
          are += x.x * y.x + x.y * y.y;  // conj(x) y
          aim += x.x * y.y - x.y * y.x;
        }
#pragma unroll
        for (int msk = 1; msk < 8; msk <<= 1) {
          arr += __shfl_xor(arr, msk);
          ass += __shfl_xor(ass, msk);
          are += __shfl_xor(are, msk);
          aim += __shfl_xor(aim, msk);
        }
        const double sigma = (double)(sg[r] * sg[s]);
        const double aabs = hypot(are, aim);
        // eta = sgn(Re a_rs) |a_rs| is real; the 2x2 problem on [e^{ia} g_r, g_s] is real
        const double eta = (are < 0.0 ? -1.0 : 1.0) * aabs;
        double cs = 1.0, sn = 0.0;
        int rc = rot_params(arr, ass, eta, sigma, tol, &cs, &sn);
        if (rc > 0) {
          const double pr = are / eta, pi = aim / eta;  // e^{i alpha}
          double2* Wr = W + r * LDR;
          double2* Ws = W + s * LDR;
          for (int i = sub; i < m; i += 8) {
            double2 x = Rr[i], y = Rs[i];
            double fr = pr * x.x - pi * x.y, fi = pr * x.y + pi * x.x;
            Rr[i] = double2{cs * fr - sigma * sn * y.x, cs * fi - sigma * sn * y.y};
            Rs[i] = double2{sn * fr + cs * y.x, sn * fi + cs * y.y};
            double2 u = Wr[i], w = Ws[i];
            double gr = pr * u.x - pi * u.y, gi = pr * u.y + pi * u.x;
            Wr[i] = double2{cs * gr - sigma * sn * w.x, cs * gi - sigma * sn * w.y};
            Ws[i] = double2{sn * gr + cs * w.x, sn * gi + cs * w.y};
          }
          if (sub == 0) atomicAdd(&s_cnt, 1);
        } else if (rc < 0 && sub == 0) {
          atomicOr(&s_bad, 1);
        }
      }
      __syncthreads();
    }
    const int cnt = s_cnt;
    if (tid == 0) {
      s_total += cnt;
      s_sweeps++;
    }
    __syncthreads();
    if (cnt == 0) break;
  }
  if (tid == 0) {
    atomicAdd(&st->rotations, (unsigned long long)s_total);
    atomicAdd(&st->inner_sweeps, (unsigned long long)s_sweeps);
    atomicAdd(&st->pivot_cols, (unsigned long long)m);
    atomicAdd(&st->pivot_cols3, (unsigned long long)m * m * m);
  }
  if (s_bad && tid == 0) atomicOr(&st->breakdown, 1);
  const int rotated = s_total > 0;
  if (rotated) {
    double2* Wo = reinterpret_cast<double2*>(Wout) + (size_t)p * (kMaxPivot * kMaxPivot);
    for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
      int c = e >> 6, r = e & 63;
      if (r < m && c < m) Wo[c * kMaxPivot + r] = W[c * LDR + r];
    }
  }
  if (tid == 0) {
    rotflag[p] = rotated;
    if (rotated) atomicAdd(&st->pivots_rotated, 1);
  }
}

// Update, complex: D^T = W^T X^T with Re = Wr^T Xr^T - Wi^T Xi^T and
// Im = Wi^T Xr^T + Wr^T Xi^T.
__global__ __launch_bounds__(256) void k_update_c128(double* __restrict__ G, int ldg, int n,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     const double* __restrict__ Wg, const int* __restrict__ rotflag,
                                                     int rows_per_chunk) {
  const int p = blockIdx.y, ch = blockIdx.x;
  if (!rotflag[p]) return;
  __shared__ double2 Ws[kMaxPivot * LDW];
  __shared__ int scol[kMaxPivot];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int ks = (m + 3) >> 2;
  const double2* Wp = reinterpret_cast<const double2*>(Wg) + (size_t)p * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int c = e >> 6, r = e & 63;
    Ws[c * LDW + r] = (r < m && c < m) ? Wp[c * kMaxPivot + r] : double2{0.0, 0.0};
  }
  if (tid < kMaxPivot) scol[tid] = (tid < m) ? cols[p * kMaxPivot + tid] : -1;
  __syncthreads();
  double2* Gc = reinterpret_cast<double2*>(G);
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  for (int row0 = r0 + wave * 16; row0 < r1; row0 += 64) {
    const int row = row0 + c16;
    double xr[16], xi[16];
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      int pc = scol[4 * kk + g];
      double2 v = (kk < ks && pc >= 0 && row < r1) ? Gc[(size_t)pc * ldg + row] : double2{0.0, 0.0};
      xr[kk] = v.x;
      xi[kk] = v.y;
    }
#pragma unroll
    for (int I = 0; I < 4; I++) {
      if (I < nt) {
        d4 ar = d4{0.0, 0.0, 0.0, 0.0}, ai = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk++)
          if (kk < ks) {
            double2 w = Ws[(16 * I + c16) * LDW + 4 * kk + g];
            ar = mfma16(w.x, xr[kk], ar);
            ar = mfma16(-w.y, xi[kk], ar);
            ai = mfma16(w.y, xr[kk], ai);
            ai = mfma16(w.x, xi[kk], ai);
          }
#pragma unroll
        for (int v = 0; v < 4; v++) {
          int oc = 16 * I + 4 * v + g;
          int pc = scol[oc];
          if (oc < m && row < r1) Gc[(size_t)pc * ldg + row] = double2{ar[v], ai[v]};
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small kernels: stats reset, non-finite scan, finalisation.
// ---------------------------------------------------------------------------
__global__ void k_reset_stats(SweepStats* st) {
  if (threadIdx.x == 0) {
    st->max_off_bits = 0ull;
    st->pivots_rotated = 0;
    st->breakdown = 0;
    st->nonfinite = 0;
    st->zero_col = 0;
    st->rotations = 0ull;
    st->inner_sweeps = 0ull;
    st->pivot_cols = 0ull;
    st->pivot_cols3 = 0ull;
  }
}

__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ G, int ldg, int n, int w,
                                                      SweepStats* st) {
  const int col = blockIdx.x;
  const double* c = G + (size_t)col * ldg * w;
  int bad = 0;
  for (int i = threadIdx.x; i < n * w; i += 256) bad |= !isfinite(c[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1);
}

// d[q] = ||G[:, colmap[q]]||^2 ; one block per column, fixed-order tree reduction
__global__ __launch_bounds__(256) void k_colnorm(const double* __restrict__ G, int ldg, int n, int w,
                                                 const int* __restrict__ colmap, double* __restrict__ d) {
  __shared__ double red[256];
  const int q = blockIdx.x, tid = threadIdx.x;
  const double* c = G + (size_t)colmap[q] * ldg * w;
  double s = 0.0;
  for (int i = tid; i < n * w; i += 256) s += c[i] * c[i];
  red[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0) d[q] = red[0];
}

// rank[q] = #{q' : lam[q'] > lam[q] or (lam[q'] == lam[q] and colmap[q'] < colmap[q])}
__global__ __launch_bounds__(256) void k_rank(int n, const double* __restrict__ d, const signed char* __restrict__ sgn,
                                              const int* __restrict__ colmap, int* __restrict__ rank,
                                              double* __restrict__ lambda, SweepStats* st) {
  __shared__ double sl[256];
  __shared__ int sc[256];
  const int q = blockIdx.x * 256 + threadIdx.x;
  const double lq = q < n ? (double)sgn[q] * d[q] : 0.0;
  const int cq = q < n ? colmap[q] : 0;
  int rk = 0;
  for (int b = 0; b < n; b += 256) {
    int k = b + threadIdx.x;
    sl[threadIdx.x] = k < n ? (double)sgn[k] * d[k] : 0.0;
    sc[threadIdx.x] = k < n ? colmap[k] : 0;
    __syncthreads();
    const int lim = min(256, n - b);
    for (int j = 0; j < lim; j++) rk += (sl[j] > lq) || (sl[j] == lq && sc[j] < cq);
    __syncthreads();
  }
  if (q < n) {
    rank[q] = rk;
    lambda[rk] = lq;
    if (!(d[q] > 0.0)) atomicOr(&st->zero_col, 1);
  }
}

// V[:, rank[q]] = G[:, colmap[q]] / sqrt(d[q]) ; one block per column
__global__ __launch_bounds__(256) void k_write_v(const double* __restrict__ G, int ldg, int n, int w,
                                                 const int* __restrict__ colmap, const double* __restrict__ d,
                                                 const int* __restrict__ rank, double* __restrict__ V, int ldv) {
  const int q = blockIdx.x;
  const double* c = G + (size_t)colmap[q] * ldg * w;
  double* o = V + (size_t)rank[q] * ldv * w;
  const double dq = d[q];
  const double inv = dq > 0.0 ? 1.0 / sqrt(dq) : 0.0;
  for (int i = threadIdx.x; i < n * w; i += 256) o[i] = c[i] * inv;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_gram_f64(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_gram_f64, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part);
}

void launch_pivot_f64(const double* part, int nch, const PivotList& pl, double tol, int inner_max,
                      int inner_mode, double* W, int* rotflag, SweepStats* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_pivot_f64, dim3(pl.count), dim3(256), 0, stream, part, nch, pl.m, pl.nfirst, pl.sg, tol,
                     inner_max, inner_mode, W, rotflag, st);
}

void launch_update_f64(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                       int rows_per_chunk, hipStream_t stream) {
  int nch = (n + rows_per_chunk - 1) / rows_per_chunk;
  hipLaunchKernelGGL(k_update_f64, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, W,
                     rotflag, rows_per_chunk);
}

void launch_gram_c128(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                      double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_gram_c128, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part);
}

void launch_pivot_c128(const double* part, int nch, const PivotList& pl, double tol, int inner_max,
                       int inner_mode, double* W, int* rotflag, SweepStats* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_pivot_c128, dim3(pl.count), dim3(256), 0, stream, part, nch, pl.m, pl.nfirst, pl.sg, tol,
                     inner_max, inner_mode, W, rotflag, st);
}

void launch_update_c128(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                        int rows_per_chunk, hipStream_t stream) {
  int nch = (n + rows_per_chunk - 1) / rows_per_chunk;
  hipLaunchKernelGGL(k_update_c128, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, W,
                     rotflag, rows_per_chunk);
}

void launch_reset_stats(SweepStats* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, stream, st);
}

void launch_check_finite(const double* G, int ldg, int n, int cplx, SweepStats* st, hipStream_t stream) {
  hipLaunchKernelGGL(k_check_finite, dim3(n), dim3(256), 0, stream, G, ldg, n, cplx ? 2 : 1, st);
}

void launch_finalize(const double* G, int ldg, int n, int cplx, const int* colmap, const signed char* sgn,
                     double* d, int* rank, double* lambda, double* V, int ldv, SweepStats* st,
                     hipStream_t stream) {
  const int w = cplx ? 2 : 1;
  hipLaunchKernelGGL(k_colnorm, dim3(n), dim3(256), 0, stream, G, ldg, n, w, colmap, d);
  hipLaunchKernelGGL(k_rank, dim3((n + 255) / 256), dim3(256), 0, stream, n, d, sgn, colmap, rank, lambda, st);
  hipLaunchKernelGGL(k_write_v, dim3(n), dim3(256), 0, stream, G, ldg, n, w, colmap, d, rank, V, ldv);
}

}  // namespace jj
