// Device-side bookkeeping for batched solves: every problem of a batch walks
// through its own block steps and sweeps; these kernels advance the per-problem
// state after each step, scan inputs for non-finite values and finalise the
// eigenpairs (lambda_i = j_i ||g_i||^2, v_i = g_i / ||g_i||, eq. 2.10), one
// workgroup per problem.
#include "jj_device.h"

#include <math.h>

namespace jj {

// After a step: next step of the problem's sweep, or end of the sweep with the
// convergence test of Section 5.3 (a sweep in which no pivot rotated).  A
// problem in mixed sweeps never converges in one: it leaves FP32 after a sweep
// whose largest scaled off-diagonal is below mix_switch, after a sweep with no
// rotation, or after a sweep in which an FP32 Gram block could not be factored.
__global__ void k_batch_advance(int count, const int* __restrict__ nsteps, int* __restrict__ step,
                                int* __restrict__ sweep, int* __restrict__ active, int* __restrict__ status,
                                SweepStats* __restrict__ st, double* __restrict__ final_off, int max_sweeps,
                                int* __restrict__ active_count, int* __restrict__ prec,
                                int* __restrict__ mixed_sweeps, double mix_switch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || !active[i]) return;
  const int t = step[i] + 1;
  if (t < nsteps[i]) {
    step[i] = t;
    return;
  }
  const int s = sweep[i] + 1;
  sweep[i] = s;
  SweepStats& c = st[i];
  const double off = __longlong_as_double((long long)c.max_off_bits);
  final_off[i] = off;
  int done = 0, code = 0;
  if (c.breakdown) {
    done = 1;
    code = 2;
  } else if (prec != nullptr && prec[i]) {
    mixed_sweeps[i] += 1;
    if (off < mix_switch || c.pivots_rotated == 0 || c.soft_fail) prec[i] = 0;
    if (s >= max_sweeps) {
      done = 1;
      code = 1;
    }
  } else if (c.pivots_rotated == 0) {
    done = 1;
    code = 0;
  } else if (s >= max_sweeps) {
    done = 1;
    code = 1;
  }
  if (done) {
    active[i] = 0;
    status[i] = code;
    atomicSub(active_count, 1);
  } else {
    step[i] = 0;
    c.max_off_bits = 0ull;
    c.pivots_rotated = 0;
    c.breakdown = 0;
    c.soft_fail = 0;
  }
}

// One workgroup per problem: flag non-finite entries of G.
__global__ __launch_bounds__(256) void k_batch_check_finite(double* const* __restrict__ gptr,
                                                            const int* __restrict__ ldg, const int* __restrict__ nrow,
                                                            const int* __restrict__ width, int* __restrict__ bad) {
  const int i = blockIdx.x;
  const int n = nrow[i], w = width[i];
  const double* G = gptr[i];
  int b = 0;
  for (int c = 0; c < n; c++)
    for (int r = threadIdx.x; r < n * w; r += 256) b |= !isfinite(G[(size_t)c * ldg[i] * w + r]);
  if (__any(b) && (threadIdx.x & 63) == 0) atomicOr(&bad[i], 1);
}

// One workgroup per problem: column norms (one wave per column, fixed-order
// reduction), ranks by (lambda descending, input column ascending), then
// lambda and V in rank order.
__global__ __launch_bounds__(256) void k_batch_finalize(double* const* __restrict__ gptr, const int* __restrict__ ldg,
                                                        const int* __restrict__ nrow, const int* __restrict__ width,
                                                        const int* __restrict__ colmap, const int* __restrict__ cm_off,
                                                        const signed char* __restrict__ sgn,
                                                        double* const* __restrict__ lam_ptr,
                                                        double* const* __restrict__ v_ptr, const int* __restrict__ ldv,
                                                        double* __restrict__ dwork, int* __restrict__ rkwork,
                                                        int* __restrict__ zero_col) {
  const int i = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = nrow[i], w = width[i];
  const double* G = gptr[i];
  const int* cm = colmap + cm_off[i];
  const signed char* sg = sgn + cm_off[i];
  double* d = dwork + cm_off[i];
  int* rk = rkwork + cm_off[i];
  for (int q = wave; q < n; q += 4) {
    const double* col = G + (size_t)cm[q] * ldg[i] * w;
    double s = 0.0;
    for (int r = lane; r < n * w; r += 64) s += col[r] * col[r];
#pragma unroll
    for (int msk = 32; msk > 0; msk >>= 1) s += __shfl_xor(s, msk);
    if (lane == 0) d[q] = s;
  }
  __syncthreads();
  double* lam = lam_ptr[i];
  int zc = 0;
  for (int q = tid; q < n; q += 256) {
    const double lq = (double)sg[q] * d[q];
    const int cq = cm[q];
    int r = 0;
    for (int j = 0; j < n; j++) {
      const double lj = (double)sg[j] * d[j];
      r += (lj > lq) || (lj == lq && cm[j] < cq);
    }
    rk[q] = r;
    lam[r] = lq;
    zc |= !(d[q] > 0.0);
  }
  if (zc) atomicOr(&zero_col[i], 1);
  __syncthreads();
  double* V = v_ptr[i];
  for (int q = wave; q < n; q += 4) {
    const double* col = G + (size_t)cm[q] * ldg[i] * w;
    double* out = V + (size_t)rk[q] * ldv[i] * w;
    const double inv = d[q] > 0.0 ? 1.0 / sqrt(d[q]) : 0.0;
    for (int r = lane; r < n * w; r += 64) out[r] = col[r] * inv;
  }
}

void launch_batch_advance(int count, const int* nsteps, int* step, int* sweep, int* active, int* status,
                          SweepStats* st, double* final_off, int max_sweeps, int* active_count, int* prec,
                          int* mixed_sweeps, double mix_switch, hipStream_t stream) {
  launch(k_batch_advance, dim3((count + 255) / 256), dim3(256), 0, stream, count, nsteps, step, sweep, active,
         status, st, final_off, max_sweeps, active_count, prec, mixed_sweeps, mix_switch);
}

void launch_batch_check_finite(int count, double* const* gptr, const int* ldg, const int* nrow, const int* width,
                               int* bad, hipStream_t stream) {
  launch(k_batch_check_finite, dim3(count), dim3(256), 0, stream, gptr, ldg, nrow, width, bad);
}

void launch_batch_finalize(int count, double* const* gptr, const int* ldg, const int* nrow, const int* width,
                           const int* colmap, const int* cm_off, const signed char* sgn, double* const* lam_ptr,
                           double* const* v_ptr, const int* ldv, double* dwork, int* rkwork, int* zero_col,
                           hipStream_t stream) {
  launch(k_batch_finalize, dim3(count), dim3(256), 0, stream, gptr, ldg, nrow, width, colmap, cm_off, sgn,
                     lam_ptr, v_ptr, ldv, dwork, rkwork, zero_col);
}

}  // namespace jj
