// Pivot-block solver (paper, Section 5.3 steps 2-3): for each pair of
// block-columns, from the Gram block A_P (eq. 3.6):
//   1. convergence test on the scaled off-diagonal |a_rs| / sqrt(a_rr a_ss);
//   2. Cholesky A_P = R^* R (eq. 3.8);
//   3. one-sided J-Jacobi on the columns of R, accumulating W_P (eq. 3.12,
//      Algorithms 3.1/3.2): R <- R W_P, W_P <- W_P W, one J-unitary plane
//      rotation per column pair (trigonometric for equal signs, hyperbolic
//      for opposite signs), with the phase of eq. 2.3 in the complex case.
//
// Inner ordering.  An inner sweep visits every column pair of the pivot once:
//   (a) within each of the two blocks: circle round-robin, R and W_P in LDS;
//   (b) across the blocks: slot k keeps column k of the first block in
//       registers for the whole pass while the columns of the second block
//       move between slots: for two equal power-of-two blocks by the XOR
//       schedule (slot k meets second-block column k ^ gray(q) in round q;
//       moves by DPP or lane permutes within a wavefront, through LDS for the
//       3 of 31 moves that cross wavefronts), otherwise through an LDS ring
//       (slot k meets second-block column (k + q) mod L in round q).
// Block-oriented steps (Section 3.4 / Algorithm 5.1) run (b) once; full
// diagonalisation repeats (a)+(b) until an inner sweep applies no rotation.
#include "jj_device.h"

#include <math.h>

namespace jj {

constexpr int LDR = kMaxPivot + 1;

// ---- scalar helpers: real (double) and complex (double2) ----
__device__ __forceinline__ double zero_of(double) { return 0.0; }
__device__ __forceinline__ double2 zero_of(double2) { return double2{0.0, 0.0}; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(double2 a) { return a.x * a.x + a.y * a.y; }
// accumulate conj(a) b
__device__ __forceinline__ void cdot(double a, double b, double& re, double& im) { re += a * b; }
__device__ __forceinline__ void cdot(double2 a, double2 b, double& re, double& im) {
  re += a.x * b.x + a.y * b.y;
  im += a.x * b.y - a.y * b.x;
}
// (pr + i pi) * x ; the real case has phase 1
__device__ __forceinline__ double phase_mul(double pr, double pi, double x) { return x; }
__device__ __forceinline__ double2 phase_mul(double pr, double pi, double2 x) {
  return double2{pr * x.x - pi * x.y, pr * x.y + pi * x.x};
}
__device__ __forceinline__ double lin2(double a, double x, double b, double y) { return a * x + b * y; }
__device__ __forceinline__ double2 lin2(double a, double2 x, double b, double2 y) {
  return double2{a * x.x + b * y.x, a * x.y + b * y.y};
}
// a - conj(u) v * dinv
__device__ __forceinline__ double schur(double a, double u, double v, double dinv) { return a - (u * dinv) * v; }
__device__ __forceinline__ double2 schur(double2 a, double2 u, double2 v, double dinv) {
  const double ur = u.x * dinv, ui = u.y * dinv;
  return double2{a.x - (ur * v.x + ui * v.y), a.y - (ur * v.y - ui * v.x)};
}
// f x (plain product; the conjugation is folded into f by the caller)
__device__ __forceinline__ double cmul_conj_first(double f, double x) { return f * x; }
__device__ __forceinline__ double2 cmul_conj_first(double2 f, double2 x) {
  return double2{f.x * x.x - f.y * x.y, f.x * x.y + f.y * x.x};
}
__device__ __forceinline__ double one_like(double) { return 1.0; }
__device__ __forceinline__ double2 one_like(double2) { return double2{1.0, 0.0}; }
__device__ __forceinline__ double scale(double a, double s) { return a * s; }
__device__ __forceinline__ double2 scale(double2 a, double s) { return double2{a.x * s, a.y * s}; }
__device__ __forceinline__ double conj_of(double a) { return a; }
__device__ __forceinline__ double2 conj_of(double2 a) { return double2{a.x, -a.y}; }
__device__ __forceinline__ double real_of(double a) { return a; }
__device__ __forceinline__ double real_of(double2 a) { return a.x; }
__device__ __forceinline__ bool finite_of(double a) { return isfinite(a); }
__device__ __forceinline__ bool finite_of(double2 a) { return isfinite(a.x) && isfinite(a.y); }

template <bool C>
struct Scalar;
template <>
struct Scalar<false> {
  typedef double T;
};
template <>
struct Scalar<true> {
  typedef double2 T;
};

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// Order LDS accesses among the lanes of one wavefront (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reciprocal and reciprocal square root from the hardware estimates (about
// 2^-23 relative) refined by two Newton steps each, r <- r + r (1 - x r) and
// y <- y + (y/2)(1 - x y^2), which leaves an error of about one unit in the last
// place with no preferred direction.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; it++) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; it++) y = fma(0.5 * y, fma(-(d * y), y, 1.0), y);
  return y;
}
// sqrt(x) for x >= 0 (exact zero for zero), without a branch
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = x * rsqrt_nr(fmax(x, 1e-300));
  return x > 0.0 ? y : 0.0;
}
// One Newton step only (relative error about 2^-46): for t, whose rounding
// decides how far a rotation reduces its pair, not the J-unitarity of the
// rotation (cs and sn are formed from the t actually used).
__device__ __forceinline__ double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double sqrt_nr1(double x) {
  const double d = fmax(x, 1e-300);
  double y = __builtin_amdgcn_rsq(d);
  y = fma(0.5 * y, fma(-(d * y), y, 1.0), y);
  return x > 0.0 ? x * y : 0.0;
}

// Rotation for the 2x2 pivot [arr eta; eta ass] (eta real) with sigma = +j_r j_s
// (Algorithm 3.1 read with sigma = +j_r j_s).  With N = sigma a_ss - a_rr
// (= 2 eta theta), t = sgn(theta) / (|theta| + sqrt(theta^2 + sigma)) is
// evaluated as sgn(N eta) 2|eta| / (|N| + sqrt(N^2 + 4 sigma eta^2)) after an
// exact power-of-two scaling of N and eta; cs = 1/sqrt(1 + sigma t^2), with
// 1 - t^2 = (1-|t|)(1+|t|), and sn = cs t, so that the applied rotation is
// J-unitary to working precision whatever the rounding of t.  The hyperbolic
// rotation exists iff |N| > 2|eta|.
// Returns 0: below tol, 1: (cs, sn) set, -1: hyperbolic breakdown (cs and sn
// are meaningful only for 1).
// The threshold test |eta| > tol sqrt(a_rr) sqrt(a_ss) uses the hardware
// reciprocal-square-root estimates (an error of 2^-23 can only change the
// decision for a pair lying at the threshold) and is evaluated beside the
// rotation instead of before it: the dependent chain of a round is the
// rotation alone.
__device__ __forceinline__ int rot_params(double arr, double ass, double eta, double sigma, double tol,
                                          double* cs, double* sn) {
  const bool above = fabs(eta) * (__builtin_amdgcn_rsq(arr) * __builtin_amdgcn_rsq(ass)) > tol;
  const double N = sigma * ass - arr;
  const double e2 = 2.0 * fabs(eta);
  const bool no_hyp = sigma < 0.0 && fabs(N) <= e2;
  const int ex = ilogb(fmax(fabs(N), e2));
  const double Ns = ldexp(N, -ex), Es = ldexp(e2, -ex);
  double t = Es * rcp_nr1(fabs(Ns) + sqrt_nr1(fma(Ns, Ns, sigma * (Es * Es))));
  if ((N < 0.0) != (eta < 0.0)) t = -t;
  const double at = fabs(t);
  const double c = rsqrt_nr(sigma > 0.0 ? fma(t, t, 1.0) : (1.0 - at) * (1.0 + at));
  *cs = c;
  *sn = c * t;
  return !above ? 0 : (no_hyp ? -1 : 1);
}

// Move a double across lanes with a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Lane exchanges within a wavefront: DPP row rotation by 8 inside 16-lane rows
// (the value of lane ^ 8), and a lane permute from a byte address (lane ^ x) * 4.
__device__ __forceinline__ double xor8_of(double v) { return dpp_f64<0x128>(v); }
__device__ __forceinline__ double2 xor8_of(double2 v) { return double2{xor8_of(v.x), xor8_of(v.y)}; }
__device__ __forceinline__ double bperm_of(double v, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 bperm_of(double2 v, int addr) {
  return double2{bperm_of(v.x, addr), bperm_of(v.y, addr)};
}

// Sum over the LPS lanes of a slot (slots are aligned groups of LPS lanes).
// LPS == 8: xor-1 and xor-2 quad permutations, then the half-row mirror, which
// pairs quad 0 with quad 1 of each 8-lane half: three DPP steps, no LDS.
template <int LPS>
__device__ __forceinline__ double slot_sum(double v) {
  if constexpr (LPS == 8 || LPS == 16) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror: quad 0 <-> quad 1 of each 8-lane half
    if constexpr (LPS == 16) v += dpp_f64<0x140>(v);  // row_mirror: half 0 <-> half 1 of the row
    return v;
  } else {
#pragma unroll
    for (int msk = 1; msk < LPS; msk <<= 1) v += __shfl_xor(v, msk);
    return v;
  }
}

// Rotation of one column pair from the three dot products; returns -1/0/1 as
// rot_params and the phase (pr, pi) of e^{i alpha} = a_rs / eta.
__device__ __forceinline__ int pair_rotation(double arr, double ass, double are, double aim, bool cplx, double sigma,
                                             double tol, double* cs, double* sn, double* pr, double* pi) {
  double eta;
  if (cplx) {
    // |a_rs| with an exact power-of-two scaling against under/overflow
    const int ex = ilogb(fmax(fmax(fabs(are), fabs(aim)), 1e-300));
    const double xr = ldexp(are, -ex), xi = ldexp(aim, -ex);
    const double ms = sqrt_nr(fma(xr, xr, xi * xi));
    const double einv = (are < 0.0 ? -1.0 : 1.0) * rcp_nr(ms);
    eta = (are < 0.0 ? -1.0 : 1.0) * ldexp(ms, ex);
    *pr = xr * einv;
    *pi = xi * einv;
  } else {
    eta = are;
  }
  const int rc = rot_params(arr, ass, eta, sigma, tol, cs, sn);
  if (!(rc > 0 && cplx)) {
    *pr = 1.0;
    *pi = 0.0;
  }
  return rc;
}

// Value of v in lane l (l uniform across the wave).
__device__ __forceinline__ double readlane_of(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 readlane_of(double2 v, int l) {
  return double2{readlane_of(v.x, l), readlane_of(v.y, l)};
}

// |a| f for a scale factor f > 0 (the scaled off-diagonal measure)
__device__ __forceinline__ double abs_scaled(double a, double f) { return fabs(a) * f; }

// One Cholesky panel (rows r0..r0+kn-1) held as s[ii] = S[r0 + ii][lane]:
// row k of R is row k of S times 1/sqrt(s_kk), then each later row i of the
// panel subtracts conj(r_ki) * (row k of R), r_ki being lane i's entry.
// DEFER > 0: only the next row's factor r_k,k+1 is taken by a lane read (the
// dependent chain from one diagonal entry to the next); row k also goes to the
// 16 x 64 LDS buffer rb, from which the later rows' factors are read, and
// their updates are applied one row later, beside the next square root.
// DEFER == 1 reads the factors one row ahead into registers (about 30 more
// values held); DEFER == 2 prefetches only the one that the next row's chain
// needs and reads the others where they are used.  Every entry takes the
// updates of rows 0, 1, ... in that order, with the same operations.
// Returns nonzero if a pivot s_kk is not positive and finite (the caller stops
// after the panel; the steps after it run on meaningless values).
template <bool FULL, int DEFER, typename T>
__device__ __forceinline__ int chol_panel(T (&s)[16], int r0, int kn, int lane, T* rb) {
  int bad = 0;
  T rp[16];  // DEFER == 1: row kk - 1 of R at columns r0 + ii, ii >= kk + 1
  T rn = zero_of(T());  // DEFER == 2: r_{kk-1, kk+1}
#pragma unroll
  for (int kk = 0; kk < 16; kk++) {
    if (FULL || kk < kn) {
      const double d = real_of(readlane_of(s[kk], r0 + kk));  // uniform across the wave
      bad |= !(d > 0.0 && isfinite(d));
      const double y = rsqrt_nr(d);
      s[kk] = scale(s[kk], y);
      if (lane == r0 + kk) s[kk] = scale(one_like(s[kk]), d * y);  // real positive diagonal
      if constexpr (DEFER > 0) {
        rb[64 * kk + lane] = s[kk];  // every lane: no branch in the unrolled panel
        if (kk + 1 < 16 && (FULL || kk + 1 < kn)) {
          if (kk >= 1)
            s[kk + 1] = lin2(1.0, s[kk + 1], -1.0,
                             cmul_conj_first(conj_of(DEFER == 1 ? rp[kk + 1] : rn), s[kk - 1]));
          const T rk1 = readlane_of(s[kk], r0 + kk + 1);
          s[kk + 1] = lin2(1.0, s[kk + 1], -1.0, cmul_conj_first(conj_of(rk1), s[kk]));
        }
        wave_sync();  // the row's LDS writes before the reads below
        if constexpr (DEFER == 1) {
          T rc[16];
#pragma unroll
          for (int ii = kk + 2; ii < 16; ii++)
            if (FULL || ii < kn) rc[ii] = rb[64 * kk + r0 + ii];
#pragma unroll
          for (int ii = kk + 2; ii < 16; ii++) {
            if (kk >= 1 && (FULL || ii < kn))
              s[ii] = lin2(1.0, s[ii], -1.0, cmul_conj_first(conj_of(rp[ii]), s[kk - 1]));
            rp[ii] = rc[ii];
          }
        } else {
          const T rnew = (kk + 2 < 16 && (FULL || kk + 2 < kn)) ? rb[64 * kk + r0 + kk + 2] : zero_of(T());
#pragma unroll
          for (int ii = kk + 2; ii < 16; ii++)
            if (kk >= 1 && (FULL || ii < kn))
              s[ii] = lin2(1.0, s[ii], -1.0, cmul_conj_first(conj_of(rb[64 * (kk - 1) + r0 + ii]), s[kk - 1]));
          rn = rnew;
        }
      } else {
#pragma unroll
        for (int ii = kk + 1; ii < 16; ii++) {
          if (FULL || ii < kn) {
            const T rki = readlane_of(s[kk], r0 + ii);
            s[ii] = lin2(1.0, s[ii], -1.0, cmul_conj_first(conj_of(rki), s[kk]));
          }
        }
      }
    }
  }
  return bad;
}

typedef double d4p __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4p mfma16p(double a, double b, d4p c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Trailing update of the Cholesky after the panel of rows r0..r0+15:
// S[16I.., 16J..] -= R_p[:, 16I..]^* R_p[:, 16J..] for the tiles
// r0 + 16 <= 16I <= 16J < m.  Real: one wavefront takes all tiles (four MFMAs
// each); complex: one tile per wavefront (sixteen MFMAs each, at most six
// tiles; the tiles are disjoint and the panel rows they read are not written).
// MFMA lane l supplies A[l%16][l/16], B[l/16][l%16] and holds
// D[4v + l/16][l%16]; S and R share the column-major LDS array.
__device__ __forceinline__ bool trailing_tile(int r0, int m, int wave, int& I, int& J) {
  const int tn = (m + 15) >> 4;
  int k = wave;
  for (I = (r0 >> 4) + 1; I < tn; I++)
    for (J = I; J < tn; J++)
      if (k-- == 0) return true;
  return false;
}
__device__ __forceinline__ void chol_trailing(double* R, int r0, int m, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  const int tn = (m + 15) >> 4;
  for (int I = (r0 >> 4) + 1; I < tn; I++)
    for (int J = I; J < tn; J++) {
      d4p acc;
#pragma unroll
      for (int v = 0; v < 4; v++) acc[v] = R[(16 * J + c16) * LDR + 16 * I + 4 * v + g];
#pragma unroll
      for (int q = 0; q < 4; q++)
        acc = mfma16p(-R[(16 * I + c16) * LDR + r0 + 4 * q + g], R[(16 * J + c16) * LDR + r0 + 4 * q + g], acc);
#pragma unroll
      for (int v = 0; v < 4; v++) R[(16 * J + c16) * LDR + 16 * I + 4 * v + g] = acc[v];
    }
}
// Complex: Re -= Xr^T Yr + Xi^T Yi, Im -= Xr^T Yi - Xi^T Yr.
__device__ __forceinline__ void chol_trailing(double2* R, int r0, int m, int wave, int lane) {
  const int c16 = lane & 15, g = lane >> 4;
  int I, J;
  if (trailing_tile(r0, m, wave, I, J)) {
      d4p are, aim;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const double2 a = R[(16 * J + c16) * LDR + 16 * I + 4 * v + g];
        are[v] = a.x;
        aim[v] = a.y;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double2 x = R[(16 * I + c16) * LDR + r0 + 4 * q + g];
        const double2 y = R[(16 * J + c16) * LDR + r0 + 4 * q + g];
        are = mfma16p(-x.x, y.x, are);
        are = mfma16p(-x.y, y.y, are);
        aim = mfma16p(-x.x, y.y, aim);
        aim = mfma16p(x.y, y.x, aim);
      }
#pragma unroll
      for (int v = 0; v < 4; v++) R[(16 * J + c16) * LDR + 16 * I + 4 * v + g] = double2{are[v], aim[v]};
    }
}

// DENSE: at most 128 registers per lane (a few spills), so that two real
// workgroups share a CU; used for batched launches, whose thousands of pivots
// are bound by the latency of each one and gain from a second workgroup per CU.
// Single solves (one pivot per CU at most) use the unconstrained build.
// CHOL: the Cholesky panel form (chol_panel's DEFER).  The deferred forms
// shorten the factorisation; launches that diagonalise their pivots in full
// spend nearly all their time in the inner sweeps, which compile about 3%
// faster beside the lane-read form, and take that one.
template <bool CPLX, int LPS, bool DENSE, int CHOL>
__global__ __launch_bounds__(64 * LPS) __attribute__((amdgpu_waves_per_eu(DENSE ? 4 : 1, 8))) void k_pivot(const double* __restrict__ part, int nch, int n0,
                                                    int rows_per_chunk, const int* __restrict__ mlist,
                                                    const int* __restrict__ nfirst,
                                                    const signed char* __restrict__ sgl, double tol, double tol64,
                                                    int inner_max,
                                                    int mode, int soft, double* __restrict__ Wout,
                                                    int* __restrict__ rotflag, SweepStats* st0, Batch bt,
                                                    int* __restrict__ refine, const int* __restrict__ only,
                                                    double* Gd, int ldgd, const int* __restrict__ cols) {
  typedef typename Scalar<CPLX>::T T;
  constexpr int NT = 64 * LPS;  // two halves of 32 slots
  constexpr int HT = 32 * LPS;  // threads of one half
  constexpr int RPL = kMaxPivot / LPS;  // rows of one column held by a lane
  __shared__ T lds[2 * kMaxPivot * LDR];
  __shared__ double redv[NT / 64];
  __shared__ double s_dinv[kMaxPivot];
  __shared__ int s_cnt, s_bad;
  __shared__ signed char s_sg[kMaxPivot];
  __shared__ int ring_sg[2][32];
  __shared__ double prm[2][32][5];  // rotation of each slot in a cross round: cs, sn, -sigma sn, phase
  __shared__ int prc[2][32];        // 1: that rotation is applied
  __shared__ T s_rb[CHOL == 0 ? 1 : 16 * 64];  // Cholesky: the rows of the current panel
  T* R = lds;
  T* W = lds + kMaxPivot * LDR;
  const int bslot = blockIdx.x, tid = threadIdx.x;
  if (only != nullptr && !only[bslot]) return;  // a re-solve launch: this pivot was solved
  int p = bslot, n = n0, ldgm = ldgd;
  double* Gm = Gd;
  SweepStats* st = st0;
  if (!batch_resolve(bt, bslot, p, Gm, ldgm, n, st)) return;
  // partials present for this pivot's rows (fewer than nch for short problems in a batch)
  const int nchp = min(nch, (n + rows_per_chunk - 1) / rows_per_chunk);
  if (bt.slot_prob != nullptr) {
    const int prob = bt.slot_prob[bslot];
    tol = bt.tol[prob];
    if (bt.prec != nullptr && bt.prec[prob]) {  // mixed sweep: threshold above FP32 Gram noise
      tol = fmax(tol, 0x1p-20);
      soft = 1;
    }
    if (mode == 2) mode = (bt.step[prob] == 0) ? 0 : 1;  // block-oriented, per problem
  }
  const int m = mlist[p];
  const int n1 = nfirst[p], n2 = m - n1;
  if (tid < kMaxPivot) s_sg[tid] = sgl[p * kMaxPivot + tid];
  // single-solve mixed sweeps: a pair whose FP32 block could not be factored
  // earlier in the solve has its Gram block formed in FP64 from then on (flag
  // refine[slot], kept across sweeps) and is solved as in an FP64 sweep
  if (refine != nullptr && refine[bslot]) {
    soft = 0;
    tol = tol64;
  }
  const signed char* sg = s_sg;  // signs of the pivot's columns, in LDS
  // the instance whose direct mode takes the within-block pairs by XOR passes
  // in registers (real, lane-read Cholesky form; the other instances keep their
  // register allocation)
  constexpr bool kLevels = !DENSE && !CPLX && CHOL == 0;
  // the instances that serve the direct mode (mode 3): single solves, the real
  // lane-read Cholesky form and the complex kernel
  constexpr bool kDirect = !DENSE && (CPLX || CHOL == 0);

  {
  // ---- 1. A_P = sum of the chunk partials (upper 16x16 tiles), Hermitian fill ----
  // Thread u of each 256-element tile takes element (u / 16, u % 16) of it; the
  // chunk loads of EB tiles are issued together, then summed in chunk order.
  const T* P = reinterpret_cast<const T*>(part) + (size_t)bslot * nch * (kMaxPivot * kMaxPivot);
  if constexpr (!CPLX && NT == 512) {
    // real, 512 threads: two adjacent columns of a tile row per thread (16-byte
    // loads, half the load instructions), the same sums in the same order
    constexpr int EB2 = 3;  // 3 x 512 threads >= 1280 column pairs of the ten upper tiles
    const double2* P2 = reinterpret_cast<const double2*>(P);
    double2 v[EB2][kMaxChunks];
    int rr[EB2], cc[EB2];
#pragma unroll
    for (int h = 0; h < EB2; h++) {
      const int u = tid + h * NT, t = u >> 7, w = u & 127;
      const int I = t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3));
      const int J = t - (I == 0 ? 0 : (I == 1 ? 3 : (I == 2 ? 5 : 6)));
      const int r = 16 * I + (w >> 3), c = 16 * J + 2 * (w & 7);
      const bool ok = t < 10 && r < m && c < m;
      rr[h] = ok ? r : -1;
      cc[h] = c;
#pragma unroll
      for (int k = 0; k < kMaxChunks; k++)
        v[h][k] = (ok && k < nchp) ? P2[((size_t)k * (kMaxPivot * kMaxPivot) + r * kMaxPivot + c) >> 1]
                                   : double2{0.0, 0.0};
    }
#pragma unroll
    for (int h = 0; h < EB2; h++) {
      if (rr[h] >= 0) {
        double2 sum = v[h][0];
#pragma unroll
        for (int k = 1; k < kMaxChunks; k++) sum = lin2(1.0, sum, 1.0, v[h][k]);
        R[cc[h] * LDR + rr[h]] = sum.x;
        if (cc[h] + 1 < m) R[(cc[h] + 1) * LDR + rr[h]] = sum.y;
      }
    }
  } else {
    constexpr int EB = 5;  // all loads of the partials in flight at once
    for (int u0 = tid; u0 < 10 * 256; u0 += EB * NT) {
      T v[EB][kMaxChunks];
      int rr[EB], cc[EB];
#pragma unroll
      for (int h = 0; h < EB; h++) {
        const int u = u0 + h * NT, t = u >> 8, w = u & 255;
        // upper tiles in the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)
        const int I = t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3));
        const int J = t - (I == 0 ? 0 : (I == 1 ? 3 : (I == 2 ? 5 : 6)));
        const int r = 16 * I + (w >> 4), c = 16 * J + (w & 15);
        const bool ok = t < 10 && r < m && c < m;
        rr[h] = ok ? r : -1;
        cc[h] = c;
#pragma unroll
        for (int k = 0; k < kMaxChunks; k++)
          v[h][k] = (ok && k < nchp) ? P[(size_t)k * (kMaxPivot * kMaxPivot) + r * kMaxPivot + c] : zero_of(T());
      }
#pragma unroll
      for (int h = 0; h < EB; h++) {
        if (rr[h] >= 0) {
          T sum = v[h][0];
#pragma unroll
          for (int k = 1; k < kMaxChunks; k++) sum = lin2(1.0, sum, 1.0, v[h][k]);
          R[cc[h] * LDR + rr[h]] = sum;
        }
      }
    }
  }
  if (tid == 0) {
    s_bad = 0;
    s_cnt = 0;
  }
  __syncthreads();
  // Only the upper triangle is formed: the off-diagonal test reads it, and the
  // Cholesky below reads and writes no entry left of the diagonal that feeds
  // an entry on or right of it (it writes zeros there).

  // ---- 2. scaled off-diagonal test; zero or non-finite diagonal = breakdown ----
  if (tid < kMaxPivot) {
    const double d = tid < m ? real_of(R[tid * LDR + tid]) : 1.0;
    const bool okd = d > 0.0 && isfinite(d);
    if (!okd) atomicOr(&s_bad, 1);
    s_dinv[tid] = okd ? rsqrt_nr(d) : 0.0;
  }
  __syncthreads();
  // complex: the largest squared modulus, one square root at the end
  double off = 0.0;
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
    const int r = e & 63, c = e >> 6;
    if (r < c && c < m) {
      if constexpr (CPLX) {
        const T a = R[c * LDR + r];
        const double f = s_dinv[r] * s_dinv[c], x = a.x * f, y = a.y * f;
        off = fmax(off, fma(x, x, y * y));
      } else {
        off = fmax(off, abs_scaled(R[c * LDR + r], s_dinv[r] * s_dinv[c]));
      }
    }
  }
#pragma unroll
  for (int msk = 32; msk > 0; msk >>= 1) off = fmax(off, __shfl_xor(off, msk));
  if ((tid & 63) == 0) redv[tid >> 6] = off;
  __syncthreads();
  off = redv[0];
  for (int w = 1; w < NT / 64; w++) off = fmax(off, redv[w]);
  if constexpr (CPLX) off = sqrt_nr(off);
  if (tid == 0) atomic_max_nonneg(&st->max_off_bits, isfinite(off) ? off : 1.0e300);
  if (s_bad || (off <= tol && !(kDirect && mode == 3))) {
    if (tid == 0) {
      rotflag[bslot] = 0;
      if (s_bad) {
        if (soft) {
          atomicAdd(&st->soft_fail, 1);
          if (refine != nullptr) refine[bslot] = 1;
        }
        else atomicOr(&st->breakdown, 1);
      }
    }
    return;
  }

  // ---- 3. Cholesky A_P = R^* R by wavefront 0, in panels of 16 rows ----
  // Panel rows r0..r0+15: lane j holds S[r0 + ii][j] of the current Schur
  // complement S in registers.  Row k of R is row k of S times 1/sqrt(s_kk);
  // the later rows i of the panel then subtract conj(r_ki) * (row k of R), with
  // r_ki read from lane i.  The rows below the panel take the same update as
  // 16x16 tiles on the FP64 matrix cores (S_IJ -= R_pI^* R_pJ), through LDS.
  {
    const int wave = tid >> 6, lane = tid & 63;
    if (tid >= 64) {
      // W_P = I, written by the other wavefronts while the first panel is factored
      for (int e = tid - 64; e < kMaxPivot * kMaxPivot; e += NT - 64) {
        int r = e & 63, c = e >> 6;
        if (r < m && c < m) {
          T one = zero_of(T());
          if constexpr (CPLX) one.x = (r == c) ? 1.0 : 0.0; else one = (r == c) ? 1.0 : 0.0;
          W[c * LDR + r] = one;
        }
      }
    }
    auto panel = [&](int r0) {  // wavefront 0; false if a pivot is not positive
      const int kn = min(16, m - r0);
      T s[16];
#pragma unroll
      for (int ii = 0; ii < 16; ii++)
        s[ii] = (lane >= r0 && lane < m && ii < kn) ? R[lane * LDR + r0 + ii] : zero_of(T());
      const int bad = kn == 16 ? chol_panel<true, CHOL>(s, r0, kn, lane, s_rb)
                               : chol_panel<false, CHOL>(s, r0, kn, lane, s_rb);
      if (bad) return false;
      // rows r0..r0+kn-1 of R, zero left of the diagonal and beyond column m
#pragma unroll
      for (int ii = 0; ii < 16; ii++)
        if (ii < kn) R[lane * LDR + r0 + ii] = (lane < r0 + ii || lane >= m) ? zero_of(T()) : s[ii];
      return true;
    };
    if constexpr (CPLX) {
      // trailing tiles spread over the wavefronts, a workgroup barrier per panel
      for (int r0 = 0; r0 < m; r0 += 16) {
        if (wave == 0 && !panel(r0) && lane == 0) s_bad = 1;
        __syncthreads();
        if (s_bad) break;
        if (r0 + 16 < m) {
          chol_trailing(R, r0, m, wave, lane);
          __syncthreads();
        }
      }
    } else {
      // wavefront 0 alone, wavefront-level synchronisation
      if (wave == 0) {
        int ok = 1;
        for (int r0 = 0; r0 < m && ok; r0 += 16) {
          ok = panel(r0);
          if (ok && r0 + 16 < m) {
            wave_sync();
            chol_trailing(R, r0, m, lane);
            wave_sync();
          }
        }
        if (lane == 0 && !ok) s_bad = 1;
      }
      __syncthreads();
    }
    if (s_bad) {
      if (tid == 0) {
        rotflag[bslot] = 0;
        if (soft) {
          atomicAdd(&st->soft_fail, 1);
          if (refine != nullptr) refine[bslot] = 1;
        }
        else atomicOr(&st->breakdown, 1);
      }
      return;
    }
  }

  }  // phases 1-3

  // ---- direct mode (one pivot holding all n <= kMaxPivot columns of G): the
  // non-blocked one-sided J-Jacobi on G itself (Algorithm 3.2), G's rows in
  // place of R's.  The Gram block and its Cholesky factor above serve only to
  // test that G has full column rank to working precision, as in every blocked
  // step (a failed factorisation is a breakdown). ----
  if (kDirect && mode == 3) {
    __syncthreads();  // the factor in R is no longer read
    const T* Gc = reinterpret_cast<const T*>(Gm);
    for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
      const int r = e & 63, c = e >> 6;
      if (c < m) R[c * LDR + r] = r < n ? Gc[(size_t)cols[p * kMaxPivot + c] * ldgm + r] : zero_of(T());
    }
    __syncthreads();
  }

  // ---- 4. inner sweeps ----
  // half 0 (threads 0..HT-1) holds columns of R, half 1 columns of W_P in the
  // split cross pass; elsewhere half 0 works on both and half 1 waits
  const int half = tid / HT, slot = (tid % HT) / LPS, sub = tid % LPS;
  const int L = max(n1, n2);
  const bool full = mode == 0 || (kDirect && mode == 3);  // within-block pairs too, inner sweeps up to inner_max
  const int nsweeps = full ? inner_max : 1;
  int total = 0, sweeps_run = 0, last_cnt = 0;
  for (int it = 0; it < nsweeps; it++) {
    int cnt = 0;
    sweeps_run++;
    // One XOR pass over groups of Lv slots (Lv a power of two, Lv <= L): group
    // g pairs columns 2 Lv g .. 2 Lv g + Lv - 1 with the next Lv columns, every
    // pair once, in Lv rounds; Lv = L is the cross pass of the two blocks.
    auto xor_level = [&](const int Lv) {
      __syncthreads();  // the columns written back by the previous pass are in place
      T* M = half == 0 ? R : W;
      // group of Lv slots: first-block columns ca, second-block columns from cb on
      const int local = slot & (Lv - 1), base = 2 * Lv * (slot / Lv);
      const int ca = base + local, cb = base + Lv + local;
      T a[RPL], b[RPL];
#pragma unroll
      for (int i = 0; i < RPL; i++) {
        const int row = sub + LPS * i;
        const bool ok = row < m && slot < L;
        a[i] = ok ? M[ca * LDR + row] : zero_of(T());
        b[i] = ok ? M[cb * LDR + row] : zero_of(T());
      }
      __syncthreads();
      // LDS exchange buffers (aliasing R and W_P): per half two parities of 32 slots x 64 rows
      T* ringh = lds + half * (4 * 32 * kMaxPivot / 2);
      const double sr = slot < L ? (double)sg[ca] : 0.0;
      double ss = slot < L ? (double)sg[cb] : 0.0;  // sign of the held second-block column (half 0)
      for (int q = 0; q <= Lv; q++) {
        if (half == 0 && q < Lv && slot < L) {
          double arr = 0.0, ass = 0.0, are = 0.0, aim = 0.0;
#pragma unroll
          for (int i = 0; i < RPL; i++) {
            arr += abs2(a[i]);
            ass += abs2(b[i]);
            cdot(a[i], b[i], are, aim);
          }
          arr = slot_sum<LPS>(arr);
          ass = slot_sum<LPS>(ass);
          are = slot_sum<LPS>(are);
          if (CPLX) aim = slot_sum<LPS>(aim);
          const double sigma = sr * ss;
          double cs, sn, pr, pi;
          const int rc = pair_rotation(arr, ass, are, aim, CPLX, sigma, tol, &cs, &sn, &pr, &pi);
          if (sub == 0) {
            prm[q & 1][slot][0] = cs;
            prm[q & 1][slot][1] = sn;
            prm[q & 1][slot][2] = -sigma * sn;
            prm[q & 1][slot][3] = pr;
            prm[q & 1][slot][4] = pi;
            prc[q & 1][slot] = rc > 0;
          }
          if (rc > 0) {
#pragma unroll
            for (int i = 0; i < RPL; i++) {
              const T f = phase_mul(pr, pi, a[i]), g = b[i];
              a[i] = lin2(cs, f, -sigma * sn, g);
              b[i] = lin2(sn, f, cs, g);
            }
            cnt += (sub == 0);
          } else if (rc < 0 && sub == 0) {
            atomicOr(&s_bad, 1);
          }
        } else if (half == 1 && q >= 1 && slot < L && prc[(q - 1) & 1][slot]) {
          const double* pp = prm[(q - 1) & 1][slot];
          const double cs = pp[0], sn = pp[1], msn = pp[2], pr = pp[3], pi = pp[4];
#pragma unroll
          for (int i = 0; i < RPL; i++) {
            const T u = phase_mul(pr, pi, a[i]), w = b[i];
            a[i] = lin2(cs, u, msn, w);
            b[i] = lin2(sn, u, cs, w);
          }
        }
        // move of the held column: half 0 into round q + 1, half 1 into round q
        const int mq = half == 0 ? q + 1 : q;
        const int bit = (mq >= 1 && mq < Lv) ? __builtin_ctz(mq) : -1;
        const int lx = bit >= 0 ? (LPS << bit) : 0;
        if (lx == 8) {
          if (half == 0) ss = xor8_of(ss);
#pragma unroll
          for (int i = 0; i < RPL; i++) b[i] = xor8_of(b[i]);
        } else if (lx > 0 && lx < 64) {
          const int addr = ((tid & 63) ^ lx) << 2;
          if (half == 0) ss = bperm_of(ss, addr);
#pragma unroll
          for (int i = 0; i < RPL; i++) b[i] = bperm_of(b[i], addr);
        }
        double2* ring = reinterpret_cast<double2*>(ringh + (q & 1) * (32 * kMaxPivot));
        if (lx >= 64) {
          if (half == 0 && sub == 0) ring_sg[q & 1][slot] = (int)ss;
          if constexpr (CPLX) {
#pragma unroll
            for (int j = 0; j < RPL; j++) ring[(j * 32 + slot) * LPS + sub] = b[j];
          } else {
#pragma unroll
            for (int j = 0; j < RPL / 2; j++) ring[(j * 32 + slot) * LPS + sub] = double2{b[2 * j], b[2 * j + 1]};
          }
        }
        __syncthreads();
        if (lx >= 64) {
          const int from = slot ^ (1 << bit);
          if (half == 0) ss = (double)ring_sg[q & 1][from];
          if constexpr (CPLX) {
#pragma unroll
            for (int j = 0; j < RPL; j++) b[j] = ring[(j * 32 + from) * LPS + sub];
          } else {
#pragma unroll
            for (int j = 0; j < RPL / 2; j++) {
              const double2 v = ring[(j * 32 + from) * LPS + sub];
              b[2 * j] = v.x;
              b[2 * j + 1] = v.y;
            }
          }
        }
      }
      __syncthreads();
      // write the columns back: slot k holds second-block column k ^ gray(Lv - 1) = k ^ (Lv / 2)
      const int sfin = base + Lv + (local ^ (Lv >> 1));
      if (slot < L) {
#pragma unroll
        for (int i = 0; i < RPL; i++) {
          const int row = sub + LPS * i;
          if (row < m) {
            M[ca * LDR + row] = a[i];
            M[sfin * LDR + row] = b[i];
          }
        }
      }
    };
    // (a) within-block pairs.  The direct mode with two equal power-of-two
    // blocks (real): XOR passes over groups of L/2, L/4, ..., 1 slots, the
    // pairs inside each half, quarter, ... of both blocks, all in registers
    // (L - 1 rounds).  Otherwise circle round-robin on each block, data in LDS
    // (the order that the blocked steps keep: at n = 4096 the XOR order took
    // 40 sweeps instead of 38).
    if (full && kLevels && mode == 3 && L >= 2 && n1 == n2 && (L & (L - 1)) == 0) {
      for (int Lv = L >> 1; Lv >= 1; Lv >>= 1) xor_level(Lv);
    } else if (full) {
      const int blk = slot >> 4, hs = slot & 15;  // slots 0-15: block 1, 16-31: block 2
      const int nb = blk == 0 ? n1 : n2, base = blk == 0 ? 0 : n1;
      const int nbp = nb + (nb & 1);
      const int rounds = max(n1 + (n1 & 1), n2 + (n2 & 1)) - 1;
      for (int q = 0; q < rounds; q++) {
        int r = -1, s = -1;
        if (nbp >= 2 && q < nbp - 1 && hs < nbp / 2) {
          int a = hs == 0 ? 0 : ((hs - 1 + q) % (nbp - 1)) + 1;
          int b = ((nbp - 1 - hs - 1 + q) % (nbp - 1)) + 1;
          r = min(a, b);
          s = max(a, b);
        }
        if (half == 0 && r >= 0 && s < nb) {
          T* Rr = R + (base + r) * LDR;
          T* Rs = R + (base + s) * LDR;
          double arr = 0.0, ass = 0.0, are = 0.0, aim = 0.0;
          for (int i = sub; i < m; i += LPS) {
            T x = Rr[i], y = Rs[i];
            arr += abs2(x);
            ass += abs2(y);
            cdot(x, y, are, aim);
          }
          arr = slot_sum<LPS>(arr);
          ass = slot_sum<LPS>(ass);
          are = slot_sum<LPS>(are);
          if (CPLX) aim = slot_sum<LPS>(aim);
          const double sigma = (double)(sg[base + r] * sg[base + s]);
          double cs, sn, pr, pi;
          int rc = pair_rotation(arr, ass, are, aim, CPLX, sigma, tol, &cs, &sn, &pr, &pi);
          if (rc > 0) {
            for (int i = sub; i < m; i += LPS) {
              T f = phase_mul(pr, pi, Rr[i]), g = Rs[i];
              Rr[i] = lin2(cs, f, -sigma * sn, g);
              Rs[i] = lin2(sn, f, cs, g);
            }
            if (!(kDirect && mode == 3)) {  // the direct mode keeps no W_P
              T* Wr = W + (base + r) * LDR;
              T* Ws = W + (base + s) * LDR;
              for (int i = sub; i < m; i += LPS) {
                T u = phase_mul(pr, pi, Wr[i]), w = Ws[i];
                Wr[i] = lin2(cs, u, -sigma * sn, w);
                Ws[i] = lin2(sn, u, cs, w);
              }
            }
            cnt += (sub == 0);
          } else if (rc < 0 && sub == 0) {
            atomicOr(&s_bad, 1);
          }
        }
        __syncthreads();
      }
    }
    // (b) cross pairs: first-block column `slot` stays in registers while the
    // second-block columns move between slots.  Two equal power-of-two blocks
    // use the XOR schedule: in round q slot k meets second-block column
    // k ^ gray(q); from one round to the next a single bit b of gray(q) flips, so
    // every held column moves to slot k ^ 2^b, within the wavefront (DPP or lane
    // permute) while that slot lies in the same wavefront and through LDS
    // otherwise (3 of 31 moves for 32 columns).  There the work is split: the
    // wavefronts of half 0 hold the columns of R, compute each round's
    // rotations and publish them; those of half 1 hold the same columns of W_P
    // and apply the rotations of the previous round, so the W_P updates run
    // beside the next round's dot products (one barrier per round).  Other
    // shapes use the ring: slot k meets column (k + q) mod L, all columns
    // moving one slot down per round through LDS, done by half 0 alone.
    if (L > 0 && n2 > 0 && n1 == n2 && (L & (L - 1)) == 0) {
      if constexpr (kLevels) {
        xor_level(L);
      } else {  // the batched kernel: the same pass, its register allocation kept
        T* M = half == 0 ? R : W;
        T a[RPL], b[RPL];
#pragma unroll
        for (int i = 0; i < RPL; i++) {
          const int row = sub + LPS * i;
          const bool ok = row < m && slot < L;
          a[i] = ok ? M[slot * LDR + row] : zero_of(T());
          b[i] = ok ? M[(n1 + slot) * LDR + row] : zero_of(T());
        }
        __syncthreads();
        // LDS exchange buffers (aliasing R and W_P): per half two parities of 32 slots x 64 rows
        T* ringh = lds + half * (4 * 32 * kMaxPivot / 2);
        const double sr = slot < L ? (double)sg[slot] : 0.0;
        double ss = slot < L ? (double)sg[n1 + slot] : 0.0;  // sign of the held second-block column (half 0)
        for (int q = 0; q <= L; q++) {
          if (half == 0 && q < L && slot < L) {
            double arr = 0.0, ass = 0.0, are = 0.0, aim = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; i++) {
              arr += abs2(a[i]);
              ass += abs2(b[i]);
              cdot(a[i], b[i], are, aim);
            }
            arr = slot_sum<LPS>(arr);
            ass = slot_sum<LPS>(ass);
            are = slot_sum<LPS>(are);
            if (CPLX) aim = slot_sum<LPS>(aim);
            const double sigma = sr * ss;
            double cs, sn, pr, pi;
            const int rc = pair_rotation(arr, ass, are, aim, CPLX, sigma, tol, &cs, &sn, &pr, &pi);
            if (sub == 0) {
              prm[q & 1][slot][0] = cs;
              prm[q & 1][slot][1] = sn;
              prm[q & 1][slot][2] = -sigma * sn;
              prm[q & 1][slot][3] = pr;
              prm[q & 1][slot][4] = pi;
              prc[q & 1][slot] = rc > 0;
            }
            if (rc > 0) {
#pragma unroll
              for (int i = 0; i < RPL; i++) {
                const T f = phase_mul(pr, pi, a[i]), g = b[i];
                a[i] = lin2(cs, f, -sigma * sn, g);
                b[i] = lin2(sn, f, cs, g);
              }
              cnt += (sub == 0);
            } else if (rc < 0 && sub == 0) {
              atomicOr(&s_bad, 1);
            }
          } else if (half == 1 && q >= 1 && slot < L && prc[(q - 1) & 1][slot]) {
            const double* pp = prm[(q - 1) & 1][slot];
            const double cs = pp[0], sn = pp[1], msn = pp[2], pr = pp[3], pi = pp[4];
#pragma unroll
            for (int i = 0; i < RPL; i++) {
              const T u = phase_mul(pr, pi, a[i]), w = b[i];
              a[i] = lin2(cs, u, msn, w);
              b[i] = lin2(sn, u, cs, w);
            }
          }
          // move of the held column: half 0 into round q + 1, half 1 into round q
          const int mq = half == 0 ? q + 1 : q;
          const int bit = (mq >= 1 && mq < L) ? __builtin_ctz(mq) : -1;
          const int lx = bit >= 0 ? (LPS << bit) : 0;
          if (lx == 8) {
            if (half == 0) ss = xor8_of(ss);
#pragma unroll
            for (int i = 0; i < RPL; i++) b[i] = xor8_of(b[i]);
          } else if (lx > 0 && lx < 64) {
            const int addr = ((tid & 63) ^ lx) << 2;
            if (half == 0) ss = bperm_of(ss, addr);
#pragma unroll
            for (int i = 0; i < RPL; i++) b[i] = bperm_of(b[i], addr);
          }
          double2* ring = reinterpret_cast<double2*>(ringh + (q & 1) * (32 * kMaxPivot));
          if (lx >= 64) {
            if (half == 0 && sub == 0) ring_sg[q & 1][slot] = (int)ss;
            if constexpr (CPLX) {
#pragma unroll
              for (int j = 0; j < RPL; j++) ring[(j * 32 + slot) * LPS + sub] = b[j];
            } else {
#pragma unroll
              for (int j = 0; j < RPL / 2; j++) ring[(j * 32 + slot) * LPS + sub] = double2{b[2 * j], b[2 * j + 1]};
            }
          }
          __syncthreads();
          if (lx >= 64) {
            const int from = slot ^ (1 << bit);
            if (half == 0) ss = (double)ring_sg[q & 1][from];
            if constexpr (CPLX) {
#pragma unroll
              for (int j = 0; j < RPL; j++) b[j] = ring[(j * 32 + from) * LPS + sub];
            } else {
#pragma unroll
              for (int j = 0; j < RPL / 2; j++) {
                const double2 v = ring[(j * 32 + from) * LPS + sub];
                b[2 * j] = v.x;
                b[2 * j + 1] = v.y;
              }
            }
          }
        }
        __syncthreads();
        // write the columns back: slot k holds second-block column k ^ gray(L - 1) = k ^ (L / 2)
        const int sfin = slot ^ (L >> 1);
        if (slot < L) {
#pragma unroll
          for (int i = 0; i < RPL; i++) {
            const int row = sub + LPS * i;
            if (row < m) {
              M[slot * LDR + row] = a[i];
              M[(n1 + sfin) * LDR + row] = b[i];
            }
          }
        }
      }
    } else if (L > 0 && n2 > 0) {
      // ring schedule, half 0 only (half 1 takes part in the barriers)
      T rr[RPL], wr[RPL], rs[RPL], ws[RPL];
      const bool act = half == 0;
      const bool have_r = act && slot < n1;
#pragma unroll
      for (int i = 0; i < RPL; i++) {
        const int row = sub + LPS * i;
        const bool ok = row < m;
        rr[i] = (have_r && ok) ? R[slot * LDR + row] : zero_of(T());
        wr[i] = (have_r && ok) ? W[slot * LDR + row] : zero_of(T());
        rs[i] = (act && slot < n2 && ok) ? R[(n1 + slot) * LDR + row] : zero_of(T());
        ws[i] = (act && slot < n2 && ok) ? W[(n1 + slot) * LDR + row] : zero_of(T());
      }
      __syncthreads();
      T* ring0 = lds;
      T* ring1 = lds + 2 * 32 * kMaxPivot;  // each ring: 2 x 32 slots x 64 rows of T
      const double sr = have_r ? (double)sg[slot] : 0.0;
      double ss = (act && slot < n2) ? (double)sg[n1 + slot] : 0.0;
      for (int q = 0; q < L; q++) {
        int sidx = slot + q;  // second-block column held by this slot: (slot + q) mod L
        if (sidx >= L) sidx -= L;
        if (act && slot < L && have_r && sidx < n2) {
          double arr = 0.0, ass = 0.0, are = 0.0, aim = 0.0;
#pragma unroll
          for (int i = 0; i < RPL; i++) {
            arr += abs2(rr[i]);
            ass += abs2(rs[i]);
            cdot(rr[i], rs[i], are, aim);
          }
          arr = slot_sum<LPS>(arr);
          ass = slot_sum<LPS>(ass);
          are = slot_sum<LPS>(are);
          if (CPLX) aim = slot_sum<LPS>(aim);
          const double sigma = sr * ss;
          double cs, sn, pr, pi;
          const int rc = pair_rotation(arr, ass, are, aim, CPLX, sigma, tol, &cs, &sn, &pr, &pi);
          if (rc > 0) {
#pragma unroll
            for (int i = 0; i < RPL; i++) {
              T f = phase_mul(pr, pi, rr[i]), g = rs[i];
              rr[i] = lin2(cs, f, -sigma * sn, g);
              rs[i] = lin2(sn, f, cs, g);
              T u = phase_mul(pr, pi, wr[i]), w = ws[i];
              wr[i] = lin2(cs, u, -sigma * sn, w);
              ws[i] = lin2(sn, u, cs, w);
            }
            cnt += (sub == 0);
          } else if (rc < 0 && sub == 0) {
            atomicOr(&s_bad, 1);
          }
        }
        if (q + 1 < L) {
          // slot k receives the second-block column of slot (k + 1) mod L; the
          // ring holds 16-byte elements (two reals or one complex)
          double2* ring = reinterpret_cast<double2*>((q & 1) ? ring1 : ring0);
          const int from = slot + 1 < L ? slot + 1 : 0;
          const bool mv = act && slot < L;
          if (mv) {
            if (sub == 0) ring_sg[q & 1][slot] = (int)ss;
            if constexpr (CPLX) {
#pragma unroll
              for (int j = 0; j < RPL; j++) {
                ring[(j * 32 + slot) * LPS + sub] = rs[j];
                ring[((RPL + j) * 32 + slot) * LPS + sub] = ws[j];
              }
            } else {
#pragma unroll
              for (int j = 0; j < RPL / 2; j++) {
                ring[(j * 32 + slot) * LPS + sub] = double2{rs[2 * j], rs[2 * j + 1]};
                ring[((RPL / 2 + j) * 32 + slot) * LPS + sub] = double2{ws[2 * j], ws[2 * j + 1]};
              }
            }
          }
          __syncthreads();
          if (mv) {
            ss = (double)ring_sg[q & 1][from];
            if constexpr (CPLX) {
#pragma unroll
              for (int j = 0; j < RPL; j++) {
                rs[j] = ring[(j * 32 + from) * LPS + sub];
                ws[j] = ring[((RPL + j) * 32 + from) * LPS + sub];
              }
            } else {
#pragma unroll
              for (int j = 0; j < RPL / 2; j++) {
                const double2 u = ring[(j * 32 + from) * LPS + sub];
                const double2 v = ring[((RPL / 2 + j) * 32 + from) * LPS + sub];
                rs[2 * j] = u.x;
                rs[2 * j + 1] = u.y;
                ws[2 * j] = v.x;
                ws[2 * j + 1] = v.y;
              }
            }
          }
        }
      }
      __syncthreads();
      // write the columns back: slot k holds second-block column (k + L - 1) mod L
      const int sfin = (slot + L - 1) % L;
      if (act) {
#pragma unroll
        for (int i = 0; i < RPL; i++) {
          const int row = sub + LPS * i;
          if (row < m) {
            if (have_r) {
              R[slot * LDR + row] = rr[i];
              W[slot * LDR + row] = wr[i];
            }
            if (slot < L && sfin < n2) {
              R[(n1 + sfin) * LDR + row] = rs[i];
              W[(n1 + sfin) * LDR + row] = ws[i];
            }
          }
        }
      }
    }
    if (cnt) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    const int c_all = s_cnt;
    __syncthreads();
    if (tid == 0) s_cnt = 0;
    total += c_all;
    last_cnt = c_all;
    if (c_all == 0) break;
    __syncthreads();
  }
  if (s_bad && tid == 0) {
    if (soft) {
      atomicAdd(&st->soft_fail, 1);
      if (refine != nullptr) refine[bslot] = 1;
    } else {
      atomicOr(&st->breakdown, 1);
    }
  }
  if (s_bad && soft && refine != nullptr) {
    // left as it is in this sweep: the pair is solved from an FP64 Gram block
    // from the next sweep on
    if (tid == 0) rotflag[bslot] = 0;
    return;
  }

  if (kDirect && mode == 3) {
    // G~ = G W: the rotated columns go back to G; converged iff the last inner
    // sweep applied no rotation (counted in pivots_rotated otherwise)
    T* Gc = reinterpret_cast<T*>(Gm);
    if (!s_bad)
      for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
        const int r = e & 63, c = e >> 6;
        if (c < m && r < n) Gc[(size_t)cols[p * kMaxPivot + c] * ldgm + r] = R[c * LDR + r];
      }
    if (tid == 0) {
      rotflag[bslot] = 0;
      if (last_cnt > 0) atomicAdd(&st->pivots_rotated, 1);
      atomicAdd(&st->rotations, (unsigned long long)total);
      atomicAdd(&st->inner_sweeps, (unsigned long long)sweeps_run);
      atomicAdd(&st->pivot_cols, (unsigned long long)m);
      atomicAdd(&st->pivot_cols3, (unsigned long long)m * m * m);
    }
    return;
  }

  // ---- 5. W_P out ----
  const int rotated = total > 0;
  if (rotated) {
    T* Wo = reinterpret_cast<T*>(Wout) + (size_t)bslot * (kMaxPivot * kMaxPivot);
    for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
      int c = e >> 6, r = e & 63;
      if (r < m && c < m) Wo[c * kMaxPivot + r] = W[c * LDR + r];
    }
  }
  if (tid == 0) {
    rotflag[bslot] = rotated;
    if (rotated) atomicAdd(&st->pivots_rotated, 1);
    atomicAdd(&st->rotations, (unsigned long long)total);
    atomicAdd(&st->inner_sweeps, (unsigned long long)sweeps_run);
    atomicAdd(&st->pivot_cols, (unsigned long long)m);
    atomicAdd(&st->pivot_cols3, (unsigned long long)m * m * m);
  }
}

constexpr int kPivotLPS = 8;

void launch_pivot_f64(const double* part, int nch, int n, int rows_per_chunk, const PivotList& pl, double tol,
                      double tol64, int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                      hipStream_t stream, const Batch& b, int* refine, const int* only, double* G, int ldg) {
  // batched launches: two workgroups per CU, lane-read Cholesky (register budget)
  if (b.slot_prob != nullptr)
    launch((k_pivot<false, kPivotLPS, true, 0>), dim3(pl.count), dim3(64 * kPivotLPS), 0, stream, part, nch, n,
           rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, tol64, inner_max, inner_mode, soft, W, rotflag, st, b, refine, only,
           G, ldg, pl.cols);
  // full diagonalisation (mode 0, several inner sweeps): the lane-read Cholesky
  else if ((inner_mode == 0 && inner_max > 1) || inner_mode == 3)
    launch((k_pivot<false, kPivotLPS, false, 0>), dim3(pl.count), dim3(64 * kPivotLPS), 0, stream, part, nch, n,
           rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, tol64, inner_max, inner_mode, soft, W, rotflag, st, b, refine, only,
           G, ldg, pl.cols);
  else
    launch((k_pivot<false, kPivotLPS, false, 1>), dim3(pl.count), dim3(64 * kPivotLPS), 0, stream, part, nch, n,
           rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, tol64, inner_max, inner_mode, soft, W, rotflag, st, b, refine, only,
           G, ldg, pl.cols);
}

void launch_pivot_c128(const double* part, int nch, int n, int rows_per_chunk, const PivotList& pl, double tol,
                       double tol64, int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                       hipStream_t stream, const Batch& b, int* refine, const int* only, double* G, int ldg) {
  launch((k_pivot<true, kPivotLPS, false, 2>), dim3(pl.count), dim3(64 * kPivotLPS), 0, stream, part, nch, n,
                     rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, tol64, inner_max, inner_mode, soft, W, rotflag, st, b, refine, only,
           G, ldg, pl.cols);
}

}  // namespace jj
