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
//       move one slot per round through an LDS ring, so that slot k meets
//       second-block column (k + q) mod L in round q.
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
__device__ __forceinline__ double abs_of(double a) { return fabs(a); }
__device__ __forceinline__ double abs_of(double2 a) { return hypot(a.x, a.y); }
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

// Rotation for the 2x2 pivot [arr eta; eta ass] (eta real) with sigma = +j_r j_s
// (Algorithm 3.1 read with sigma = +j_r j_s).  With N = sigma a_ss - a_rr
// (= 2 eta theta), t = sgn(theta) / (|theta| + sqrt(theta^2 + sigma)) is
// evaluated as sgn(N eta) 2|eta| / (|N| + sqrt(N^2 + 4 sigma eta^2)) after an
// exact power-of-two scaling of N and eta; cs = 1/sqrt(1 + sigma t^2), with
// 1 - t^2 = (1-|t|)(1+|t|).  The hyperbolic rotation exists iff |N| > 2|eta|.
// Returns 0: below tol, 1: (cs, sn) set, -1: hyperbolic breakdown.
__device__ __forceinline__ int rot_params(double arr, double ass, double eta, double sigma, double tol,
                                          double* cs, double* sn) {
  if (!(fabs(eta) > tol * sqrt(arr) * sqrt(ass))) return 0;
  const double N = sigma * ass - arr;
  const double e2 = 2.0 * fabs(eta);
  if (sigma < 0.0 && fabs(N) <= e2) return -1;
  const int ex = ilogb(fmax(fabs(N), e2));
  const double Ns = ldexp(N, -ex), Es = ldexp(e2, -ex);
  double t = Es / (fabs(Ns) + sqrt(Ns * Ns + sigma * (Es * Es)));
  if ((N < 0.0) != (eta < 0.0)) t = -t;
  const double at = fabs(t);
  // correctly rounded sqrt and division: a biased reciprocal square root would
  // make every rotation slightly non-J-unitary in the same direction
  const double c = 1.0 / sqrt(sigma > 0.0 ? 1.0 + t * t : (1.0 - at) * (1.0 + at));
  *cs = c;
  *sn = c * t;
  return 1;
}

// Move a double across lanes with a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
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
    const double aabs = hypot(are, aim);
    eta = (are < 0.0 ? -1.0 : 1.0) * aabs;
  } else {
    eta = are;
  }
  int rc = rot_params(arr, ass, eta, sigma, tol, cs, sn);
  if (rc > 0 && cplx) {
    *pr = are / eta;
    *pi = aim / eta;
  } else {
    *pr = 1.0;
    *pi = 0.0;
  }
  return rc;
}

template <bool CPLX, int LPS>
__global__ __launch_bounds__(32 * LPS) void k_pivot(const double* __restrict__ part, int nch, int n0,
                                                    int rows_per_chunk, const int* __restrict__ mlist,
                                                    const int* __restrict__ nfirst,
                                                    const signed char* __restrict__ sgl, double tol, int inner_max,
                                                    int mode, int soft, double* __restrict__ Wout,
                                                    int* __restrict__ rotflag, SweepStats* st0, Batch bt) {
  typedef typename Scalar<CPLX>::T T;
  constexpr int NT = 32 * LPS;
  constexpr int RPL = kMaxPivot / LPS;  // rows of one column held by a lane
  __shared__ T lds[2 * kMaxPivot * LDR];
  __shared__ double redv[NT];
  __shared__ __align__(16) T rowb[kMaxPivot];
  __shared__ int s_cnt, s_bad;
  __shared__ signed char s_sg[kMaxPivot];
  __shared__ int ring_sg[2][32];
  T* R = lds;
  T* W = lds + kMaxPivot * LDR;
  const int bslot = blockIdx.x, tid = threadIdx.x;
  int p = bslot, n = n0, ldg_unused = 0;
  double* G_unused = nullptr;
  SweepStats* st = st0;
  if (!batch_resolve(bt, bslot, p, G_unused, ldg_unused, n, st)) return;
  // partials present for this pivot's rows (fewer than nch for short problems in a batch)
  const int nchp = min(nch, (n + rows_per_chunk - 1) / rows_per_chunk);
  if (bt.slot_prob != nullptr) {
    const int prob = bt.slot_prob[bslot];
    tol = bt.tol[prob];
    if (mode == 2) mode = (bt.step[prob] == 0) ? 0 : 1;  // block-oriented, per problem
  }
  const int m = mlist[p];
  const int n1 = nfirst[p], n2 = m - n1;
  if (tid < kMaxPivot) s_sg[tid] = sgl[p * kMaxPivot + tid];
  const signed char* sg = s_sg;  // signs of the pivot's columns, in LDS

  // ---- 1. A_P = sum of the chunk partials (upper 16x16 tiles), Hermitian fill ----
  // all chunk loads of an element are issued before the (fixed-order) sum
  const T* P = reinterpret_cast<const T*>(part) + (size_t)bslot * nch * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && (r >> 4) <= (c >> 4)) {
      T v[kMaxChunks];
#pragma unroll
      for (int k = 0; k < kMaxChunks; k++)
        v[k] = k < nchp ? P[(size_t)k * (kMaxPivot * kMaxPivot) + e] : zero_of(T());
      T s = v[0];
#pragma unroll
      for (int k = 1; k < kMaxChunks; k++) s = lin2(1.0, s, 1.0, v[k]);
      R[c * LDR + r] = s;
    }
  }
  if (tid == 0) {
    s_bad = 0;
    s_cnt = 0;
  }
  __syncthreads();
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r > c) R[c * LDR + r] = conj_of(R[r * LDR + c]);
  }
  __syncthreads();

  // ---- 2. scaled off-diagonal test; zero or non-finite diagonal = breakdown ----
  double off = 0.0;
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
    int r = e >> 6, c = e & 63;
    if (r < m && c < m && r < c) {
      double v = abs_of(R[c * LDR + r]) / (sqrt(real_of(R[r * LDR + r])) * sqrt(real_of(R[c * LDR + c])));
      off = fmax(off, v);
    }
  }
  for (int k = tid; k < m; k += NT) {
    double d = real_of(R[k * LDR + k]);
    if (!(d > 0.0) || !isfinite(d)) atomicOr(&s_bad, 1);
  }
  redv[tid] = off;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) redv[tid] = fmax(redv[tid], redv[tid + s]);
    __syncthreads();
  }
  off = redv[0];
  if (tid == 0) atomic_max_nonneg(&st->max_off_bits, isfinite(off) ? off : 1.0e300);
  if (s_bad || off <= tol) {
    if (tid == 0) {
      rotflag[bslot] = 0;
      if (s_bad) atomicOr(soft ? &st->soft_fail : &st->breakdown, 1);
    }
    return;
  }

  // ---- 3. Cholesky A_P = R^* R by one wavefront, without workgroup barriers ----
  // Lane i keeps row i of the Schur complement in registers.  Phase k: lane k
  // publishes its (final) row k to LDS, every lane i > k subtracts
  // (conj(a_ki)/a_kk) * row k from its row; lanes i <= k are finished.  Row i of
  // R is row i of the last Schur complement scaled by 1/sqrt(a_ii); the entries
  // left of the diagonal are cleared.
  {
    T* rowbuf = reinterpret_cast<T*>(rowb);
    int bad = 0;
    if (tid < 64) {
      const int i = tid;
      T a[kMaxPivot];
#pragma unroll
      for (int c = 0; c < kMaxPivot; c++) a[c] = (i < m && c < m) ? R[c * LDR + i] : zero_of(T());
      double mydiag = 1.0;
      for (int k = 0; k < m; k++) {
        if (i == k) {  // publish the part of row k right of column k (16-column groups)
#pragma unroll
          for (int g = 0; g < kMaxPivot / 16; g++)
            if (16 * g + 15 >= k) {
#pragma unroll
              for (int c = 0; c < 16; c++) rowbuf[16 * g + c] = a[16 * g + c];
            }
        }
        wave_sync();
        const double d = real_of(rowbuf[k]);
        if (!(d > 0.0) || !isfinite(d)) {
          bad = 1;
          break;
        }
        if (i == k) mydiag = d;
        const double dinv = 1.0 / d;
        // S_ic -= S_ik S_kc / S_kk with S_ik = conj(S_ki) = conj(rowbuf[i]); columns
        // c <= k of the rows i > k are left of the diagonal and never read again
        T f = (i > k && i < m) ? scale(conj_of(rowbuf[i]), dinv) : zero_of(T());
#pragma unroll
        for (int g = 0; g < kMaxPivot / 16; g++) {
          if (16 * g + 15 > k) {
            T rb[16];
#pragma unroll
            for (int c = 0; c < 16; c++) rb[c] = rowbuf[16 * g + c];
#pragma unroll
            for (int c = 0; c < 16; c++) a[16 * g + c] = lin2(1.0, a[16 * g + c], -1.0, cmul_conj_first(f, rb[c]));
          }
        }
        wave_sync();
      }
      if (!bad) {
        const double rs = 1.0 / sqrt(mydiag);
#pragma unroll
        for (int c = 0; c < kMaxPivot; c++) {
          if (i < m && c < m) {
            T v = (c < i) ? zero_of(T()) : scale(a[c], rs);
            if (c == i) v = scale(one_like(v), sqrt(mydiag));  // real positive diagonal
            R[c * LDR + i] = v;
          }
        }
      }
      if (tid == 0) s_bad = bad;
    }
    __syncthreads();
    if (s_bad) {
      if (tid == 0) {
        rotflag[bslot] = 0;
        atomicOr(soft ? &st->soft_fail : &st->breakdown, 1);
      }
      return;
    }
    for (int e = tid; e < kMaxPivot * kMaxPivot; e += NT) {
      int r = e & 63, c = e >> 6;
      if (r < m && c < m) {
        T one = zero_of(T());
        if constexpr (CPLX) one.x = (r == c) ? 1.0 : 0.0; else one = (r == c) ? 1.0 : 0.0;
        W[c * LDR + r] = one;
      }
    }
    __syncthreads();
  }

  // ---- 4. inner sweeps ----
  const int slot = tid / LPS, sub = tid % LPS;
  const int L = max(n1, n2);
  const int nsweeps = mode == 0 ? inner_max : 1;
  int total = 0, sweeps_run = 0;
  for (int it = 0; it < nsweeps; it++) {
    int cnt = 0;
    sweeps_run++;
    // (a) within-block pairs, circle round-robin on each block, data in LDS
    if (mode == 0) {
      const int half = slot >> 4, hs = slot & 15;  // slots 0-15: block 1, 16-31: block 2
      const int nb = half == 0 ? n1 : n2, base = half == 0 ? 0 : n1;
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
        if (r >= 0 && s < nb) {
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
            T* Wr = W + (base + r) * LDR;
            T* Ws = W + (base + s) * LDR;
            for (int i = sub; i < m; i += LPS) {
              T f = phase_mul(pr, pi, Rr[i]), g = Rs[i];
              Rr[i] = lin2(cs, f, -sigma * sn, g);
              Rs[i] = lin2(sn, f, cs, g);
              T u = phase_mul(pr, pi, Wr[i]), w = Ws[i];
              Wr[i] = lin2(cs, u, -sigma * sn, w);
              Ws[i] = lin2(sn, u, cs, w);
            }
            cnt += (sub == 0);
          } else if (rc < 0 && sub == 0) {
            atomicOr(&s_bad, 1);
          }
        }
        __syncthreads();
      }
    }
    // (b) cross pairs: first-block column `slot` stays in registers, second-block
    // columns move one slot down per round through an LDS ring (aliasing R/W)
    if (L > 0 && n2 > 0) {
      T rr[RPL], wr[RPL], rs[RPL], ws[RPL];
      const bool have_r = slot < n1;
#pragma unroll
      for (int i = 0; i < RPL; i++) {
        const int row = sub + LPS * i;
        const bool ok = row < m;
        rr[i] = (have_r && ok) ? R[slot * LDR + row] : zero_of(T());
        wr[i] = (have_r && ok) ? W[slot * LDR + row] : zero_of(T());
        rs[i] = (slot < n2 && ok) ? R[(n1 + slot) * LDR + row] : zero_of(T());
        ws[i] = (slot < n2 && ok) ? W[(n1 + slot) * LDR + row] : zero_of(T());
      }
      __syncthreads();
      T* ring0 = lds;
      T* ring1 = lds + 2 * 32 * kMaxPivot;  // each ring: 2 x 32 slots x 64 rows of T
      const double sr = have_r ? (double)sg[slot] : 0.0;
      double ss = slot < n2 ? (double)sg[n1 + slot] : 0.0;  // sign of the held second-block column
      for (int q = 0; q < L; q++) {
        int sidx = slot + q;  // second-block column held by this slot: (slot + q) mod L
        if (sidx >= L) sidx -= L;
        if (slot < L && have_r && sidx < n2) {
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
          int rc = pair_rotation(arr, ass, are, aim, CPLX, sigma, tol, &cs, &sn, &pr, &pi);
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
          // ring holds 16-byte elements (two reals or one complex) so that each
          // lane moves its share with 128-bit LDS accesses
          double2* ring = reinterpret_cast<double2*>((q & 1) ? ring1 : ring0);
          if (slot < L && sub == 0) ring_sg[q & 1][slot] = (int)ss;
          if (slot < L) {
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
          if (slot < L) {
            const int from = slot + 1 < L ? slot + 1 : 0;
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
                const double2 a = ring[(j * 32 + from) * LPS + sub];
                const double2 b = ring[((RPL / 2 + j) * 32 + from) * LPS + sub];
                rs[2 * j] = a.x;
                rs[2 * j + 1] = a.y;
                ws[2 * j] = b.x;
                ws[2 * j + 1] = b.y;
              }
            }
          }
        }
      }
      __syncthreads();
      // write the columns back: slot k holds second-block column (k + L - 1) mod L
      const int sfin = (slot + L - 1) % L;
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
    if (cnt) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    const int c_all = s_cnt;
    __syncthreads();
    if (tid == 0) s_cnt = 0;
    total += c_all;
    if (c_all == 0) break;
    __syncthreads();
  }
  if (s_bad && tid == 0) atomicOr(soft ? &st->soft_fail : &st->breakdown, 1);

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
                      int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                      hipStream_t stream, const Batch& b) {
  hipLaunchKernelGGL((k_pivot<false, kPivotLPS>), dim3(pl.count), dim3(32 * kPivotLPS), 0, stream, part, nch, n,
                     rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, inner_max, inner_mode, soft, W, rotflag, st, b);
}

void launch_pivot_c128(const double* part, int nch, int n, int rows_per_chunk, const PivotList& pl, double tol,
                       int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                       hipStream_t stream, const Batch& b) {
  hipLaunchKernelGGL((k_pivot<true, kPivotLPS>), dim3(pl.count), dim3(32 * kPivotLPS), 0, stream, part, nch, n,
                     rows_per_chunk, pl.m, pl.nfirst, pl.sg, tol, inner_max, inner_mode, soft, W, rotflag, st, b);
}

}  // namespace jj
