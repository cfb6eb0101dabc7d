// Front end of the method on gfx950: the factorization H = G J G^* of a
// Hermitian H (paper, Section 2.2, eq. 2.5).
//
// Bunch-Parlett factorization with complete pivoting, P H P^T = M D M^*
// (M unit lower triangular, D block diagonal with blocks of order 1 and 2),
// then each 2x2 block of D is diagonalised and the columns of M are scaled:
// G' = M Q |Lambda|^{1/2}, J = sign(Lambda), G = P^T G'.  If the trailing
// matrix becomes negligible after r columns (|s_ij| <= tol max|h_ij| for all
// its entries), H has rank r and G is n x r of full column rank (the last
// paragraphs of Section 2.2).
//
// Pivot rule (Bunch and Parlett's complete pivoting): on the trailing matrix
// S, mu0 = max |s_ij|, mu1 = max |s_ii|, alpha = (1 + sqrt 17) / 8; a 1x1 pivot
// on the largest diagonal entry if mu1 >= alpha mu0, otherwise a 2x2 pivot on
// the largest entry (p, q), p > q, with q moved to position k and p to k + 1.
// Ties go to the entry with the smallest column-major index (the first met
// scanning the lower triangle column by column).
//
// Storage and launches: H is copied into a workspace A (n x n, column-major);
// only its lower triangle is used.  Columns of M overwrite the lower triangle
// as they are formed (LAPACK's layout), symmetric interchanges are applied to
// the lower triangle and to the rows of the finished columns of M.  One step is
// two launches:
//   k_bp_select (one workgroup): reduces the per-workgroup maxima of the
//       trailing matrix left by the previous launch, picks the pivot, applies
//       the interchanges, forms the column(s) of M and keeps the unscaled
//       pivot column(s) for the update;
//   k_bp_update (a fixed grid of kBpGroups workgroups striding over 256 x 8
//       tiles of the trailing lower triangle): the rank-1 or rank-2 Schur
//       update, fused with the search for the next step's maxima.
// The step count is data dependent (2x2 pivots take two columns); every step
// reads the state from device memory, so the host enqueues n + 1 steps and the
// launches past the end return at once.  k_bp_build_g forms G from M and D.
//
// The arithmetic follows the oracle's order of operations (no contraction into
// fused multiply-adds; complex products as (ac - bd, ad + bc)), so decisions
// taken on equal data are the same.
#include <hip/hip_runtime.h>

#include "jj_device.h"

namespace jj {

// modulus of a real (w = 1) or complex (w = 2) entry
__device__ __forceinline__ double absv(double re, double im, int w) { return w == 2 ? hypot(re, im) : fabs(re); }

// maxima of a set of entries: mu0 over all entries with its column-major index,
// mu1 over diagonal entries with its row index; ties to the smaller index
__device__ __forceinline__ void bp_better(double v, long long idx, double& best, long long& bidx) {
  if (v > best || (v == best && idx < bidx)) {
    best = v;
    bidx = idx;
  }
}

__global__ __launch_bounds__(kBpThreads) void k_bp_update(double* __restrict__ A, int n, int w,
                                                          const double* __restrict__ pcol, BPState* st,
                                                          BPPartial* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double s_mu0[kBpThreads], s_mu1[kBpThreads];
  __shared__ long long s_i0[kBpThreads], s_i1[kBpThreads];
  const int tid = threadIdx.x;
  const int done = st->done;
  const int kc = st->kcur, s = st->s;
  const int k1 = kc + s;  // first row / column of the trailing matrix after this update
  double mu0 = -1.0, mu1 = -1.0;
  long long i0 = 0x7fffffffffffffffll, i1 = 0x7fffffffffffffffll;
  int bad = 0;
  if (!done && k1 < n) {
    const int t = n - k1;
    const int ncb = (t + 7) >> 3, nrb = (t + kBpThreads - 1) / kBpThreads;
    const long long ntiles = (long long)ncb * nrb;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      const int cb = (int)(tile / nrb), rb = (int)(tile % nrb);
      const int j0 = k1 + 8 * cb;
      const int i = k1 + kBpThreads * rb + tid;
      if (k1 + kBpThreads * rb + kBpThreads - 1 < j0) continue;  // tile above the diagonal
      if (i >= n) continue;
      double l1r = 0, l1i = 0, l2r = 0, l2i = 0;
      if (s >= 1) {
        l1r = A[((size_t)kc * n + i) * w];
        if (w == 2) l1i = A[((size_t)kc * n + i) * w + 1];
      }
      if (s == 2) {
        l2r = A[((size_t)(kc + 1) * n + i) * w];
        if (w == 2) l2i = A[((size_t)(kc + 1) * n + i) * w + 1];
      }
      const int jend = min(j0 + 8, n);
      for (int j = j0; j < jend && j <= i; j++) {
        double* a = A + ((size_t)j * n + i) * w;
        double vr = a[0], vi = w == 2 ? a[1] : 0.0;
        if (s >= 1) {
          // s_ij -= l_i1 conj(p_j1) [+ l_i2 conj(p_j2)], p the unscaled pivot columns
          const double p1r = pcol[(size_t)j * 2 * w], p1i = w == 2 ? -pcol[(size_t)j * 2 * w + 1] : 0.0;
          double tr, ti;
          if (w == 2) {
            tr = l1r * p1r - l1i * p1i;
            ti = l1r * p1i + l1i * p1r;
          } else {
            tr = l1r * p1r;
            ti = 0.0;
          }
          if (s == 2) {
            const double p2r = pcol[(size_t)j * 2 * w + w], p2i = w == 2 ? -pcol[(size_t)j * 2 * w + w + 1] : 0.0;
            if (w == 2) {
              tr = tr + (l2r * p2r - l2i * p2i);
              ti = ti + (l2r * p2i + l2i * p2r);
            } else {
              tr = tr + l2r * p2r;
            }
          }
          vr = vr - tr;
          vi = vi - ti;
          if (i == j) vi = 0.0;
          a[0] = vr;
          if (w == 2) a[1] = vi;
        } else if (i == j) {
          vi = 0.0;  // the imaginary part of a Hermitian diagonal is not read
        }
        if (!isfinite(vr) || !isfinite(vi)) bad = 1;
        const double av = absv(vr, vi, w);
        bp_better(av, (long long)j * n + i, mu0, i0);
        if (i == j) bp_better(av, i, mu1, i1);
      }
    }
  }
  if (bad) atomicOr(&st->nonfinite, 1);
  s_mu0[tid] = mu0;
  s_i0[tid] = i0;
  s_mu1[tid] = mu1;
  s_i1[tid] = i1;
  __syncthreads();
  for (int h = kBpThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      bp_better(s_mu0[tid + h], s_i0[tid + h], s_mu0[tid], s_i0[tid]);
      bp_better(s_mu1[tid + h], s_i1[tid + h], s_mu1[tid], s_i1[tid]);
    }
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = BPPartial{s_mu0[0], s_i0[0], s_mu1[0], s_i1[0]};
}

// symmetric interchange of positions a < b in the lower-triangle storage of A
// at step k: rows of M (columns < k) and of the trailing columns left of a,
// the diagonal, column a against row b between them, and the columns below b
__device__ void bp_swap(double* A, int n, int w, int* perm, int a, int b) {
  const int tid = threadIdx.x;
  if (a != b) {
    for (int c = tid; c < a; c += kBpThreads)
      for (int q = 0; q < w; q++) {
        double* x = A + ((size_t)c * n + a) * w + q;
        double* y = A + ((size_t)c * n + b) * w + q;
        const double t = *x;
        *x = *y;
        *y = t;
      }
    for (int i = a + 1 + tid; i < b; i += kBpThreads) {
      // (i, a) <-> conj((b, i))
      double* x = A + ((size_t)a * n + i) * w;
      double* y = A + ((size_t)i * n + b) * w;
      const double xr = x[0], yr = y[0];
      x[0] = yr;
      y[0] = xr;
      if (w == 2) {
        const double xi = x[1], yi = y[1];
        x[1] = -yi;
        y[1] = -xi;
      }
    }
    for (int i = b + 1 + tid; i < n; i += kBpThreads)
      for (int q = 0; q < w; q++) {
        double* x = A + ((size_t)a * n + i) * w + q;
        double* y = A + ((size_t)b * n + i) * w + q;
        const double t = *x;
        *x = *y;
        *y = t;
      }
    if (tid == 0) {
      double* da = A + ((size_t)a * n + a) * w;
      double* db = A + ((size_t)b * n + b) * w;
      const double t = da[0];
      da[0] = db[0];
      db[0] = t;
      if (w == 2) A[((size_t)a * n + b) * w + 1] = -A[((size_t)a * n + b) * w + 1];  // (b, a) conjugated
      const int pt = perm[a];
      perm[a] = perm[b];
      perm[b] = pt;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBpThreads) void k_bp_select(double* __restrict__ A, int n, int w, double tol,
                                                          double* __restrict__ pcol, BPState* st,
                                                          const BPPartial* __restrict__ part, int nparts,
                                                          int* __restrict__ perm, int* __restrict__ piv,
                                                          double* __restrict__ dblk) {
#pragma clang fp contract(off)
  __shared__ double s_mu0[kBpThreads], s_mu1[kBpThreads];
  __shared__ long long s_i0[kBpThreads], s_i1[kBpThreads];
  __shared__ int s_go;
  const int tid = threadIdx.x;
  if (st->done) return;
  double mu0 = -1.0, mu1 = -1.0;
  long long i0 = 0x7fffffffffffffffll, i1 = 0x7fffffffffffffffll;
  for (int q = tid; q < nparts; q += kBpThreads) {
    const BPPartial p = part[q];
    bp_better(p.mu0, p.idx0, mu0, i0);
    bp_better(p.mu1, p.idx1, mu1, i1);
  }
  s_mu0[tid] = mu0;
  s_i0[tid] = i0;
  s_mu1[tid] = mu1;
  s_i1[tid] = i1;
  __syncthreads();
  for (int h = kBpThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      bp_better(s_mu0[tid + h], s_i0[tid + h], s_mu0[tid], s_i0[tid]);
      bp_better(s_mu1[tid + h], s_i1[tid + h], s_mu1[tid], s_i1[tid]);
    }
    __syncthreads();
  }
  mu0 = s_mu0[0];
  mu1 = s_mu1[0];
  const long long idx0 = s_i0[0];
  const int idx1 = (int)s_i1[0];
  const int k = st->k;
  if (tid == 0) {
    if (k == 0) st->hmax = mu0;
    const double hmax = k == 0 ? mu0 : st->hmax;
    s_go = (k < n && !st->nonfinite && mu0 > tol * hmax) ? 1 : 0;
    if (!s_go) {
      st->done = 1;
      st->rank = k;
      st->s = 0;
    }
  }
  __syncthreads();
  if (!s_go) return;
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  const bool one = mu1 >= alpha * mu0;
  if (one) {
    bp_swap(A, n, w, perm, k, idx1);
    const double d = A[((size_t)k * n + k) * w];
    for (int i = k + 1 + tid; i < n; i += kBpThreads) {
      double* a = A + ((size_t)k * n + i) * w;
      pcol[(size_t)i * 2 * w] = a[0];
      a[0] = a[0] / d;
      if (w == 2) {
        pcol[(size_t)i * 2 * w + 1] = a[1];
        a[1] = a[1] / d;
      }
    }
    if (tid == 0) {
      piv[k] = 1;
      dblk[(size_t)k * 2] = d;
      st->kcur = k;
      st->s = 1;
      st->k = k + 1;
    }
  } else {
    const int p0 = (int)(idx0 % n), q0 = (int)(idx0 / n);  // p0 > q0 >= k
    bp_swap(A, n, w, perm, k, q0);
    bp_swap(A, n, w, perm, k + 1, p0);
    const double e11 = A[((size_t)k * n + k) * w];
    const double e22 = A[((size_t)(k + 1) * n + k + 1) * w];
    const double br = A[((size_t)k * n + k + 1) * w], bi = w == 2 ? A[((size_t)k * n + k + 1) * w + 1] : 0.0;
    const double ab = absv(br, bi, w);
    const double det = e11 * e22 - ab * ab;
    for (int i = k + 2 + tid; i < n; i += kBpThreads) {
      double* x = A + ((size_t)k * n + i) * w;
      double* y = A + ((size_t)(k + 1) * n + i) * w;
      const double xr = x[0], xi = w == 2 ? x[1] : 0.0, yr = y[0], yi = w == 2 ? y[1] : 0.0;
      pcol[(size_t)i * 2 * w] = xr;
      pcol[(size_t)i * 2 * w + w] = yr;
      if (w == 2) {
        pcol[(size_t)i * 2 * w + 1] = xi;
        pcol[(size_t)i * 2 * w + w + 1] = yi;
        // l1 = (x e22 - y b) / det, l2 = (y e11 - x conj(b)) / det
        const double ybr = yr * br - yi * bi, ybi = yr * bi + yi * br;
        const double xcr = xr * br - xi * (-bi), xci = xr * (-bi) + xi * br;
        x[0] = (xr * e22 - ybr) / det;
        x[1] = (xi * e22 - ybi) / det;
        y[0] = (yr * e11 - xcr) / det;
        y[1] = (yi * e11 - xci) / det;
      } else {
        x[0] = (xr * e22 - yr * br) / det;
        y[0] = (yr * e11 - xr * br) / det;
      }
    }
    if (tid == 0) {
      piv[k] = 2;
      piv[k + 1] = -2;  // second column of a 2x2 block
      dblk[(size_t)k * 2] = e11;
      dblk[(size_t)(k + 1) * 2] = e22;
      dblk[(size_t)k * 2 + 1] = 0.0;
      st->kcur = k;
      st->s = 2;
      st->k = k + 2;
    }
  }
}

// G[perm[i], c] = (M Q |Lambda|^{1/2})[i, c] for the first `rank` columns,
// J[c] = sign(Lambda_c); columns c >= rank are zeroed.  One workgroup per column.
__global__ __launch_bounds__(kBpThreads) void k_bp_build_g(const double* __restrict__ A, int n, int w,
                                                           const BPState* st, const int* __restrict__ perm,
                                                           const int* __restrict__ piv,
                                                           const double* __restrict__ dblk, double* __restrict__ G,
                                                           int ldg, signed char* __restrict__ J) {
#pragma clang fp contract(off)
  const int c = blockIdx.x, tid = threadIdx.x;
  const int r = st->rank;
  double* g = G + (size_t)c * ldg * w;
  if (c >= r) {
    for (int i = tid; i < n * w; i += kBpThreads) g[i] = 0.0;
    if (tid == 0) J[c] = 0;
    return;
  }
  const int pv = piv[c];
  if (pv == 1) {
    const double d = dblk[(size_t)c * 2];
    const double sq = sqrt(fabs(d));
    for (int i = tid; i < n; i += kBpThreads) {
      double mr = 0.0, mi = 0.0;
      if (i == c) {
        mr = 1.0;
      } else if (i > c) {
        mr = A[((size_t)c * n + i) * w];
        if (w == 2) mi = A[((size_t)c * n + i) * w + 1];
      }
      double* o = G + ((size_t)c * ldg + perm[i]) * w;
      o[0] = mr * sq;
      if (w == 2) o[1] = mi * sq;
    }
    if (tid == 0) J[c] = d > 0.0 ? 1 : -1;
    return;
  }
  // 2x2 block at (c0, c0 + 1): E = [a conj(b); b e], diagonalised by one rotation
  const int c0 = pv == 2 ? c : c - 1;
  const double a = dblk[(size_t)c0 * 2], e = dblk[(size_t)(c0 + 1) * 2];
  const double br = A[((size_t)c0 * n + c0 + 1) * w], bi = w == 2 ? A[((size_t)c0 * n + c0 + 1) * w + 1] : 0.0;
  const double ab = absv(br, bi, w);
  const double phr = br / ab, phi = w == 2 ? bi / ab : 0.0;
  const double zeta = (e - a) / (2.0 * ab);
  const double t = (zeta < 0.0 ? -1.0 : 1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  const double mu = pv == 2 ? a - t * ab : e + t * ab;
  const double sq = sqrt(fabs(mu));
  for (int i = tid; i < n; i += kBpThreads) {
    // columns of M: l1 (unit at c0, zero at c0 + 1), l2 (unit at c0 + 1)
    double l1r = 0.0, l1i = 0.0, l2r = 0.0, l2i = 0.0;
    if (i == c0) {
      l1r = 1.0;
    } else if (i == c0 + 1) {
      l2r = 1.0;
    } else if (i > c0 + 1) {
      l1r = A[((size_t)c0 * n + i) * w];
      l2r = A[((size_t)(c0 + 1) * n + i) * w];
      if (w == 2) {
        l1i = A[((size_t)c0 * n + i) * w + 1];
        l2i = A[((size_t)(c0 + 1) * n + i) * w + 1];
      }
    }
    double gr, gi;
    if (pv == 2) {
      // (l1 cs - l2 (sn ph)) s1
      const double qr = sn * phr, qi = sn * phi;
      const double pr = w == 2 ? l2r * qr - l2i * qi : l2r * qr;
      const double pi = w == 2 ? l2r * qi + l2i * qr : 0.0;
      gr = (l1r * cs - pr) * sq;
      gi = (l1i * cs - pi) * sq;
    } else {
      // (l1 sn + l2 (cs ph)) s2
      const double qr = cs * phr, qi = cs * phi;
      const double pr = w == 2 ? l2r * qr - l2i * qi : l2r * qr;
      const double pi = w == 2 ? l2r * qi + l2i * qr : 0.0;
      gr = (l1r * sn + pr) * sq;
      gi = (l1i * sn + pi) * sq;
    }
    double* o = G + ((size_t)c * ldg + perm[i]) * w;
    o[0] = gr;
    if (w == 2) o[1] = gi;
  }
  if (tid == 0) J[c] = mu > 0.0 ? 1 : -1;
}

__global__ void k_bp_init(BPState* st, int* perm, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = i;
  if (i == 0) {
    st->k = 0;
    st->done = 0;
    st->kcur = 0;
    st->s = 0;
    st->rank = 0;
    st->hmax = 0.0;
    st->nonfinite = 0;
  }
}

// ---- null space of a singular H (Section 2.2, last paragraph): Householder QR
// of U~ (n x r) and the last n - r columns of its Q ----

// fixed-order sum over the workgroup (kBpThreads values in LDS)
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int h = kBpThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Reflector of x = A[k:, k]: v = x - alpha e_1, alpha = -e^{i arg x_k} ||x||
// (sgn 0 = +1), beta = ||v||^2; v (zero above row k) to Vh[:, k].  One workgroup.
__global__ __launch_bounds__(kBpThreads) void k_hh_reflector(const double* __restrict__ A, int n, int lda, int w,
                                                             int k, double* __restrict__ Vh, double* __restrict__ beta) {
  __shared__ double red[kBpThreads];
  const int tid = threadIdx.x;
  const double* x = A + (size_t)k * lda * w;
  double* v = Vh + (size_t)k * n * w;
  double s2 = 0.0;
  for (int i = k + tid; i < n; i += kBpThreads) {
    const double xr = x[(size_t)i * w], xi = w == 2 ? x[(size_t)i * w + 1] : 0.0;
    s2 += xr * xr + xi * xi;
  }
  const double nx = sqrt(block_sum(s2, red));
  const double x0r = x[(size_t)k * w], x0i = w == 2 ? x[(size_t)k * w + 1] : 0.0;
  const double a0 = w == 2 ? hypot(x0r, x0i) : fabs(x0r);
  const double phr = a0 > 0.0 ? x0r / a0 : 1.0, phi = a0 > 0.0 ? x0i / a0 : 0.0;
  double b2 = 0.0;
  for (int i = tid; i < n; i += kBpThreads) {
    double vr = 0.0, vi = 0.0;
    if (i > k) {
      vr = x[(size_t)i * w];
      vi = w == 2 ? x[(size_t)i * w + 1] : 0.0;
    } else if (i == k) {
      vr = x0r + phr * nx;
      vi = x0i + phi * nx;
    }
    v[(size_t)i * w] = vr;
    if (w == 2) v[(size_t)i * w + 1] = vi;
    b2 += vr * vr + vi * vi;
  }
  const double b = block_sum(b2, red);
  if (tid == 0) beta[k] = b;
}

// M[:, j] -= (2 / beta_k) v_k (v_k^* M[:, j]) over rows k..n-1, for the ncols
// columns starting at col0; one workgroup per column.
__global__ __launch_bounds__(kBpThreads) void k_hh_apply(double* __restrict__ M, int n, int ldm, int w, int col0,
                                                         const double* __restrict__ Vh, const double* __restrict__ beta,
                                                         int k) {
  __shared__ double red[kBpThreads];
  const int tid = threadIdx.x;
  const double b = beta[k];
  if (!(b > 0.0)) return;
  double* m = M + (size_t)(col0 + blockIdx.x) * ldm * w;
  const double* v = Vh + (size_t)k * n * w;
  double sr = 0.0, si = 0.0;
  for (int i = k + tid; i < n; i += kBpThreads) {
    const double vr = v[(size_t)i * w], vi = w == 2 ? v[(size_t)i * w + 1] : 0.0;
    const double mr = m[(size_t)i * w], mi = w == 2 ? m[(size_t)i * w + 1] : 0.0;
    sr += vr * mr + vi * mi;  // conj(v) m
    si += vr * mi - vi * mr;
  }
  sr = block_sum(sr, red);
  if (w == 2) si = block_sum(si, red);
  const double fr = sr * (2.0 / b), fi = si * (2.0 / b);
  for (int i = k + tid; i < n; i += kBpThreads) {
    const double vr = v[(size_t)i * w], vi = w == 2 ? v[(size_t)i * w + 1] : 0.0;
    m[(size_t)i * w] -= vr * fr - vi * fi;
    if (w == 2) m[(size_t)i * w + 1] -= vr * fi + vi * fr;
  }
}

// E (n x ncols, ld lde) = rows r.. of the identity: E[i, c] = (i == r + c)
__global__ void k_identity_tail(double* __restrict__ E, int n, int lde, int w, int r) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    E[((size_t)c * lde + i) * w] = i == r + c ? 1.0 : 0.0;
    if (w == 2) E[((size_t)c * lde + i) * w + 1] = 0.0;
  }
}

void launch_identity_tail(int cplx, double* E, int n, int lde, int r, hipStream_t stream) {
  if (n > r) launch(k_identity_tail, dim3(n - r), dim3(256), 0, stream, E, n, lde, cplx ? 2 : 1, r);
}

void launch_nullspace(int cplx, double* A, int n, int r, double* Vh, double* beta, double* E, int lde,
                      hipStream_t stream) {
  const int w = cplx ? 2 : 1;
  for (int k = 0; k < r; k++) {
    launch(k_hh_reflector, dim3(1), dim3(kBpThreads), 0, stream, (const double*)A, n, n, w, k, Vh, beta);
    launch(k_hh_apply, dim3(r - k), dim3(kBpThreads), 0, stream, A, n, n, w, k, (const double*)Vh,
           (const double*)beta, k);
  }
  launch(k_identity_tail, dim3(n - r), dim3(256), 0, stream, E, n, lde, w, r);
  for (int k = r - 1; k >= 0; k--)
    launch(k_hh_apply, dim3(n - r), dim3(kBpThreads), 0, stream, E, n, lde, w, 0, (const double*)Vh,
           (const double*)beta, k);
}

void launch_bp_init(BPState* st, int* perm, int n, hipStream_t stream) {
  launch(k_bp_init, dim3((n + 255) / 256), dim3(256), 0, stream, st, perm, n);
}

void launch_bp_update(double* A, int n, int cplx, const double* pcol, BPState* st, BPPartial* part,
                      hipStream_t stream) {
  launch(k_bp_update, dim3(kBpGroups), dim3(kBpThreads), 0, stream, A, n, cplx ? 2 : 1, pcol, st, part);
}

void launch_bp_select(double* A, int n, int cplx, double tol, double* pcol, BPState* st, const BPPartial* part,
                      int* perm, int* piv, double* dblk, hipStream_t stream) {
  launch(k_bp_select, dim3(1), dim3(kBpThreads), 0, stream, A, n, cplx ? 2 : 1, tol, pcol, st, part, kBpGroups,
         perm, piv, dblk);
}

void launch_bp_build_g(const double* A, int n, int cplx, const BPState* st, const int* perm, const int* piv,
                       const double* dblk, double* G, int ldg, signed char* J, hipStream_t stream) {
  launch(k_bp_build_g, dim3(n), dim3(kBpThreads), 0, stream, A, n, cplx ? 2 : 1, st, perm, piv, dblk, G, ldg, J);
}

}  // namespace jj
