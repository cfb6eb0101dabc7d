/* Seeded synthetic inputs with a known spectrum for the J-Jacobi eigensolver.
 *
 * This module only builds inputs.  It holds none of the eigensolver's
 * arithmetic and is shared by the tests (which feed its output both to the CPU
 * oracle and to the GPU library), the smoke check and the benchmark.
 *
 * Construction (the known-spectrum construction G = Q diag(sqrt|lambda|) W):
 *   J      : p entries +1 and n-p entries -1, in a seeded random order.
 *   lambda : |lambda_i| log-uniform in [lo, hi], lambda_i = j_i |lambda_i|.
 *   W      : a product of `nrot` random J-unitary plane rotations acting on
 *            column pairs (r, s), r != s uniform: trigonometric with a uniform
 *            angle when j_r = j_s, hyperbolic [ch sh; sh ch] with
 *            phi ~ U[-1, 1] when j_r != j_s; complex inputs first multiply
 *            column r by a uniform phase.  W^* J W = J, so G J G^* = Q diag(lambda) Q^*.
 *   Q      : Haar-distributed orthogonal/unitary, as a product of Householder
 *            reflectors of decreasing size, each mapping e_k to a uniformly
 *            distributed unit vector (G. W. Stewart, SIAM J. Numer. Anal. 17, 1980).
 *
 * Determinism: every random number is a pure function of (seed, stream, index)
 * through the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014), and
 * the only floating-point operations are +, -, *, / and sqrt, evaluated in a fixed
 * order (exp and log below are written out with those operations).  The same
 * binary therefore produces bit-identical inputs on any x86-64 host and for any
 * thread count.  Build with -O2 -ffp-contract=off (no FMA contraction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- counter-based random numbers ---------------- */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static uint64_t rnd_u64(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t key = mix64(seed * 0x9E3779B97F4A7C15ULL + stream + 1);
  return mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
}
/* uniform in [0, 1) with 53 random bits */
static double rnd_u01(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return (double)(rnd_u64(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------- exp / log from +,-,*,/ only ---------------- */
static const double LN2 = 0.69314718055994530942;
static double gen_exp(double x) {
  /* x = k ln2 + r, |r| <= ln2/2; exp(r) by its Taylor series */
  double kf = floor(x / LN2 + 0.5);
  double r = x - kf * LN2;
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 30; i++) {
    term = term * r / (double)i;
    sum = sum + term;
  }
  return ldexp(sum, (int)kf);
}
static double gen_log(double x) {
  /* x = m 2^e, m in [0.5, 1); ln m = 2 atanh(z), z = (m-1)/(m+1) */
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752) { m = 2.0 * m; e = e - 1; }
  double z = (m - 1.0) / (m + 1.0), z2 = z * z, zp = z, sum = 0.0;
  for (int i = 0; i < 40; i++) {
    sum = sum + zp / (double)(2 * i + 1);
    zp = zp * z2;
  }
  return (double)e * LN2 + 2.0 * sum;
}

/* standard normal by Marsaglia's polar method; attempt counter in the low bits */
static double rnd_normal(uint64_t seed, uint64_t stream, uint64_t ctr) {
  for (uint64_t a = 0;; a++) {
    double u = 2.0 * rnd_u01(seed, stream, (ctr << 12) + 2 * a) - 1.0;
    double v = 2.0 * rnd_u01(seed, stream, (ctr << 12) + 2 * a + 1) - 1.0;
    double s = u * u + v * v;
    if (s > 0.0 && s < 1.0) return u * sqrt(-2.0 * gen_log(s) / s);
  }
}
/* uniformly distributed point on the unit circle (cos, sin of a uniform angle) */
static void rnd_circle(uint64_t seed, uint64_t stream, uint64_t ctr, double* c, double* s) {
  for (uint64_t a = 0;; a++) {
    double u = 2.0 * rnd_u01(seed, stream, (ctr << 12) + 2 * a) - 1.0;
    double v = 2.0 * rnd_u01(seed, stream, (ctr << 12) + 2 * a + 1) - 1.0;
    double q = u * u + v * v;
    if (q > 1e-6 && q < 1.0) {
      double r = sqrt(q);
      *c = u / r;
      *s = v / r;
      return;
    }
  }
}

enum { ST_SIGNS = 1, ST_SHUFFLE, ST_LAMBDA, ST_ROT, ST_REFL, ST_LASTSIGN };

/* Fill J (p positives in seeded random order) and prescribed eigenvalues. */
static void make_signs_and_spectrum(int n, int p, double lo, double hi, uint64_t seed,
                                    signed char* J, double* lam) {
  for (int i = 0; i < n; i++) J[i] = (signed char)(i < p ? 1 : -1);
  for (int i = n - 1; i > 0; i--) { /* Fisher-Yates */
    int k = (int)(rnd_u01(seed, ST_SHUFFLE, (uint64_t)i) * (double)(i + 1));
    if (k > i) k = i;
    signed char t = J[i];
    J[i] = J[k];
    J[k] = t;
  }
  double llo = gen_log(lo), lhi = gen_log(hi);
  for (int i = 0; i < n; i++) {
    double u = rnd_u01(seed, ST_LAMBDA, (uint64_t)i);
    lam[i] = (double)J[i] * gen_exp(llo + u * (lhi - llo));
  }
}

/* B (n x n, column-major, complex interleaved if cplx) = diag(sqrt|lam|) W */
static void make_B(int n, int cplx, const signed char* J, const double* lam, int nrot,
                   uint64_t seed, double* B) {
  int w = cplx ? 2 : 1;
  memset(B, 0, sizeof(double) * (size_t)w * n * n);
  for (int i = 0; i < n; i++) B[w * ((size_t)i * n + i)] = sqrt(fabs(lam[i]));
  if (n < 2) return;
  for (int k = 0; k < nrot; k++) {
    uint64_t c0 = (uint64_t)k * 8;
    int r = (int)(rnd_u01(seed, ST_ROT, c0) * n);
    if (r >= n) r = n - 1;
    int s = (int)(rnd_u01(seed, ST_ROT, c0 + 1) * (n - 1));
    if (s >= n - 1) s = n - 2;
    if (s >= r) s++;
    double* br = B + (size_t)w * r * n;
    double* bs = B + (size_t)w * s * n;
    if (cplx) { /* column r times e^{i alpha} */
      double ca, sa;
      rnd_circle(seed, ST_ROT, c0 + 2, &ca, &sa);
      for (int i = 0; i < n; i++) {
        double re = br[2 * i], im = br[2 * i + 1];
        br[2 * i] = ca * re - sa * im;
        br[2 * i + 1] = sa * re + ca * im;
      }
    }
    double m00, m01, m10, m11; /* [b_r b_s] <- [b_r b_s] [m00 m01; m10 m11] */
    if (J[r] == J[s]) {
      double c, sn;
      rnd_circle(seed, ST_ROT, c0 + 3, &c, &sn);
      m00 = c; m01 = sn; m10 = -sn; m11 = c;
    } else {
      double phi = 2.0 * rnd_u01(seed, ST_ROT, c0 + 4) - 1.0;
      double ep = gen_exp(phi), em = 1.0 / ep;
      double ch = 0.5 * (ep + em), sh = 0.5 * (ep - em);
      m00 = ch; m01 = sh; m10 = sh; m11 = ch;
    }
    for (int i = 0; i < w * n; i++) {
      double x = br[i], y = bs[i];
      br[i] = m00 * x + m10 * y;
      bs[i] = m01 * x + m11 * y;
    }
  }
}

/* dot of length m with four interleaved partial sums combined in a fixed order */
static double dot4(const double* a, const double* b, int m) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int i = 0;
  for (; i + 3 < m; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < m; i++) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

/* G = Q B with Q Haar: Q = H_0 diag(1,H_1) ... diag(I_{n-1}, d), where H_k maps
 * e_k to x_k/||x_k||, x_k ~ N(0, I_{n-k}) (complex: standard complex normal). */
static void apply_haar(int n, int cplx, uint64_t seed, double* G, int nthreads) {
  int w = cplx ? 2 : 1;
  /* reflector k: v (length n-k, scalar type), beta = 2/(v^* v), omega = -x0/|x0| */
  size_t* off = (size_t*)malloc(sizeof(size_t) * (n + 1));
  off[0] = 0;
  for (int k = 0; k < n; k++) off[k + 1] = off[k] + (size_t)w * (n - k);
  double* V = (double*)malloc(sizeof(double) * (off[n] ? off[n] : 1));
  double* beta = (double*)malloc(sizeof(double) * n);
  double* omg = (double*)malloc(sizeof(double) * 2 * n);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int k = 0; k < n; k++) {
    int m = n - k;
    double* v = V + off[k];
    double nx2 = 0;
    for (int i = 0; i < w * m; i++) {
      uint64_t ctr = ((uint64_t)k << 24) + (uint64_t)i;
      double x = rnd_normal(seed, ST_REFL, ctr);
      if (cplx) x = x * 0.70710678118654752;
      v[i] = x;
      nx2 += x * x;
    }
    double nx = sqrt(nx2);
    double a0 = cplx ? sqrt(v[0] * v[0] + v[1] * v[1]) : fabs(v[0]);
    double ph_re, ph_im; /* x0/|x0| */
    if (a0 > 0) {
      ph_re = v[0] / a0;
      ph_im = cplx ? v[1] / a0 : 0.0;
    } else {
      ph_re = 1.0;
      ph_im = 0.0;
    }
    if (m == 1) { /* 1x1 block: multiply by the phase of x0 (maps e to x/|x|) */
      beta[k] = 0.0;
      omg[2 * k] = ph_re;
      omg[2 * k + 1] = ph_im;
      continue;
    }
    /* v = x + (x0/|x0|) ||x|| e_0 ; H = -(x0/|x0|) (I - beta v v^*) satisfies H e_0 = x/||x|| */
    v[0] += ph_re * nx;
    if (cplx) v[1] += ph_im * nx;
    double vv = 0;
    for (int i = 0; i < w * m; i++) vv += v[i] * v[i];
    beta[k] = 2.0 / vv;
    omg[2 * k] = -ph_re;
    omg[2 * k + 1] = -ph_im;
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
  for (int j = 0; j < n; j++) {
    double* x = G + (size_t)w * j * n;
    for (int k = n - 1; k >= 0; k--) {
      int m = n - k;
      double* y = x + (size_t)w * k;
      const double* v = V + off[k];
      double ore = omg[2 * k], oim = omg[2 * k + 1];
      if (!cplx) {
        if (m > 1) {
          double tau = beta[k] * dot4(v, y, m);
          for (int i = 0; i < m; i++) y[i] = y[i] - tau * v[i];
        }
        for (int i = 0; i < m; i++) y[i] = ore * y[i];
      } else {
        if (m > 1) {
          /* tau = beta v^* y (complex) */
          double tr = 0, ti = 0;
          for (int i = 0; i < m; i++) {
            tr += v[2 * i] * y[2 * i] + v[2 * i + 1] * y[2 * i + 1];
            ti += v[2 * i] * y[2 * i + 1] - v[2 * i + 1] * y[2 * i];
          }
          tr *= beta[k];
          ti *= beta[k];
          for (int i = 0; i < m; i++) {
            double vr = v[2 * i], vi = v[2 * i + 1];
            y[2 * i] = y[2 * i] - (tr * vr - ti * vi);
            y[2 * i + 1] = y[2 * i + 1] - (tr * vi + ti * vr);
          }
        }
        for (int i = 0; i < m; i++) {
          double re = y[2 * i], im = y[2 * i + 1];
          y[2 * i] = ore * re - oim * im;
          y[2 * i + 1] = ore * im + oim * re;
        }
      }
    }
  }
  free(off);
  free(V);
  free(beta);
  free(omg);
}

/* Build one input.
 *   n, cplx      order and scalar kind (0 real, 1 complex)
 *   p            number of +1 entries in J (0..n)
 *   lo, hi       |lambda| range, 0 < lo <= hi
 *   nrot         number of random J-unitary rotations in W
 *   seed         64-bit seed
 *   haar         1: G = Q diag(sqrt|lambda|) W with Haar Q; 0: G = diag(sqrt|lambda|) W
 * Outputs: J[n], lam[n] (prescribed eigenvalues, lam[i] belongs to column i of
 * Q), G (n x n column-major; complex interleaved (re, im)).
 * Returns 0, or -1 on invalid arguments. */
int jjgen_make(int n, int cplx, int p, double lo, double hi, int nrot, unsigned long long seed,
               int haar, signed char* J, double* lam, double* G, int nthreads) {
  if (n < 0 || p < 0 || p > n || !(lo > 0) || !(hi >= lo) || nrot < 0) return -1;
  if (n == 0) return 0;
  if (nthreads < 1) nthreads = 1;
  make_signs_and_spectrum(n, p, lo, hi, (uint64_t)seed, J, lam);
  make_B(n, cplx, J, lam, nrot, (uint64_t)seed, G);
  if (haar) apply_haar(n, cplx, (uint64_t)seed, G, nthreads);
  return 0;
}

/* Uniform doubles in [0,1) and integers in [lo, hi] for Python-side recipes
 * (batch sizes, inertia draws) that must match across hosts. */
void jjgen_uniform(unsigned long long seed, unsigned long long stream, long long count, double* out) {
  for (long long i = 0; i < count; i++) out[i] = rnd_u01((uint64_t)seed, 1000 + (uint64_t)stream, (uint64_t)i);
}
