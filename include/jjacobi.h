/* jjacobi.h -- C ABI of the MI355X (gfx950) one-sided hyperbolic J-Jacobi eigensolver.
 *
 * Problem (paper, Section 2.2-2.3, eq. 2.5-2.6 and 2.10-2.11): given a factor G
 * (n x n, full column rank) and J = diag(j_1..j_n), j_i = +-1, compute the
 * eigenpairs of the Hermitian matrix H = G J G^*.  The method applies J-unitary
 * transformations from the right, G <- G W (eq. 2.9 / 3.4), until the columns
 * of G are mutually orthogonal; then
 *     lambda_i = j_i * ||g_i||^2      and      v_i = g_i / ||g_i||
 * (eq. 2.10-2.11 and the final two lines of Algorithm 5.2).
 *
 * The blocked process (Sections 3.1-3.3, 4.2, 5.3): the columns are reordered so
 * that J = diag(I_nu, -I_{n-nu}) (Section 2.3, last paragraph), split into an
 * even number of almost equal blocks (eq. 3.2-3.3), and every sweep visits each
 * pair of blocks once in round-robin order, nblocks/2 disjoint pairs at a time.
 * Per pair: Gram block A_P = [G_i G_j]^* [G_i G_j] (eq. 3.6), Cholesky factor R
 * (eq. 3.8), one-sided J-Jacobi on R accumulating W_P (eq. 3.12, Algorithms
 * 3.1-3.2), and the update [G_i G_j] <- [G_i G_j] W_P (Section 3.3, last
 * paragraph before Algorithm 3.1).
 *
 * Conventions common to all entry points
 *   - Matrices are column-major.  G, V and lambda are DEVICE pointers owned by
 *     the caller; J is a HOST array of n signed chars, each +1 or -1.
 *   - Complex data (dtype 1) is interleaved (re, im) double pairs; ld counts
 *     complex elements.
 *   - G is overwritten (destroyed) by the solve.  V must not overlap G.
 *   - On return lambda[k], V[:,k] is the k-th eigenpair, sorted by lambda
 *     descending, ties broken by ascending input column index.
 *   - tol <= 0 selects tol = n * 2^-53: a column pair is rotated iff
 *     |g_r^* g_s| > tol * ||g_r|| * ||g_s||.  max_sweeps <= 0 selects 100.
 *   - Work is ordered on the stream given in jj_opts (NULL: the null stream);
 *     the call returns after the solve has completed on that stream.
 *   - The library keeps a cached device workspace per device (released by
 *     jjacobi_release_workspace); calls are serialised by an internal mutex.
 *
 * Return value (LAPACK style)
 *    0  converged
 *    1  not converged within max_sweeps (outputs are still written)
 *    2  numerical breakdown: G is numerically rank deficient (a pivot block
 *       Cholesky failed, a hyperbolic rotation did not exist, or a final column
 *       is zero)
 *    3  non-finite input
 *    4  HIP runtime error (jjacobi_status_string(4) gives the last message)
 *   -k  the k-th argument is invalid (null pointer, n < 0, ld < max(1, n),
 *       J[i] not +-1, unknown dtype, ...)
 */
#ifndef JJACOBI_H
#define JJACOBI_H

#ifdef __cplusplus
extern "C" {
#endif

#define JJ_OK 0
#define JJ_NOT_CONVERGED 1
#define JJ_BREAKDOWN 2
#define JJ_NONFINITE 3
#define JJ_HIP_ERROR 4
#define JJ_SCRATCH_TOO_SMALL 5 /* jjacobi_solve_noalloc only: see there */

#define JJ_F64 0 /* real double */
#define JJ_C128 1 /* complex double, interleaved */

/* Options.  Zero-initialised fields select the defaults noted. */
typedef struct jj_opts {
  void* stream;          /* hipStream_t to order the work on; NULL: null stream */
  int block_width;       /* target block width n_t of eq. 3.2: at most 32, or 64 for
                            three-level pivots (Section 5; plain FP64, block-oriented, no
                            diagonal pass; otherwise 32 is used); 0: library choice: 32, or
                            the fastest candidate (16, 32, and 64 for single solves) on the
                            first problem of each (dtype, size) class seen by the process,
                            timed over a whole solve up to n = 2048 and over two sweeps
                            above (each after one untimed sweep): single solves with
                            n >= 1024, every batched problem with n > 64 */
  int inner_max_sweeps;  /* cap on inner sweeps of one pivot solve (Algorithm 3.2 max_it);
                            0: 12 */
  int diag_pass;         /* diagonal-block pre-processing (Algorithm 3.3, first inner loop):
                            0: off (default), 1: first sweep only, 2: every sweep */
  int inner_mode;        /* 0: block-oriented (Section 3.4, Algorithm 5.1): the
                               first step of a sweep makes one full inner pass per
                               pivot, the other steps one pass over the off-diagonal
                               block;
                            1: full pivot diagonalisation (full block, Section 3.3),
                               up to inner_max_sweeps inner sweeps;
                            -1 (jjacobi_default_opts): library choice: tuned together
                               with the block width where the width is tuned (whole
                               solves of both variants up to n = 1024), else 0 */
  int precision;         /* 0: FP64 throughout; 1: mixed (FP32 Gram in pre-sweeps) */
  double mixed_switch;   /* mixed: the solve leaves its FP32-Gram sweeps after a sweep
                            whose max scaled off-diagonal is below this; 0: 0.1
                            (measured: the FP32 Gram's error slows the last,
                            quadratically converging sweeps, not the earlier ones) */
  int strategy;          /* 0: round-robin block pairing (Section 4.2);
                            1: modulus pairing (Section 4.1) */
  int profile;           /* 1: time every kernel launch with HIP events on the stream
                            (read back with jjacobi_last_profile) */
  double* history;       /* host array or NULL: entry k receives the largest scaled
                            off-diagonal |a_rs|/sqrt(a_rr a_ss) met in sweep k+1 */
  int history_len;       /* entries available in history */
  int step_groups;       /* graph-replayed sweeps: 0 or 1 (default): one step after the
                            other; G > 1: the pairs of a step are split into G groups and
                            each group's kernels depend only on the groups that last
                            touched its blocks (groups of consecutive steps may overlap;
                            same results; slower than 1 with the HIP runtime measured) */
  int reserved[7];
} jj_opts;

/* Per-solve report (all fields written when the pointer is non-NULL). */
typedef struct jj_info {
  int status;              /* same code as the return value */
  int sweeps;              /* block sweeps executed */
  int block_width;         /* largest block size used */
  int nblocks;             /* number of blocks */
  long long pivots_rotated;/* pivot blocks whose transformation was not the identity */
  double final_offdiag;    /* max scaled off-diagonal |a_rs|/sqrt(a_rr a_ss) seen by the
                              Gram checks of the last sweep */
  double seconds;          /* wall-clock time of the solve */
  int mixed_sweeps;        /* sweeps that used the FP32 Gram (precision 1) */
  int mixed_resolved;      /* pairs of blocks whose FP32 Gram block could not be factored
                              in those sweeps; each is left for that sweep and formed
                              and solved in FP64 in the later mixed sweeps */
  int rank;                /* jjacobi_eigh: rank of H found by the front end */
  int inner_mode;          /* inner mode used (0 block-oriented, 1 full) */
  int reserved[4];
} jj_info;

/* Fill *opts with the defaults. */
void jjacobi_default_opts(jj_opts* opts);

/* Real symmetric H = G J G^T, G float64 (n x n, leading dimension ldg), by the
 * blocked one-sided J-Jacobi process (Sections 3.3-3.4 and 5.3, Algorithm 5.2
 * on one device): lambda_i = j_i ||g~_i||^2, v_i = g~_i / ||g~_i|| (eq. 2.10-2.11).
 * lambda: n doubles; V: n x n doubles, leading dimension n.  Default options. */
int jjacobi_solve(double* G, const signed char* J, int n, int ldg, double* lambda, double* V,
                  double tol, int max_sweeps);

/* Complex Hermitian H = G J G^*, G complex128 interleaved (n x n, ldg): the
 * same process with complex rotations (eq. 2.3 and the complex hyperbolic
 * rotations of Section 2.3).  lambda: n doubles; V: n x n complex128, leading
 * dimension n.  Default options. */
int jjacobi_zsolve(void* G, const signed char* J, int n, int ldg, double* lambda, void* V,
                   double tol, int max_sweeps);

/* General form of the two above (Sections 2.3, 3 and 5): dtype JJ_F64 or
 * JJ_C128, V with leading dimension ldv >= n, options (nullable: defaults;
 * the pivot variants of Sections 3.3/3.4, the pairings of Section 4, the
 * diagonal-block pass of Algorithm 3.3) and report (nullable). */
int jjacobi_solve_ex(int dtype, void* G, const signed char* J, int n, int ldg, double* lambda,
                     void* V, int ldv, double tol, int max_sweeps, const jj_opts* opts,
                     jj_info* info);

/* The same solve with no device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, results and status codes are those of
 * jjacobi_solve_ex.  The workspace is a fixed device array inside the library
 * (JJ_NOALLOC_SCRATCH_BYTES per device, held until the process ends); no
 * hipMalloc, hipFree, stream, event or graph is created.  The kernels run
 * eagerly on opts->stream (NULL: the null stream), the block width is
 * opts->block_width or 32 (never timed), and opts->profile is ignored.
 * A solve whose workspace does not fit returns JJ_SCRATCH_TOO_SMALL before
 * any device work (jjacobi_status_string(5) gives the bytes it needs); it fits
 * for real n <= 4096 and complex n <= 2048 at the default block width without
 * the diagonal-block pass.  Every call on a device shares that device's array
 * and leaves its contents behind; the library's lock serialises calls within
 * a process and each call has finished on the device when it returns, so
 * calls that overlapped on one device (one in flight while another starts)
 * would race on it and are excluded by that lock. */
#define JJ_NOALLOC_SCRATCH_BYTES ((unsigned long long)32 << 20)
int jjacobi_solve_noalloc(int dtype, void* G, const signed char* J, int n, int ldg, double* lambda,
                          void* V, int ldv, double tol, int max_sweeps, const jj_opts* opts,
                          jj_info* info);

/* Rectangular factor (Section 2.2, last paragraphs): G has m >= n rows and n
 * columns of full column rank, e.g. the factor of a singular H = G J G^* of
 * rank n and order m.  lambda receives the n nonzero eigenvalues of H
 * (descending), V (m x n, leading dimension ldv >= m) their unit eigenvectors,
 * the columns of U~ in G W = U~ Sigma (the HSVD of G).  ldg >= m.  tol <= 0
 * selects m * 2^-53.  Otherwise as jjacobi_solve_ex (argument k of this
 * signature for status -k).  m = n is the square solve. */
int jjacobi_solve_rect(int dtype, void* G, const signed char* J, int m, int n, int ldg, double* lambda,
                       void* V, int ldv, double tol, int max_sweeps, const jj_opts* opts, jj_info* info);

/* Front end (Section 2.2, eq. 2.5): the factor G and signs J of a Hermitian
 * H = G J G^*, by the Bunch-Parlett factorization P H P^T = M D M^* with
 * complete pivoting (Bunch and Parlett 1971: 1x1 pivot on the largest diagonal
 * entry when it is at least alpha = (1 + sqrt 17)/8 times the largest entry of
 * the trailing matrix, otherwise a 2x2 pivot on the largest entry), then
 * D's 2x2 blocks diagonalised by one rotation each and M's columns scaled:
 * G = P^T M Q |Lambda|^{1/2}, J = sign(Lambda).  G is lower block triangular
 * up to the row permutation.
 *   H     device, n x n, leading dimension ldh; only the lower triangle is read
 *         (complex: the imaginary parts of the diagonal are ignored); not modified.
 *   G     device out, n x n, leading dimension ldg >= n: the first *rank
 *         columns receive G, the others are zeroed.
 *   J     host out, n signed chars: the first *rank are the signs, the rest 0.
 *   rank  host out: r.  The factorization stops when every entry of the
 *         trailing matrix is at most tol * max|h_ij| (tol <= 0: n * 2^-53); H
 *         then has rank r and G is n x r of full column rank.
 * Runs on opts->stream (nullable opts); returns after completion.  Returns 0,
 * JJ_NONFINITE (3) for a non-finite entry in the lower triangle, JJ_HIP_ERROR,
 * or -k for an invalid k-th argument. */
int jjacobi_factor(int dtype, const void* H, int n, int ldh, void* G, int ldg, signed char* J, int* rank,
                   double tol, const jj_opts* opts);

/* Eigenpairs of a Hermitian H given explicitly: jjacobi_factor (default rank
 * tolerance) followed by jjacobi_solve_rect on the n x r factor.  H (device,
 * n x n, ldh, lower triangle read) is destroyed: G is formed in its storage.
 * lambda (n doubles): the r nonzero eigenvalues descending, then n - r zeros;
 * V (n x n, ldv >= n): their unit eigenvectors, then an orthonormal basis of
 * the null space of a singular H (the last n - r columns of Q in the
 * Householder QR of the first r columns, Section 2.2).  info->rank receives
 * r.  tol and
 * max_sweeps as for the solve.  Status codes as jjacobi_solve_ex (argument k of
 * this signature for -k). */
int jjacobi_eigh(int dtype, void* H, int n, int ldh, double* lambda, void* V, int ldv, double tol,
                 int max_sweeps, const jj_opts* opts, jj_info* info);

/* Many independent problems in one call, each solved by the process of
 * jjacobi_solve_ex (the problems share launches; not a form the paper states)
 * (problem k uses dtype[k], G[k], J[k],
 * n[k], ldg[k], lambda[k], V[k], ldv[k]; all device pointers except J[k]).
 * info: array of count reports, or NULL.  Returns the largest status over the
 * problems (a negative value if an argument is invalid; then nothing runs). */
int jjacobi_solve_batched(int count, const int* dtype, void* const* G, const signed char* const* J,
                          const int* n, const int* ldg, double* const* lambda, void* const* V,
                          const int* ldv, double tol, int max_sweeps, const jj_opts* opts,
                          jj_info* info);

/* Kernel kinds reported by jjacobi_last_profile. */
#define JJ_K_GRAM 0   /* Gram block partials, eq. 3.6 */
#define JJ_K_PIVOT 1  /* pivot solve: Cholesky + inner J-Jacobi, eq. 3.8 and 3.12 */
#define JJ_K_UPDATE 2 /* block-column update, eq. 3.4 */
#define JJ_K_FINAL 3  /* column norms, ranking, eigenvectors, eq. 2.10 */
#define JJ_K_OTHER 4  /* input scan, counter resets */
#define JJ_NKINDS 5

/* Device time of the last solve on this thread that ran with opts.profile = 1. */
typedef struct jj_profile {
  double ms[8];           /* summed event-timed duration per kernel kind */
  long long launches[8];  /* launches per kind */
  long long units[8];     /* pivot problems handled per kind (UPDATE: pivots whose W_P
                             is not the identity; FINAL: columns) */
  long long rotations;    /* plane rotations applied inside pivot solves */
  long long inner_sweeps; /* inner sweeps run, summed over pivot solves */
  long long pivot_cols;   /* sum over solved pivots of their column count m */
  long long pivot_cols3;  /* sum over solved pivots of m^3 */
  int n, nblocks, block_width, sweeps, dtype, valid;
} jj_profile;

/* Copy the profile of the last profiled solve of this thread into *out (the
 * per-kernel time of the steps of Section 5.3).
 * Returns 0, or -1 if there is none (out untouched) or out is NULL. */
int jjacobi_last_profile(jj_profile* out);

/* Text for a status code (for 4: the last HIP error message of this thread). */
const char* jjacobi_status_string(int status);

/* Free the cached device workspace of every device. */
void jjacobi_release_workspace(void);

#ifdef __cplusplus
}
#endif

#endif /* JJACOBI_H */
