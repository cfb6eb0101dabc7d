/* CPU oracle for the one-sided hyperbolic (J-)Jacobi eigensolver.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The product library never links it and it
 * shares no code, header or table with the GPU path.
 *
 * Four instantiations of one plain algorithm (jj_oracle_body.inc):
 *   jjo_solve_d   real,    double working precision
 *   jjo_solve_ld  real,    long double (x87 80-bit) working precision
 *   jjo_solve_z   complex, double
 *   jjo_solve_lz  complex, long double
 * The long double forms adjudicate differences between two correct double
 * results (their difference is bounded by eps * kappa of the column-scaled G).
 * Each instantiation also holds the front end H -> G J G^* (jj_bp_body.inc,
 * jjo_bp_factor_*: Bunch-Parlett factorization and the diagonalisation of its
 * 2x2 blocks) and the rectangular solve (jjo_solve_rect_*).
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC (no FMA
 * contraction, no reassociation: every sum is evaluated in source order).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- real, double ---- */
#define RT double
#define ST double
#define IS_CPLX 0
#define FN(x) x##_d
#define R_SQRT sqrt
#define R_FABS fabs
#define R_HYPOT hypot
#include "jj_oracle_body.inc"
#include "jj_bp_body.inc"
#undef RT
#undef ST
#undef IS_CPLX
#undef FN
#undef R_SQRT
#undef R_FABS
#undef R_HYPOT

/* ---- real, long double ---- */
#define RT long double
#define ST long double
#define IS_CPLX 0
#define FN(x) x##_ld
#define R_SQRT sqrtl
#define R_FABS fabsl
#define R_HYPOT hypotl
#include "jj_oracle_body.inc"
#include "jj_bp_body.inc"
#undef RT
#undef ST
#undef IS_CPLX
#undef FN
#undef R_SQRT
#undef R_FABS
#undef R_HYPOT

/* ---- complex, double ---- */
#define RT double
#define ST double _Complex
#define IS_CPLX 1
#define FN(x) x##_z
#define R_SQRT sqrt
#define R_FABS fabs
#define R_HYPOT hypot
#define CONJ conj
#define CREAL creal
#define CIMAG cimag
#define IUNIT ((double _Complex)I)
#include "jj_oracle_body.inc"
#include "jj_bp_body.inc"
#undef RT
#undef ST
#undef IS_CPLX
#undef FN
#undef R_SQRT
#undef R_FABS
#undef R_HYPOT
#undef CONJ
#undef CREAL
#undef CIMAG
#undef IUNIT

/* ---- complex, long double ---- */
#define RT long double
#define ST long double _Complex
#define IS_CPLX 1
#define FN(x) x##_lz
#define R_SQRT sqrtl
#define R_FABS fabsl
#define R_HYPOT hypotl
#define CONJ conjl
#define CREAL creall
#define CIMAG cimagl
#define IUNIT ((long double _Complex)I)
#include "jj_oracle_body.inc"
#include "jj_bp_body.inc"
