// Internal interface between the host orchestrator (jj_solver.hip) and the
// gfx950 kernels (jj_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jj {

// Largest pivot block (two block-columns of at most 32 columns each).
constexpr int kMaxPivot = 64;
// Largest block width.
constexpr int kMaxBlock = kMaxPivot / 2;
// Largest number of row chunks of one Gram block (partials summed by the pivot solver).
constexpr int kMaxChunks = 8;

// Device-side counters of one sweep.
struct SweepStats {
  unsigned long long max_off_bits;  // max scaled off-diagonal (bit pattern of a non-negative double)
  int pivots_rotated;               // pivots whose W_P is not the identity
  int breakdown;                    // Cholesky / hyperbolic-rotation failure seen
  int nonfinite;                    // non-finite value seen in G
  int zero_col;                     // final column norm zero
  int soft_fail;                    // pivot that could not be factored in a mixed-precision sweep
  unsigned long long rotations;     // plane rotations applied by pivot solves
  unsigned long long inner_sweeps;  // inner sweeps run by pivot solves
  unsigned long long pivot_cols;    // sum of m over pivots that ran the inner solve
  unsigned long long pivot_cols3;   // sum of m^3 over the same pivots
};

// A list of P pivot problems.  Pivot p has m[p] <= kMaxPivot columns; its
// local column c < m[p] is physical column cols[p*kMaxPivot + c] of G with sign
// sg[p*kMaxPivot + c]; entries c >= m[p] are -1 / 0.  nfirst[p] is the number
// of columns that come from the first block of the pair.
struct PivotList {
  const int* cols;
  const signed char* sg;
  const int* m;
  const int* nfirst;
  int count;
};

// ---- launchers (all asynchronous on `stream`) ----

// part[p][ch][r*64 + c] = sum over rows of chunk ch of conj(G[row, col(r)]) G[row, col(c)],
// for the upper 16x16 tiles (tile(r) <= tile(c)).  Real: FP64 MFMA.
void launch_gram_f64(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream);
void launch_gram_c128(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                      double* part, hipStream_t stream);

// Same partials formed on FP32 MFMA from FP64 data converted on load (mixed-
// precision pre-sweeps); the output is FP64 in the same layout.
void launch_gram_f32mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream);
void launch_gram_c64mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream);

// Per pivot: sum the Gram partials, test convergence, Cholesky, inner one-sided
// J-Jacobi on R accumulating W_P.  W[p] (kMaxPivot x kMaxPivot, column-major,
// complex interleaved for c128) and rotflag[p] are written.
// soft = 1 (mixed-precision sweeps): a pivot whose Gram block cannot be factored
// is left untouched and counted in soft_fail instead of raising breakdown.
void launch_pivot_f64(const double* part, int nch, const PivotList& pl, double tol, int inner_max,
                      int inner_mode, int soft, double* W, int* rotflag, SweepStats* st, hipStream_t stream);
void launch_pivot_c128(const double* part, int nch, const PivotList& pl, double tol, int inner_max,
                       int inner_mode, int soft, double* W, int* rotflag, SweepStats* st, hipStream_t stream);

// [G_i G_j] <- [G_i G_j] W_P in place for pivots with rotflag set.
void launch_update_f64(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                       int rows_per_chunk, hipStream_t stream);
void launch_update_c128(double* G, int ldg, int n, const PivotList& pl, const double* W,
                        const int* rotflag, int rows_per_chunk, hipStream_t stream);

void launch_reset_stats(SweepStats* st, hipStream_t stream);
void launch_check_finite(const double* G, int ldg, int n, int cplx, SweepStats* st, hipStream_t stream);

// Finalisation: d[q] = ||G[:, colmap[q]]||^2; lam = sg*d; rank by (lam desc, colmap asc);
// lambda[rank[q]] = lam[q], V[:, rank[q]] = G[:, colmap[q]] / sqrt(d[q]).
void launch_finalize(const double* G, int ldg, int n, int cplx, const int* colmap, const signed char* sgn,
                     double* d, int* rank, double* lambda, double* V, int ldv, SweepStats* st,
                     hipStream_t stream);

}  // namespace jj
