// Internal interface between the host orchestrator (jj_solver.hip) and the
// gfx950 kernels (jj_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jj {

// Largest pivot block (two block-columns of at most 32 columns each).
constexpr int kMaxPivot = 64;
// Largest block width of a two-level pivot (a pair of blocks solved in LDS).
constexpr int kMaxBlock = kMaxPivot / 2;
// Largest three-level pivot (block width 64): its Cholesky factor R occupies a
// kMaxPivot3 x kMaxPivot3 slot of the R workspace.
constexpr int kMaxPivot3 = 2 * kMaxPivot;
// Largest number of row chunks of one Gram block (partials summed by the pivot solver).
constexpr int kMaxChunks = 8;

// Device-side counters of one sweep.
struct SweepStats {
  unsigned long long max_off_bits;  // max scaled off-diagonal (bit pattern of a non-negative double)
  int pivots_rotated;               // pivots whose W_P is not the identity
  int breakdown;                    // Cholesky / hyperbolic-rotation failure seen
  int nonfinite;                    // non-finite value seen in G
  int zero_col;                     // final column norm zero
  int soft_fail;                    // pivots that could not be factored in a mixed-precision sweep
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
  bool full = false;  // every pivot of the list has kMaxPivot columns (host-side knowledge)
};

// Optional batch descriptor.  A launch over S slots serves many independent
// problems at once: slot s belongs to problem slot_prob[s] and handles pair
// slot_k[s] of that problem's current step.  The problem's step, its active
// flag and its sweep counters live in device memory, so a sequence of steps can
// run (and be captured in a graph) without the host.  slot_prob == nullptr
// means a single-problem launch: slot s is pivot s of the tables, G / ldg / n
// come from the kernel arguments and the counters from `st`.
struct Batch {
  const int* slot_prob = nullptr;
  const int* slot_k = nullptr;
  const int* tab_base = nullptr;  // [problems] first pivot-table entry of step 0
  const int* npairs = nullptr;    // [problems] pairs per step
  const int* step = nullptr;      // [problems] current step
  const int* active = nullptr;    // [problems] 1 while being solved
  double* const* gptr = nullptr;  // [problems] G
  const int* ldg = nullptr;       // [problems]
  const int* nrow = nullptr;      // [problems] rows (= order)
  SweepStats* st = nullptr;       // [problems] counters of the current sweep
  const double* tol = nullptr;    // [problems] rotation threshold
  const int* prec = nullptr;      // [problems] 1 while the problem runs FP32-Gram (mixed) sweeps
  int prec_sel = -1;              // Gram launches: serve only problems whose prec equals this (-1: all)
};

// Resolve a launch slot: pivot-table index, matrix, rows and counters.
// Returns false for slots of problems that are not active.
__device__ __forceinline__ bool batch_resolve(const Batch& b, int slot, int& pidx, double*& G, int& ldg, int& n,
                                              SweepStats*& st) {
  if (b.slot_prob == nullptr) {
    pidx = slot;
    return true;
  }
  const int i = b.slot_prob[slot];
  if (!b.active[i]) return false;
  if (b.prec != nullptr && b.prec_sel >= 0 && b.prec[i] != b.prec_sel) return false;
  pidx = b.tab_base[i] + b.step[i] * b.npairs[i] + b.slot_k[slot];
  G = b.gptr[i];
  ldg = b.ldg[i];
  n = b.nrow[i];
  st = b.st + i;
  return true;
}

// Global-memory views of a pointer.  Matrices reached through the batch
// descriptor are pointers loaded from memory, so the compiler sees generic
// pointers and would emit FLAT accesses (whose completion counts against LDS
// traffic too); through these views it emits global loads and stores.
typedef double dv2 __attribute__((ext_vector_type(2)));  // (re, im) of one complex element
typedef __attribute__((address_space(1))) double gdbl;
typedef __attribute__((address_space(1))) dv2 gdbl2;
__device__ __forceinline__ gdbl* as_global(double* p) { return (gdbl*)p; }
__device__ __forceinline__ const gdbl* as_global(const double* p) { return (const gdbl*)p; }
__device__ __forceinline__ gdbl2* as_global2(double* p) { return (gdbl2*)p; }
__device__ __forceinline__ const gdbl2* as_global2(const double* p) { return (const gdbl2*)p; }

// Workgroups of a (chunks x slots) grid placed by XCD.  The dispatcher hands
// linear workgroup L to XCD L % 8; the pairs (slot, chunk), ordered by
// (slot % 8, slot / 8, chunk), are cut into consecutive runs, one per XCD, so
// that all chunks of slot s run on XCD s % 8 whenever the counts allow it (always
// when the number of slots is a multiple of 8), the same XCD as the pivot
// workgroup of slot s (a one-dimensional grid over slots).  The partials the
// pivot reads and the W_P the update reads then stay in that XCD's L2.
__device__ __forceinline__ void xcd_slot_chunk(int& slot, int& ch) {
  const int nch = gridDim.x, count = gridDim.y;
  const int T = nch * count;
  const int L = blockIdx.x + nch * blockIdx.y;
  const int x = L & 7;
  int pos = L >> 3;
  for (int y = 0; y < x; y++) pos += (T - y + 7) >> 3;  // workgroups on the XCDs before x
  for (int r = 0; r < 8; r++) {
    const int run = ((count - r + 7) >> 3) * nch;  // pairs whose slot is r mod 8
    if (pos < run) {
      slot = r + 8 * (pos / nch);
      ch = pos % nch;
      return;
    }
    pos -= run;
  }
  slot = 0;
  ch = 0;  // not reached: the runs cover all T pairs
}

// Events that the next kernel launch records at its own start and end
// (per-kernel profiling; the launch takes them and clears the slot).  Launches
// with no events armed are plain launches, which is what stream capture sees.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_next_launch;
template <typename F, typename... Args>
inline void launch(F kernel, const dim3& grid, const dim3& block, unsigned shm, hipStream_t stream, Args... args) {
  const LaunchEvents ev = g_next_launch;
  g_next_launch = LaunchEvents();
  if (ev.start != nullptr)
    hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, ev.start, ev.stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shm, stream, args...);
}

// ---- launchers (all asynchronous on `stream`) ----

// part[p][ch][r*64 + c] = sum over rows of chunk ch of conj(G[row, col(r)]) G[row, col(c)],
// for the upper 16x16 tiles (tile(r) <= tile(c)).  Real: FP64 MFMA.
// only (nullable): pivots with only[p] == 0 are skipped.
void launch_gram_f64(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream, const Batch& b = Batch(), const int* only = nullptr);
void launch_gram_c128(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                      double* part, hipStream_t stream, const Batch& b = Batch(), const int* only = nullptr);

// Same partials formed on FP32 MFMA (mixed-precision pre-sweeps): the same
// kernels with the operands rounded to FP32 as they leave LDS and FP32
// accumulation within a chunk; the output is FP64 in the same layout.
void launch_gram_f32mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b = Batch());
void launch_gram_c64mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b = Batch());
// Mixed-precision sweeps: one launch whose slots choose their precision, FP64
// for a single-solve slot with f64[slot] set or a batched slot whose problem
// has left its FP32 sweeps (b.prec[problem] == 0), FP32 MFMA otherwise.
void launch_gram_sel(bool cplx, const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream, const Batch& b, const int* f64);
// p[0..count) = v
void launch_fill_int(int* p, int count, int v, hipStream_t stream);

// Per pivot: sum the Gram partials, test convergence, Cholesky, inner one-sided
// J-Jacobi on R accumulating W_P.  W[p] (kMaxPivot x kMaxPivot, column-major,
// complex interleaved for c128) and rotflag[p] are written.
// soft = 1 (mixed-precision sweeps): a pivot whose Gram block cannot be factored
// is left untouched and counted in soft_fail instead of raising breakdown.
// mode: 0 full inner sweeps (inner_max), 1 off-diagonal pass only, 2 (batched
// block-oriented) full pass at step 0 of the problem's sweep, else off-diagonal,
// 3 direct: a single pivot holding every column of a G of n <= kMaxPivot rows is
// solved on G itself with up to inner_max inner sweeps (its Gram block and
// Cholesky factor only test full column rank: a failed factorisation is a
// breakdown), and the rotated columns are written back to G (G, ldg; rotflag 0,
// pivots_rotated counts the pivot if its last inner sweep rotated).
// Only the first ceil(n / rows_per_chunk) partials of a pivot are summed.
// refine (nullable, single problems in mixed sweeps): per-pair flags kept
// across sweeps; a pivot that fails softly sets its flag (and is left for this
// sweep), and a flagged pivot (its Gram block formed in FP64, see
// launch_gram_sel) is solved with tol64 and no soft failure.  only (nullable):
// pivots with only[p] == 0 return at once.
void launch_pivot_f64(const double* part, int nch, int n, int rows_per_chunk, const PivotList& pl, double tol,
                      double tol64, int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                      hipStream_t stream, const Batch& b, int* refine, const int* only, double* G, int ldg);
void launch_pivot_c128(const double* part, int nch, int n, int rows_per_chunk, const PivotList& pl, double tol,
                       double tol64, int inner_max, int inner_mode, int soft, double* W, int* rotflag, SweepStats* st,
                       hipStream_t stream, const Batch& b, int* refine, const int* only, double* G, int ldg);

// [G_i G_j] <- [G_i G_j] W_P in place for pivots with rotflag set.
// nch_u: number of row chunks in the grid (0: ceil(n / rows_per_chunk)).
void launch_update_f64(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                       int rows_per_chunk, hipStream_t stream, const Batch& b = Batch(), int nch_u = 0);
void launch_update_c128(double* G, int ldg, int n, const PivotList& pl, const double* W,
                        const int* rotflag, int rows_per_chunk, hipStream_t stream, const Batch& b = Batch(),
                        int nch_u = 0);

// Batched bookkeeping (one thread or one workgroup per problem).
// After a step: next step, or end of sweep with the per-problem convergence
// test; problems in mixed sweeps (prec[i] = 1, prec may be null) leave FP32 by
// the same rule as single solves and count their mixed sweeps.
void launch_batch_advance(int count, const int* nsteps, int* step, int* sweep, int* active, int* status,
                          SweepStats* st, double* final_off, int max_sweeps, int* active_count, int* prec,
                          int* mixed_sweeps, double mix_switch, hipStream_t stream);
void launch_batch_check_finite(int count, double* const* gptr, const int* ldg, const int* nrow, const int* width,
                               int* bad, hipStream_t stream);
void launch_batch_finalize(int count, double* const* gptr, const int* ldg, const int* nrow, const int* width,
                           const int* colmap, const int* cm_off, const signed char* sgn, double* const* lam_ptr,
                           double* const* v_ptr, const int* ldv, double* dwork, int* rkwork, int* zero_col,
                           hipStream_t stream);

void launch_reset_stats(SweepStats* st, hipStream_t stream);
// G has `rows` rows and `cols` columns (rows >= cols).
void launch_check_finite(const double* G, int ldg, int rows, int cols, int cplx, SweepStats* st, hipStream_t stream);

// Finalisation over the cols columns of G (rows rows each): d[q] = ||G[:, colmap[q]]||^2;
// lam = sg*d; rank by (lam desc, colmap asc); lambda[rank[q]] = lam[q],
// V[:, rank[q]] = G[:, colmap[q]] / sqrt(d[q]).
void launch_finalize(const double* G, int ldg, int rows, int cols, int cplx, const int* colmap,
                     const signed char* sgn, double* d, int* rank, double* lambda, double* V, int ldv,
                     SweepStats* st, hipStream_t stream);

// ---- three-level pivots (block width 64; jj_three.hip) ----
// Sum the partials of each pair's six 64-column sub-pivots (I, J, I1 J1, I1 J2,
// I2 J1, I2 J2) into A_P (order n1s[p] + n2s[p] <= 128), record the scaled
// off-diagonal of the part a step annihilates (all of A_P if first, else A_IJ),
// factor A_P = R^* R and write R to R + p * 128 * ldr (128 x 128, zero-padded).
void launch_chol128(bool cplx, const double* part, int nch, int nrows, int rows_per_chunk, const int* n1s,
                    const int* n2s, int count, double* R, int ldr, int first, SweepStats* st, hipStream_t stream);

// ---- front end H -> G J G^* (Bunch-Parlett; jj_frontend.hip) ----
constexpr int kBpThreads = 256;  // threads of every front-end workgroup (update tiles: 256 rows x 8 columns)
constexpr int kBpGroups = 1024;  // workgroups of one update launch (and partial maxima per step)

struct BPState {
  int k;          // next column to factor
  int done;       // 1 once the trailing matrix is negligible (or k = n, or non-finite input)
  int kcur, s;    // column and order (1, 2; 0: none) of the pivot the next update applies
  int rank;       // columns factored, set when done
  int nonfinite;  // a non-finite entry was met
  double hmax;    // max |h_ij| of the input
};
struct BPPartial {
  double mu0;      // largest |s_ij| of a workgroup's entries
  long long idx0;  // its column-major index j * n + i (smallest among equals)
  double mu1;      // largest |s_ii| of its diagonal entries
  long long idx1;  // its row index
};

void launch_bp_init(BPState* st, int* perm, int n, hipStream_t stream);
// Schur update of the pivot recorded in st (none at the start: a scan), fused
// with the per-workgroup maxima of the new trailing lower triangle.
void launch_bp_update(double* A, int n, int cplx, const double* pcol, BPState* st, BPPartial* part,
                      hipStream_t stream);
// Pivot choice, symmetric interchanges, column(s) of M; pcol receives the unscaled pivot columns.
void launch_bp_select(double* A, int n, int cplx, double tol, double* pcol, BPState* st, const BPPartial* part,
                      int* perm, int* piv, double* dblk, hipStream_t stream);
// Null space of a singular H: Householder QR of A (n x r, ld n; overwritten;
// reflectors to Vh, n x r, and beta, r), then E (n x (n - r), ld lde) = the
// last n - r columns of Q.  r >= 1, r < n.
void launch_nullspace(int cplx, double* A, int n, int r, double* Vh, double* beta, double* E, int lde,
                      hipStream_t stream);
// E (n x (n - r), ld lde) = rows r.. of the n x n identity (r = 0: E = I).
void launch_identity_tail(int cplx, double* E, int n, int lde, int r, hipStream_t stream);
// G = P^T M Q |Lambda|^{1/2} (first st->rank columns; the others zeroed) and J.
void launch_bp_build_g(const double* A, int n, int cplx, const BPState* st, const int* perm, const int* piv,
                       const double* dblk, double* G, int ldg, signed char* J, hipStream_t stream);

}  // namespace jj
