// gfx950 kernels of the blocked one-sided hyperbolic J-Jacobi sweep: the Gram
// and update kernels (real and complex; FP32 instances of the Gram kernels for
// the mixed-precision pre-sweeps) and the finalisation.
//
// One block step on a pair of block-columns (paper, Section 5.3, steps 1-4):
//   k_gram_real / k_gram_cplx      A_P = [G_i G_j]^* [G_i G_j]        (eq. 3.6)
//   k_pivot (jj_pivot.hip)         Cholesky A_P = R^* R (eq. 3.8), one-sided
//                                  J-Jacobi on the columns of R accumulating
//                                  W_P (eq. 3.12, Algorithms 3.1/3.2)
//   k_update_f64 / k_update_c128   [G_i G_j] <- [G_i G_j] W_P         (eq. 3.4)
// and the finalisation lambda_i = j_i ||g_i||^2, v_i = g_i/||g_i|| (eq. 2.10).
//
// MFMA: v_mfma_f64_16x16x4f64.  Lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and receives D[4v + l/16][l%16] in element v of its 4-double accumulator.
#include "jj_device.h"

#include <math.h>

#include <type_traits>

namespace jj {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Accumulators of the Gram kernels: FP64 MFMA, or FP32 MFMA for the mixed-
// precision pre-sweeps.  In the latter G stays FP64 in HBM and in LDS; the
// operands are rounded to FP32 as they leave LDS and the products accumulate
// on v_mfma_f32_16x16x4f32 (twice the FP64 matrix rate) over the chunk, the
// chunk partials being added in FP64.  Only the Gram block (eq. 3.6) is formed
// this way: the pivot solver computes every rotation and W_P in FP64 and the
// update stays FP64, so each applied transformation is J-unitary to FP64
// working precision (remark (a) of Section 2.3: inaccurate rotation
// parameters do not harm the one-sided process as long as the applied
// transformation is numerically J-unitary).  The two instructions place
// results differently: element v of lane (c16, g) is D[4v + g][c16] for FP64
// and D[4g + v][c16] for FP32 (measured on gfx950); the operand layouts agree.
typedef float f4 __attribute__((ext_vector_type(4)));
template <bool F32>
struct GAcc;
template <>
struct GAcc<false> {
  typedef d4 T;
  static __device__ __forceinline__ T zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ T mma(double a, double b, T c) { return mfma16(a, b, c); }
  static __device__ __forceinline__ d4 wide(T c) { return c; }
  static __device__ __forceinline__ int row(int v, int g) { return 4 * v + g; }
};
template <>
struct GAcc<true> {
  typedef f4 T;
  static __device__ __forceinline__ T zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ T mma(double a, double b, T c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ d4 wide(T c) { return d4{(double)c[0], (double)c[1], (double)c[2], (double)c[3]}; }
  static __device__ __forceinline__ int row(int v, int g) { return 4 * g + v; }
};

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* addr, double v) {
  atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Gram partials.  Grid (chunks, P), 256 threads.  Chunk ch covers rows
// [ch*rows_per_chunk, min(n, (ch+1)*rows_per_chunk)).  The chunk is staged
// through LDS in blocks of 32 rows by load-to-LDS instructions
// (global_load_lds_dwordx4: each lane fetches 16 bytes, one row pair of one
// column, and the instruction writes the 64 lanes' data to 1 KiB of LDS at
// base + 16 lane without passing through registers).  Three blocks rotate, two
// in flight while the third is multiplied.  In a block, column c occupies 32
// doubles and its row pair q sits in slot q ^ (c % 16): the lane that fills a
// slot fetches the row pair the slot holds, so each column is still read whole
// and contiguous, and an MFMA operand read (lane (c16, g) takes row r of column
// 16T + c16, word offset 4 ((r/2) ^ c16) + 2 (r%2) modulo the 64 banks) touches
// every bank exactly twice.  Padding columns and rows past the chunk read a
// zero pair; for an odd row count the chunk's last row, whose pair straddles
// the end, is written separately.  Wave w accumulates all 10 upper 16x16 tiles
// over rows 8w..8w+7 of every block; the four waves are reduced through LDS in
// a fixed order and the partial is written per chunk.  Measured at n = 4096
// (64 pairs of 64 columns, 8 chunks): 34.1 -> 28.9 us per launch against
// staging the blocks through registers.  Slower: three to seven blocks in
// flight, 512-thread workgroups, and each wave fetching only its own rows
// into an LDS region of its own (no barrier in the loop).
// ---------------------------------------------------------------------------
constexpr int kGramRows = 32;                        // rows per staged block
constexpr int kGramBufs = 3;                         // staged blocks
constexpr int kGramLpc = kGramRows / 2;              // lanes per column in one load instruction
constexpr int kGramCpi = 64 / kGramLpc;              // columns per load instruction
constexpr int kGramIpw = kMaxPivot / kGramCpi / 4;   // load instructions per wave per block
constexpr int kGramSmem = kGramBufs * kMaxPivot * kGramRows;
static_assert(kGramSmem >= 2 * 10 * 64 * 4, "the wave reduction reuses the staging blocks");
static_assert(kGramBufs == 3, "the loads waited for: one block issued later");

__device__ double gram_zero_pair[2];  // the source of padding: never written

typedef __attribute__((address_space(3))) void* lds_void;

// s_waitcnt with vmcnt = v (expcnt and lgkmcnt left alone): the field layout of
// gfx9 encodings, vmcnt bits 3:0 and 15:14
#define JJ_WAIT_VM(v) __builtin_amdgcn_s_waitcnt(((v) & 15) | (((v) >> 4) << 14) | 0xF70)

template <bool F32>
__device__ __forceinline__ void gram_real_body(const double* __restrict__ G0, int ldg0, int n0,
                                               const int* __restrict__ cols, const int* __restrict__ mlist,
                                               int rows_per_chunk, double* __restrict__ part, const Batch& bt,
                                               int slot, int ch, int nch, double* smem) {
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = const_cast<double*>(G0);
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (ch > 0 && ch * rows_per_chunk >= n) return;  // chunk beyond this problem's rows
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  if (m <= 0) return;  // empty pivot (a padding slot): no columns, no partial
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const int nblk = (r1 - r0 + kGramRows - 1) / kGramRows;

  // loader: instruction j of wave w fills columns kGramCpi (kGramIpw w + j) ..
  // + kGramCpi - 1; this lane, column col, fetches row pair q of each block
  const double* colp[kGramIpw];
  int qrow[kGramIpw];
#pragma unroll
  for (int j = 0; j < kGramIpw; j++) {
    const int col = kGramCpi * (kGramIpw * wave + j) + lane / kGramLpc;
    qrow[j] = 2 * ((lane % kGramLpc) ^ (col % kGramLpc));
    colp[j] = col < m ? Gm + (size_t)cols[p * kMaxPivot + col] * ldg : nullptr;
  }
  auto issue = [&](int b, int buf) {
    double* S = smem + buf * (kMaxPivot * kGramRows);
#pragma unroll
    for (int j = 0; j < kGramIpw; j++) {
      const int row = r0 + b * kGramRows + qrow[j];
      const double* src = (colp[j] != nullptr && row + 1 < r1) ? colp[j] + row : gram_zero_pair;
      __builtin_amdgcn_global_load_lds(src, (lds_void)(S + (kGramIpw * wave + j) * (kGramCpi * kGramRows)), 16, 0, 0);
    }
  };

  typename GAcc<F32>::T ac[10];
#pragma unroll
  for (int t = 0; t < 10; t++) ac[t] = GAcc<F32>::zero();
  for (int b = 0; b < kGramBufs - 1 && b < nblk; b++) issue(b, b);
  // full: all four column tiles in use, no branch around the MFMAs (a
  // conditional MFMA compiles to a block of its own with a wait for its operands)
  auto rows = [&](auto full) {
    int buf = 0;
    for (int b = 0; b < nblk; b++) {
      // this wave's loads of block b have landed once at most the later
      // blocks' (one here) are in flight; the barrier then covers every wave's.
      // A bare s_barrier: __syncthreads() is a release fence that would wait
      // for all loads in flight and undo the prefetch.
      if (b + 1 < nblk) JJ_WAIT_VM(kGramIpw);
      else JJ_WAIT_VM(0);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      const double* S = smem + buf * (kMaxPivot * kGramRows);
      if (b == nblk - 1 && ((r1 - r0) & 1)) {
        // odd row count: the last row's pair straddles the end and was loaded
        // as zeros; wave 0 writes the row itself (lane = column)
        if (wave == 0 && lane < m) {
          const int rr = r1 - 1 - (r0 + b * kGramRows);
          smem[buf * (kMaxPivot * kGramRows) + lane * kGramRows + 2 * ((rr >> 1) ^ (lane % kGramLpc)) + (rr & 1)] =
              as_global(Gm)[(size_t)cols[p * kMaxPivot + lane] * ldg + r1 - 1];
        }
        __syncthreads();
      }
      // the buffer of block b - 1, free since the barrier above
      if (b + kGramBufs - 1 < nblk) issue(b + kGramBufs - 1, buf == 0 ? kGramBufs - 1 : buf - 1);
#pragma unroll
      for (int kk = 0; kk < kGramRows / 16; kk++) {
        const int r = (kGramRows / 4) * wave + 4 * kk + g;
        double xt[4];
#pragma unroll
        for (int T = 0; T < 4; T++) xt[T] = S[(16 * T + c16) * kGramRows + 2 * ((r >> 1) ^ c16) + (r & 1)];
        int t = 0;
#pragma unroll
        for (int I = 0; I < 4; I++)
#pragma unroll
          for (int J = I; J < 4; J++) {
            if (decltype(full)::value || J < nt) ac[t] = GAcc<F32>::mma(xt[I], xt[J], ac[t]);
            t++;
          }
      }
      buf = buf == kGramBufs - 1 ? 0 : buf + 1;
    }
  };
  if (nt == 4)
    rows(std::true_type{});
  else
    rows(std::false_type{});
  __syncthreads();  // every wave is done with the blocks: the reduction reuses them
  // fixed-order reduction of the four waves: (w0 + w2) + (w1 + w3), through LDS
  d4 acc[10];
#pragma unroll
  for (int t = 0; t < 10; t++) acc[t] = GAcc<F32>::wide(ac[t]);
  d4* red = reinterpret_cast<d4*>(smem);  // [2][10][64]
  if (wave >= 2)
    for (int t = 0; t < 10; t++) red[((wave - 2) * 10 + t) * 64 + lane] = acc[t];
  __syncthreads();
  if (wave < 2)
    for (int t = 0; t < 10; t++) acc[t] += red[(wave * 10 + t) * 64 + lane];
  __syncthreads();
  if (wave == 1)
    for (int t = 0; t < 10; t++) red[t * 64 + lane] = acc[t];
  __syncthreads();
  if (wave == 0) {
    double* out = part + ((size_t)slot * nch + ch) * (kMaxPivot * kMaxPivot);
    int t = 0;
#pragma unroll
    for (int I = 0; I < 4; I++)
#pragma unroll
      for (int J = I; J < 4; J++) {
        const d4 sacc = acc[t] + red[t * 64 + lane];
        if (J < nt) {
#pragma unroll
          for (int v = 0; v < 4; v++) out[(16 * I + GAcc<F32>::row(v, g)) * kMaxPivot + 16 * J + c16] = sacc[v];
        }
        t++;
      }
  }
}

template <bool F32>
__global__ __launch_bounds__(256, 2) void k_gram_real(const double* __restrict__ G0, int ldg0, int n0,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     int rows_per_chunk, double* __restrict__ part, Batch bt,
                                                     const int* __restrict__ only) {
  __shared__ double smem[kGramSmem];  // the staged blocks; then the wave reduction
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  if (only != nullptr && !only[slot]) return;  // a re-solve launch: this pivot was solved
  gram_real_body<F32>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
}

// Mixed-precision sweeps: the precision of each slot's Gram block chosen in
// the kernel, FP64 for a single-solve slot whose flag f64[slot] is set (a pair
// whose FP32 block could not be factored earlier in the solve) and for a
// batched slot whose problem has left its FP32 sweeps, FP32 MFMA otherwise.
__device__ __forceinline__ bool gram_slot_f64(const Batch& bt, int slot, const int* f64) {
  if (bt.slot_prob != nullptr) return bt.prec == nullptr || !bt.prec[bt.slot_prob[slot]];
  return f64 != nullptr && f64[slot];
}

__global__ __launch_bounds__(256, 2) void k_gram_real_sel(const double* __restrict__ G0, int ldg0, int n0,
                                                         const int* __restrict__ cols, const int* __restrict__ mlist,
                                                         int rows_per_chunk, double* __restrict__ part, Batch bt,
                                                         const int* __restrict__ f64) {
  __shared__ double smem[kGramSmem];
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  if (gram_slot_f64(bt, slot, f64))
    gram_real_body<false>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
  else
    gram_real_body<true>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
}

// ---------------------------------------------------------------------------
// Update [G_i G_j] <- [G_i G_j] W_P in place.  Grid (nch, P), 256 threads.
// Computed transposed, D^T = W_P^T X^T, so that each lane's results are
// consecutive rows of one column (coalesced stores).  A wave loads its whole
// 16-row strip (all m columns) before writing any of it.
// ---------------------------------------------------------------------------
// W_P in LDS, column stride 68: an MFMA operand read has lanes (c16, g) at
// column 16I + c16, row 4kk + g, i.e. word offset 2 (68 c16 + g) = 8 c16 + 2g
// (mod 64 banks), so 8-byte reads spread evenly over the banks (16-byte
// complex reads too: 16 c16 + 4g).
constexpr int LDW = kMaxPivot + 4;

// FULL: every pivot of the launch has kMaxPivot columns, so the MFMA loop
// carries no branch (a conditional MFMA compiles to a block of its own with a
// wait for its LDS operand): 53.7 -> 51.8 us per launch at n = 4096, bitwise
// the same results.
template <bool FULL>
__global__ __launch_bounds__(256, 4) void k_update_f64(double* __restrict__ G0, int ldg0, int n0,
                                                    const int* __restrict__ cols, const int* __restrict__ mlist,
                                                    const double* __restrict__ Wg, const int* __restrict__ rotflag,
                                                    int rows_per_chunk, Batch bt) {
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = G0;
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (!rotflag[slot]) return;
  if (ch * rows_per_chunk >= n) return;
  gdbl* G = as_global(Gm);
  __shared__ double Ws[kMaxPivot * LDW];
  __shared__ int scol[kMaxPivot];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  if (m <= 0) return;             // empty pivot (a padding slot)
  const int nt = (m + 15) >> 4;   // output column tiles
  const int ks = (m + 3) >> 2;    // k-steps of 4 columns
  const double* Wp = Wg + (size_t)slot * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int c = e >> 6, r = e & 63;
    Ws[c * LDW + r] = (r < m && c < m) ? Wp[c * kMaxPivot + r] : 0.0;
  }
  if (tid < kMaxPivot) scol[tid] = (tid < m) ? cols[p * kMaxPivot + tid] : -1;
  __syncthreads();

  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  // Loads are unconditional, from clamped addresses (a padding column reads
  // the pivot's first column, a row past the chunk its last row), and padding
  // values are zeroed by a 0/1 factor (the matrix is finite: non-finite input
  // is rejected before the sweeps): no branch around a load, so outstanding
  // loads are counted instead of drained at every use.
  size_t coff[16];
  unsigned okbits = 0;
#pragma unroll
  for (int kk = 0; kk < 16; kk++) {
    const int pc = scol[4 * kk + g];
    const bool ok = kk < ks && pc >= 0;
    okbits |= ok ? (1u << kk) : 0u;
    coff[kk] = (size_t)(ok ? pc : scol[0]) * ldg;
  }
  // the next strip's loads are issued before the current strip's MFMAs (the
  // scheduling barrier keeps them there)
  double x[16], xn[16];
  int row0 = r0 + wave * 16;
  {
    const int row = row0 + c16;
    const unsigned ok = row < r1 ? okbits : 0u;
    const int rl = min(row, r1 - 1);
#pragma unroll
    for (int kk = 0; kk < 16; kk++) x[kk] = G[coff[kk] + rl] * ((ok >> kk) & 1u ? 1.0 : 0.0);
  }
  for (; row0 < r1; row0 += 64) {
    const int row = row0 + c16;
    const int nrow = row + 64;
    const unsigned nok = nrow < r1 ? okbits : 0u;
    const int nrl = min(nrow, r1 - 1);
#pragma unroll
    for (int kk = 0; kk < 16; kk++) xn[kk] = G[coff[kk] + nrl] * ((nok >> kk) & 1u ? 1.0 : 0.0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int I = 0; I < 4; I++) {
      if (FULL || I < nt) {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk++)
          if (FULL || kk < ks) acc = mfma16(Ws[(16 * I + c16) * LDW + 4 * kk + g], x[kk], acc);
#pragma unroll
        for (int v = 0; v < 4; v++) {
          int oc = 16 * I + 4 * v + g;
          int pc = scol[oc];
          if ((FULL || oc < m) && row < r1) G[(size_t)pc * ldg + row] = acc[v];
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < 16; kk++) x[kk] = xn[kk];
  }
}

// ---------------------------------------------------------------------------
// Complex Hermitian (complex128, interleaved).  A = X^H X is formed from real
// MFMA products: Re A = Xr^T Xr + Xi^T Xi, Im A = Xr^T Xi - Xi^T Xr.
// ---------------------------------------------------------------------------
// Complex Gram: the same load-to-LDS staging with 16-row blocks of (re, im)
// pairs (one 16-byte element per lane: 16 lanes per column, four columns per
// instruction) and row r of column c in slot r ^ (c % 16), so that a 16-byte
// operand read (word offset 4 (r ^ c16) modulo the 64 banks) touches every bank
// four times, the least for 64 such reads; no row pair straddles the end of
// the chunk.  Each upper 16x16 tile takes three real MFMA products
// (Gauss): P1 = Xr_I^T Xr_J, P2 = Xi_I^T Xi_J, P3 = (Xr_I - Xi_I)^T (Xr_J + Xi_J),
// Re A = P1 + P2, Im A = P3 - P1 + P2 (Im A = Xr^T Xi - Xi^T Xr).  The rounding
// error of every entry stays below a small multiple of eps ||x_i|| ||x_j||, the
// column-scaled bound the off-diagonal test and the rotations rely on.  Wave w
// takes row half w >> 1 of every block and tile set w & 1 (upper tiles 0-4 or
// 5-9 in row-major order); the two row halves are added in a fixed order.
constexpr int kGramRowsC = 16;                                // rows per staged block
constexpr int kGramBufsC = 3;                                 // staged blocks in rotation
constexpr int kGramIpwC = kMaxPivot * kGramRowsC / 64 / 4;    // load instructions per wave per block
static_assert(kGramBufsC >= 2 && kGramBufsC <= 4, "the loads waited for: at most two blocks issued later");
constexpr int kGramSmemC = kGramBufsC * kMaxPivot * kGramRowsC > 2 * 15 * 64 * 2
                               ? kGramBufsC * kMaxPivot * kGramRowsC
                               : 2 * 15 * 64 * 2;             // staged blocks, or the reduction (d4 = 2 dv2)

template <int TS, bool FULL, bool F32>
__device__ __forceinline__ void gram3m_tiles(const double (&xr)[4], const double (&xi)[4], int nt,
                                             typename GAcc<F32>::T (&q1)[5], typename GAcc<F32>::T (&q2)[5],
                                             typename GAcc<F32>::T (&q3)[5]) {
  constexpr int tI[2][5] = {{0, 0, 0, 0, 1}, {1, 1, 2, 2, 3}};
  constexpr int tJ[2][5] = {{0, 1, 2, 3, 1}, {2, 3, 2, 3, 3}};
#pragma unroll
  for (int u = 0; u < 5; u++) {
    const int I = tI[TS][u], J = tJ[TS][u];
    if (FULL || J < nt) {
      q1[u] = GAcc<F32>::mma(xr[I], xr[J], q1[u]);
      q2[u] = GAcc<F32>::mma(xi[I], xi[J], q2[u]);
      q3[u] = GAcc<F32>::mma(xr[I] - xi[I], xr[J] + xi[J], q3[u]);
    }
  }
}

template <int TS, bool F32>
__device__ __forceinline__ void gram3m_store(double* __restrict__ out, int nt, int c16, int g, const d4 (&q1)[5],
                                             const d4 (&q2)[5], const d4 (&q3)[5]) {
  constexpr int tI[2][5] = {{0, 0, 0, 0, 1}, {1, 1, 2, 2, 3}};
  constexpr int tJ[2][5] = {{0, 1, 2, 3, 1}, {2, 3, 2, 3, 3}};
#pragma unroll
  for (int u = 0; u < 5; u++) {
    const int I = tI[TS][u], J = tJ[TS][u];
    if (J < nt) {
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const size_t e = (size_t)(16 * I + GAcc<F32>::row(v, g)) * kMaxPivot + 16 * J + c16;
        out[2 * e] = q1[u][v] + q2[u][v];
        out[2 * e + 1] = (q3[u][v] - q1[u][v]) + q2[u][v];
      }
    }
  }
}

template <bool F32>
__device__ __forceinline__ void gram_cplx_body(const double* __restrict__ G0, int ldg0, int n0,
                                               const int* __restrict__ cols, const int* __restrict__ mlist,
                                               int rows_per_chunk, double* __restrict__ part, const Batch& bt,
                                               int slot, int ch, int nch, dv2* smem) {
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = const_cast<double*>(G0);
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (ch > 0 && ch * rows_per_chunk >= n) return;  // chunk beyond this problem's rows
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  if (m <= 0) return;  // empty pivot (a padding slot)
  const int nt = (m + 15) >> 4;
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const int nblk = (r1 - r0 + kGramRowsC - 1) / kGramRowsC;

  // loader: instruction j of wave w fills columns 4 (kGramIpwC w + j) .. + 3;
  // this lane, column col, fetches row (lane % 16) ^ (col % 16) of each block
  const dv2* colp[kGramIpwC];
  int lrow[kGramIpwC];
#pragma unroll
  for (int j = 0; j < kGramIpwC; j++) {
    const int col = 4 * (kGramIpwC * wave + j) + lane / 16;
    lrow[j] = (lane & 15) ^ (col & 15);
    colp[j] = col < m ? reinterpret_cast<const dv2*>(Gm) + (size_t)cols[p * kMaxPivot + col] * ldg : nullptr;
  }
  auto issue = [&](int b, int buf) {
    dv2* S = smem + buf * (kMaxPivot * kGramRowsC);
#pragma unroll
    for (int j = 0; j < kGramIpwC; j++) {
      const int row = r0 + b * kGramRowsC + lrow[j];
      const void* src = (colp[j] != nullptr && row < r1) ? (const void*)(colp[j] + row) : (const void*)gram_zero_pair;
      __builtin_amdgcn_global_load_lds(src, (lds_void)(S + (kGramIpwC * wave + j) * (4 * kGramRowsC)), 16, 0, 0);
    }
  };

  const int hh = wave >> 1, ts = wave & 1;
  typename GAcc<F32>::T a1[5], a2[5], a3[5];
#pragma unroll
  for (int u = 0; u < 5; u++) {
    a1[u] = GAcc<F32>::zero();
    a2[u] = GAcc<F32>::zero();
    a3[u] = GAcc<F32>::zero();
  }
  for (int b = 0; b < kGramBufsC - 1 && b < nblk; b++) issue(b, b);
  // full: all four column tiles in use, no branch around the MFMAs
  auto rows = [&](auto full) {
    int buf = 0;
    for (int b = 0; b < nblk; b++) {
      // this wave's loads of block b have landed once at most the later
      // blocks' are in flight; then a bare barrier (no release fence, which
      // would wait for every load in flight)
      const int later = min(kGramBufsC - 2, nblk - 1 - b);  // blocks issued after b
      if (later >= 2) JJ_WAIT_VM(2 * kGramIpwC);
      else if (later == 1) JJ_WAIT_VM(kGramIpwC);
      else JJ_WAIT_VM(0);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      // the buffer of block b - 1, free since the barrier above
      if (b + kGramBufsC - 1 < nblk) issue(b + kGramBufsC - 1, buf == 0 ? kGramBufsC - 1 : buf - 1);
      const dv2* S = smem + buf * (kMaxPivot * kGramRowsC);
#pragma unroll
      for (int kk = 0; kk < kGramRowsC / 8; kk++) {
        const int r = (kGramRowsC / 2) * hh + 4 * kk + g;
        double xr[4], xi[4];
#pragma unroll
        for (int T = 0; T < 4; T++) {
          const dv2 v = S[(16 * T + c16) * kGramRowsC + (r ^ c16)];
          xr[T] = v.x;
          xi[T] = v.y;
        }
        if (ts == 0)
          gram3m_tiles<0, decltype(full)::value, F32>(xr, xi, nt, a1, a2, a3);
        else
          gram3m_tiles<1, decltype(full)::value, F32>(xr, xi, nt, a1, a2, a3);
      }
      buf = buf == kGramBufsC - 1 ? 0 : buf + 1;
    }
  };
  if (nt == 4)
    rows(std::true_type{});
  else
    rows(std::false_type{});
  __syncthreads();  // every wave is done with the blocks: the reduction reuses them
  // fixed-order reduction of the two row halves through LDS, in FP64: half 0 + half 1
  d4 q1[5], q2[5], q3[5];
#pragma unroll
  for (int u = 0; u < 5; u++) {
    q1[u] = GAcc<F32>::wide(a1[u]);
    q2[u] = GAcc<F32>::wide(a2[u]);
    q3[u] = GAcc<F32>::wide(a3[u]);
  }
  d4* red = reinterpret_cast<d4*>(smem);  // [2][15][64]
  if (hh == 1)
#pragma unroll
    for (int u = 0; u < 5; u++) {
      red[(ts * 15 + u) * 64 + lane] = q1[u];
      red[(ts * 15 + 5 + u) * 64 + lane] = q2[u];
      red[(ts * 15 + 10 + u) * 64 + lane] = q3[u];
    }
  __syncthreads();
  if (hh == 0) {
#pragma unroll
    for (int u = 0; u < 5; u++) {
      q1[u] = q1[u] + red[(ts * 15 + u) * 64 + lane];
      q2[u] = q2[u] + red[(ts * 15 + 5 + u) * 64 + lane];
      q3[u] = q3[u] + red[(ts * 15 + 10 + u) * 64 + lane];
    }
    double* out = part + ((size_t)slot * nch + ch) * (2 * kMaxPivot * kMaxPivot);
    if (ts == 0)
      gram3m_store<0, F32>(out, nt, c16, g, q1, q2, q3);
    else
      gram3m_store<1, F32>(out, nt, c16, g, q1, q2, q3);
  }
}

template <bool F32>
__global__ __launch_bounds__(256, 2) void k_gram_cplx(const double* __restrict__ G0, int ldg0, int n0,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     int rows_per_chunk, double* __restrict__ part, Batch bt,
                                                     const int* __restrict__ only) {
  __shared__ dv2 smem[kGramSmemC];  // the staged blocks; then the wave reduction
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  if (only != nullptr && !only[slot]) return;  // a re-solve launch: this pivot was solved
  gram_cplx_body<F32>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
}

__global__ __launch_bounds__(256, 2) void k_gram_cplx_sel(const double* __restrict__ G0, int ldg0, int n0,
                                                         const int* __restrict__ cols, const int* __restrict__ mlist,
                                                         int rows_per_chunk, double* __restrict__ part, Batch bt,
                                                         const int* __restrict__ f64) {
  __shared__ dv2 smem[kGramSmemC];
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  if (gram_slot_f64(bt, slot, f64))
    gram_cplx_body<false>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
  else
    gram_cplx_body<true>(G0, ldg0, n0, cols, mlist, rows_per_chunk, part, bt, slot, ch, gridDim.x, smem);
}

// Update, complex: D^T = W^T X^T with Re = Wr^T Xr^T - Wi^T Xi^T and
// Im = Wi^T Xr^T + Wr^T Xi^T.
__global__ __launch_bounds__(256, 2) void k_update_c128(double* __restrict__ G0, int ldg0, int n0,
                                                     const int* __restrict__ cols, const int* __restrict__ mlist,
                                                     const double* __restrict__ Wg, const int* __restrict__ rotflag,
                                                     int rows_per_chunk, Batch bt) {
  int slot, ch;
  xcd_slot_chunk(slot, ch);
  int p = slot, ldg = ldg0, n = n0;
  double* Gm = G0;
  SweepStats* stp = nullptr;
  if (!batch_resolve(bt, slot, p, Gm, ldg, n, stp)) return;
  if (!rotflag[slot]) return;
  if (ch * rows_per_chunk >= n) return;
  __shared__ double2 Ws[kMaxPivot * LDW];
  __shared__ int scol[kMaxPivot];
  __shared__ size_t soff[kMaxPivot];  // clamped element offsets of the pivot's columns
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int c16 = lane & 15, g = lane >> 4;
  const int m = mlist[p];
  const int nt = (m + 15) >> 4;
  const int ks = (m + 3) >> 2;
  const double2* Wp = reinterpret_cast<const double2*>(Wg) + (size_t)slot * (kMaxPivot * kMaxPivot);
  for (int e = tid; e < kMaxPivot * kMaxPivot; e += 256) {
    int c = e >> 6, r = e & 63;
    Ws[c * LDW + r] = (r < m && c < m) ? Wp[c * kMaxPivot + r] : double2{0.0, 0.0};
  }
  if (tid < kMaxPivot) {
    const int pc = (tid < m) ? cols[p * kMaxPivot + tid] : -1;
    scol[tid] = pc;
    soff[tid] = (size_t)(pc >= 0 ? pc : cols[p * kMaxPivot]) * ldg;
  }
  __syncthreads();
  gdbl2* Gc = as_global2(Gm);
  const int r0 = ch * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  // unconditional loads from clamped addresses, padding zeroed by a 0/1
  // factor (finite matrix): outstanding loads are counted, not drained
  // (offsets read from LDS at each load: register budget)
  unsigned okbits = 0;
#pragma unroll
  for (int kk = 0; kk < 16; kk++) okbits |= (kk < ks && 4 * kk + g < m) ? (1u << kk) : 0u;
  // the next strip's loads are issued before the current strip's MFMAs
  dv2 x[16], xn[16];
  int row0 = r0 + wave * 16;
  {
    const int row = row0 + c16;
    const unsigned ok = row < r1 ? okbits : 0u;
    const int rl = min(row, r1 - 1);
#pragma unroll
    for (int kk = 0; kk < 16; kk++) x[kk] = Gc[soff[4 * kk + g] + rl] * ((ok >> kk) & 1u ? 1.0 : 0.0);
  }
  // full: a 64-column pivot, no branch around the MFMAs
  auto rows = [&](auto full) {
    for (; row0 < r1; row0 += 64) {
      const int row = row0 + c16;
      const int nrow = row + 64;
      const unsigned nok = nrow < r1 ? okbits : 0u;
      const int nrl = min(nrow, r1 - 1);
#pragma unroll
      for (int kk = 0; kk < 16; kk++) xn[kk] = Gc[soff[4 * kk + g] + nrl] * ((nok >> kk) & 1u ? 1.0 : 0.0);
      // three real products per complex one (Gauss): T1 = Xr Wr, T2 = Xi Wi,
      // T3 = (Xr + Xi)(Wr + Wi); Re = T1 - T2, Im = T3 - T1 - T2 (transposed here)
#pragma unroll
      for (int I = 0; I < 4; I++) {
        if (decltype(full)::value || I < nt) {
          d4 t1 = d4{0.0, 0.0, 0.0, 0.0}, t2 = d4{0.0, 0.0, 0.0, 0.0}, t3 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < 16; kk++)
            if (decltype(full)::value || kk < ks) {
              const double2 w = Ws[(16 * I + c16) * LDW + 4 * kk + g];
              t1 = mfma16(w.x, x[kk].x, t1);
              t2 = mfma16(w.y, x[kk].y, t2);
              t3 = mfma16(w.x + w.y, x[kk].x + x[kk].y, t3);
            }
#pragma unroll
          for (int v = 0; v < 4; v++) {
            int oc = 16 * I + 4 * v + g;
            int pc = scol[oc];
            if (oc < m && row < r1) Gc[(size_t)pc * ldg + row] = dv2{t1[v] - t2[v], (t3[v] - t1[v]) - t2[v]};
          }
        }
        __builtin_amdgcn_sched_barrier(0);  // one output tile at a time (register budget)
      }
#pragma unroll
      for (int kk = 0; kk < 16; kk++) x[kk] = xn[kk];
    }
  };
  if (m == kMaxPivot)
    rows(std::true_type{});
  else
    rows(std::false_type{});
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
    st->soft_fail = 0;
    st->rotations = 0ull;
    st->inner_sweeps = 0ull;
    st->pivot_cols = 0ull;
    st->pivot_cols3 = 0ull;
  }
}

__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ G, int ldg, int rows, int w,
                                                      SweepStats* st) {
  const int col = blockIdx.x;
  const double* c = G + (size_t)col * ldg * w;
  int bad = 0;
  for (int i = threadIdx.x; i < rows * w; i += 256) bad |= !isfinite(c[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->nonfinite, 1);
}

// d[q] = ||G[:, colmap[q]]||^2 ; one block per column, fixed-order tree reduction
__global__ __launch_bounds__(256) void k_colnorm(const double* __restrict__ G, int ldg, int rows, int w,
                                                 const int* __restrict__ colmap, double* __restrict__ d) {
  __shared__ double red[256];
  const int q = blockIdx.x, tid = threadIdx.x;
  const double* c = G + (size_t)colmap[q] * ldg * w;
  double s = 0.0;
  for (int i = tid; i < rows * w; i += 256) s += c[i] * c[i];
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
__global__ __launch_bounds__(256) void k_write_v(const double* __restrict__ G, int ldg, int rows, int w,
                                                 const int* __restrict__ colmap, const double* __restrict__ d,
                                                 const int* __restrict__ rank, double* __restrict__ V, int ldv) {
  const int q = blockIdx.x;
  const double* c = G + (size_t)colmap[q] * ldg * w;
  double* o = V + (size_t)rank[q] * ldv * w;
  const double dq = d[q];
  const double inv = dq > 0.0 ? 1.0 / sqrt(dq) : 0.0;
  for (int i = threadIdx.x; i < rows * w; i += 256) o[i] = c[i] * inv;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_gram_f64(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream, const Batch& b, const int* only) {
  launch(k_gram_real<false>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part, b, only);
}

void launch_gram_f32mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b) {
  launch(k_gram_real<true>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, rows_per_chunk,
         part, b, (const int*)nullptr);
}

void launch_update_f64(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                       int rows_per_chunk, hipStream_t stream, const Batch& b, int nch_u) {
  int nch = nch_u > 0 ? nch_u : (n + rows_per_chunk - 1) / rows_per_chunk;
  if (pl.full && b.slot_prob == nullptr)
    launch(k_update_f64<true>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, W, rotflag,
           rows_per_chunk, b);
  else
    launch(k_update_f64<false>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, W, rotflag,
           rows_per_chunk, b);
}

void launch_gram_c128(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                      double* part, hipStream_t stream, const Batch& b, const int* only) {
  launch(k_gram_cplx<false>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m,
                     rows_per_chunk, part, b, only);
}

void launch_gram_c64mix(const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                        double* part, hipStream_t stream, const Batch& b) {
  launch(k_gram_cplx<true>, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, rows_per_chunk,
         part, b, (const int*)nullptr);
}

void launch_gram_sel(bool cplx, const double* G, int ldg, int n, const PivotList& pl, int nch, int rows_per_chunk,
                     double* part, hipStream_t stream, const Batch& b, const int* f64) {
  if (cplx)
    launch(k_gram_cplx_sel, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, rows_per_chunk, part,
           b, f64);
  else
    launch(k_gram_real_sel, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, rows_per_chunk, part,
           b, f64);
}

__global__ void k_fill_int(int* p, int count, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

void launch_fill_int(int* p, int count, int v, hipStream_t stream) {
  if (count > 0) launch(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, stream, p, count, v);
}

void launch_update_c128(double* G, int ldg, int n, const PivotList& pl, const double* W, const int* rotflag,
                        int rows_per_chunk, hipStream_t stream, const Batch& b, int nch_u) {
  int nch = nch_u > 0 ? nch_u : (n + rows_per_chunk - 1) / rows_per_chunk;
  launch(k_update_c128, dim3(nch, pl.count), dim3(256), 0, stream, G, ldg, n, pl.cols, pl.m, W,
                     rotflag, rows_per_chunk, b);
}

void launch_reset_stats(SweepStats* st, hipStream_t stream) {
  launch(k_reset_stats, dim3(1), dim3(64), 0, stream, st);
}

void launch_check_finite(const double* G, int ldg, int rows, int cols, int cplx, SweepStats* st,
                         hipStream_t stream) {
  launch(k_check_finite, dim3(cols), dim3(256), 0, stream, G, ldg, rows, cplx ? 2 : 1, st);
}

void launch_finalize(const double* G, int ldg, int rows, int cols, int cplx, const int* colmap,
                     const signed char* sgn, double* d, int* rank, double* lambda, double* V, int ldv,
                     SweepStats* st, hipStream_t stream) {
  const int w = cplx ? 2 : 1;
  launch(k_colnorm, dim3(cols), dim3(256), 0, stream, G, ldg, rows, w, colmap, d);
  launch(k_rank, dim3((cols + 255) / 256), dim3(256), 0, stream, cols, d, sgn, colmap, rank, lambda, st);
  launch(k_write_v, dim3(cols), dim3(256), 0, stream, G, ldg, rows, w, colmap, d, rank, V, ldv);
}

}  // namespace jj
