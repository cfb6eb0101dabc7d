// Host orchestrator and C ABI of the blocked one-sided J-Jacobi eigensolver.
//
// Per solve (paper, Algorithm 5.2 and Section 5.3, on one GPU):
//   1. stable reordering of the columns so that J = diag(I_nu, -I_{n-nu})
//      (Section 2.3, last paragraph), uniform partition into an even number
//      of blocks (eq. 3.2-3.3), and the round-robin pair table (Section 4.2;
//      here the circle-method tournament with block 0 fixed, which visits
//      every pair of blocks exactly once in nblocks-1 steps of nblocks/2
//      disjoint pairs);
//   2. sweeps: for each step, Gram -> pivot solve -> update on all pairs of
//      the step at once (the pairs of one step are independent, Section 4);
//      convergence when a sweep's pivots all pass the scaled off-diagonal test
//      (Section 5.3, "no rotations" form);
//   3. finalisation lambda_i = j_i ||g_i||^2, v_i = g_i/||g_i|| (eq. 2.10).
// The columns are never moved: blocks are lists of physical column indices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "jjacobi.h"
#include "jj_device.h"

namespace jj {

thread_local LaunchEvents g_next_launch;

static thread_local std::string g_last_error;
static std::mutex g_mutex;

struct HipFail {
  hipError_t e;
};

static void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    throw HipFail{e};
  }
}

// One growing device allocation per device, carved into aligned sections.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
};
static Arena g_arena[64];

struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

static char* arena_get(size_t bytes) {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  Arena& a = g_arena[dev & 63];
  if (a.cap < bytes) {
    if (a.base) ck(hipFree(a.base), "hipFree");
    a.base = nullptr;
    a.cap = 0;
    size_t want = std::max(bytes, size_t(1) << 20);
    ck(hipMalloc((void**)&a.base, want), "hipMalloc workspace");
    a.cap = want;
  }
  return a.base;
}

// Fixed device scratch of jjacobi_solve_noalloc, for callers that cannot
// allocate device memory: one array per device in the library's code object,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device array: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is handed to kernels.
constexpr size_t kScratchBytes = JJ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
static void* g_scratch_dev[64];

static char* scratch_base() {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  void*& p = g_scratch_dev[dev & 63];
  if (p == nullptr) ck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  return (char*)p;
}

// A solve that needs more workspace than the fixed scratch holds.
struct ScratchTooSmall {
  size_t need;
};

// Optional per-launch timing with HIP events recorded on the solve stream.
struct Profiler {
  bool on = false;
  hipStream_t s = nullptr;
  size_t used = 0;
  struct Rec {
    int kind;
    size_t e0, e1;
  };

  std::vector<Rec> recs;
  jj_profile acc;
  static std::vector<hipEvent_t>& pool() {
    static std::vector<hipEvent_t> p;
    return p;
  }
  size_t mark() {
    if (!on) return 0;
    auto& P = pool();
    if (used == P.size()) {
      hipEvent_t e;
      ck(hipEventCreate(&e), "hipEventCreate");
      P.push_back(e);
    }
    ck(hipEventRecord(P[used], s), "hipEventRecord");
    return used++;
  }
  void done(int kind, size_t e0, long long units) {
    if (!on) return;
    size_t e1 = mark();
    recs.push_back(Rec{kind, e0, e1});
    acc.launches[kind]++;
    acc.units[kind] += units;
  }
  // A region of exactly one kernel: the launch itself records a pair of events
  // at its dispatch start and end, so no marker packets sit around it.
  size_t arm() {
    if (!on) return 0;
    auto& P = pool();
    while (P.size() < used + 2) {
      hipEvent_t e;
      ck(hipEventCreate(&e), "hipEventCreate");
      P.push_back(e);
    }
    g_next_launch = LaunchEvents{P[used], P[used + 1]};
    used += 2;
    return used - 2;
  }
  void done_kernel(int kind, size_t e0, long long units) {
    if (!on) return;
    recs.push_back(Rec{kind, e0, e0 + 1});
    acc.launches[kind]++;
    acc.units[kind] += units;
  }
  // call after the stream has been synchronised
  void flush() {
    if (!on) return;
    auto& P = pool();
    for (const Rec& r : recs) {
      float ms = 0.f;
      ck(hipEventElapsedTime(&ms, P[r.e0], P[r.e1]), "hipEventElapsedTime");
      acc.ms[r.kind] += ms;
    }
    recs.clear();
    used = 0;
  }
};

// Instantiated sweep graphs of one solve, by (precision, diagonal pass);
// destroyed with the solve.
struct SweepGraphs {
  hipGraphExec_t ex[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t& at(bool mix, bool diag) { return ex[mix ? 1 : 0][diag ? 1 : 0]; }
  ~SweepGraphs() {
    for (auto& r : ex)
      for (auto& e : r)
        if (e != nullptr) hipGraphExecDestroy(e);
  }
};
static thread_local jj_profile g_last_prof;
static thread_local bool g_have_prof = false;

// ---------------------------------------------------------------------------
// Host logic (exported with C linkage for the CPU tests as jjx_* helpers).
// ---------------------------------------------------------------------------

// Number of blocks: nbl = ceil(n / n_t) (eq. 3.2), at least 2, made even so
// that every block has a partner in each round-robin step.
int plan_nblocks(int n, int nt) {
  if (n < 2) return 1;
  int nbl = (n + nt - 1) / nt;
  if (nbl < 2) nbl = 2;
  if (nbl & 1) nbl++;
  if (nbl > n) nbl = n - (n & 1);
  return nbl;
}

// Uniform partition (eq. 3.3): the first n mod nbl blocks get floor(n/nbl)+1.
void plan_offsets(int n, int nbl, int* off) {
  int nmin = n / nbl, br = n % nbl;
  off[0] = 0;
  for (int l = 0; l < nbl; l++) off[l + 1] = off[l] + nmin + (l < br ? 1 : 0);
}

// Round-robin tournament: step t in [0, nbl-1), pair k in [0, nbl/2).
// Position 0 holds block 0; position i >= 1 holds block ((i - 1 + t) mod (nbl - 1)) + 1;
// pair k joins positions k and nbl-1-k.
void plan_round_robin(int nbl, int* pairs /* [(nbl-1)][nbl/2][2] */) {
  const int h = nbl / 2;
  for (int t = 0; t < nbl - 1; t++)
    for (int k = 0; k < h; k++) {
      int a = k == 0 ? 0 : ((k - 1 + t) % (nbl - 1)) + 1;
      int b = ((nbl - 1 - k - 1 + t) % (nbl - 1)) + 1;
      pairs[(t * h + k) * 2 + 0] = std::min(a, b);
      pairs[(t * h + k) * 2 + 1] = std::max(a, b);
    }
}

// Modulus pairing (Section 4.1): nbl steps per sweep; step t takes the
// anti-diagonal k = (nbl - 1 + t) mod nbl of the block matrix, i.e. the pairs
// {(i, j) : i + j = k mod nbl, i < j}, starting on the main anti-diagonal as
// the paper's layout does.  The diagonal blocks an anti-diagonal meets are
// left idle (option (b) of Section 4.1 rather than visiting them twice), so a
// step has nbl/2 or nbl/2 - 1 pairs and every pair occurs exactly once.
int plan_modulus(int nbl, int* pairs /* [nbl][nbl/2][2] */, int* counts /* [nbl] */) {
  const int h = nbl / 2;
  for (int t = 0; t < nbl; t++) {
    const int k = (nbl - 1 + t) % nbl;
    int c = 0;
    for (int i = 0; i < nbl; i++) {
      int j = ((k - i) % nbl + nbl) % nbl;
      if (i < j) {
        pairs[(t * h + c) * 2 + 0] = i;
        pairs[(t * h + c) * 2 + 1] = j;
        c++;
      }
    }
    counts[t] = c;
  }
  return nbl;
}

// Stable order with the +1 columns first (J = diag(I_nu, -I_{n-nu})).
void plan_sign_order(int n, const signed char* J, int* colmap) {
  int k = 0;
  for (int i = 0; i < n; i++)
    if (J[i] > 0) colmap[k++] = i;
  for (int i = 0; i < n; i++)
    if (J[i] < 0) colmap[k++] = i;
}

struct Plan {
  int n, nbl, nsteps, npairs_max;
  std::vector<int> off, colmap, cols, m, nfirst, count;
  std::vector<int> pblocks;  // [(step * npairs_max + pair) * 2 + {0, 1}]: the pair's two blocks
  std::vector<signed char> sgp, sgn;
};

static void build_pairs_tables(Plan& P, const std::vector<int>& pairs, int nsteps, const std::vector<int>& counts) {
  const int h = P.nbl / 2;
  P.nsteps = nsteps;
  P.npairs_max = h;
  int bmax = 0;
  for (int l = 0; l < P.nbl; l++) bmax = std::max(bmax, P.off[l + 1] - P.off[l]);
  if (2 * bmax > kMaxPivot) {
    // three-level pivots: only the pairs' blocks are tabulated here (the
    // sub-pivot tables are built by build_three_tables)
    P.count = counts;
    P.pblocks.assign((size_t)nsteps * h * 2, -1);
    for (int t = 0; t < nsteps; t++)
      for (int k = 0; k < counts[t]; k++) {
        P.pblocks[((size_t)t * h + k) * 2] = pairs[(t * h + k) * 2];
        P.pblocks[((size_t)t * h + k) * 2 + 1] = pairs[(t * h + k) * 2 + 1];
      }
    return;
  }
  P.cols.assign((size_t)nsteps * h * kMaxPivot, -1);
  P.sgp.assign((size_t)nsteps * h * kMaxPivot, 0);
  P.m.assign((size_t)nsteps * h, 0);
  P.nfirst.assign((size_t)nsteps * h, 0);
  P.count = counts;
  P.pblocks.assign((size_t)nsteps * h * 2, -1);
  for (int t = 0; t < nsteps; t++)
    for (int k = 0; k < counts[t]; k++) {
      int bi = pairs[(t * h + k) * 2], bj = pairs[(t * h + k) * 2 + 1];
      P.pblocks[((size_t)t * h + k) * 2] = bi;
      P.pblocks[((size_t)t * h + k) * 2 + 1] = bj;
      size_t base = ((size_t)t * h + k) * kMaxPivot;
      int c = 0;
      for (int q = P.off[bi]; q < P.off[bi + 1]; q++, c++) {
        P.cols[base + c] = P.colmap[q];
        P.sgp[base + c] = P.sgn[q];
      }
      P.nfirst[(size_t)t * h + k] = c;
      for (int q = P.off[bj]; q < P.off[bj + 1]; q++, c++) {
        P.cols[base + c] = P.colmap[q];
        P.sgp[base + c] = P.sgn[q];
      }
      P.m[(size_t)t * h + k] = c;
    }
}

static Plan make_plan(int n, const signed char* J, int nt, int strategy) {
  Plan P;
  P.n = n;
  P.nbl = plan_nblocks(n, nt);
  P.colmap.resize(n);
  plan_sign_order(n, J, P.colmap.data());
  P.sgn.resize(n);
  for (int q = 0; q < n; q++) P.sgn[q] = J[P.colmap[q]];
  P.off.resize(P.nbl + 1);
  plan_offsets(n, P.nbl, P.off.data());
  const int h = P.nbl / 2;
  if (P.nbl < 2) {
    P.nsteps = 0;
    P.npairs_max = 0;
    return P;
  }
  if (strategy == 1) {
    std::vector<int> pairs((size_t)P.nbl * h * 2), counts(P.nbl);
    plan_modulus(P.nbl, pairs.data(), counts.data());
    build_pairs_tables(P, pairs, P.nbl, counts);
  } else {
    std::vector<int> pairs((size_t)(P.nbl - 1) * h * 2), counts(P.nbl - 1, h);
    plan_round_robin(P.nbl, pairs.data());
    build_pairs_tables(P, pairs, P.nbl - 1, counts);
  }
  return P;
}

// Single-block pivots for the diagonal pre-processing pass (Algorithm 3.3):
// pivot l holds block l (nfirst = m, so block-oriented mode has no pairs).
static void build_diag_tables(const Plan& P, std::vector<int>& cols, std::vector<signed char>& sg,
                              std::vector<int>& m, std::vector<int>& nfirst) {
  cols.assign((size_t)P.nbl * kMaxPivot, -1);
  sg.assign((size_t)P.nbl * kMaxPivot, 0);
  m.assign(P.nbl, 0);
  nfirst.assign(P.nbl, 0);
  for (int l = 0; l < P.nbl; l++) {
    int c = 0;
    for (int q = P.off[l]; q < P.off[l + 1]; q++, c++) {
      cols[(size_t)l * kMaxPivot + c] = P.colmap[q];
      sg[(size_t)l * kMaxPivot + c] = P.sgn[q];
    }
    m[l] = c;
    nfirst[l] = c;
  }
}

// Tables of the three-level pivots (Section 5, Algorithm 5.1) for pairs of
// blocks I, J of up to 64 columns, halves I = I1 I2, J = J1 J2 (the first half
// takes the odd column):
//   six 64-column sub-pivots per pair whose Gram blocks cover A_P's upper
//   triangle: I, J, I1 J1, I1 J2, I2 J1, I2 J2 (physical columns of G);
//   inner pivots, two per pair in each of three inner steps: step 0 (the first
//   step of a sweep only) (I1 I2), (J1 J2), a full pass; step 1 (I1 J1),
//   (I2 J2) and step 2 (I1 J2), (I2 J1), passes over their off-diagonal blocks;
//   each with its columns in the pair's slot of the R workspace (pair k at
//   columns 128 k ...: I first, then J) and in G.
struct ThreeTables {
  std::vector<int> vcols, vm, n1, n2, icolR, icolG, im, inf;
  std::vector<signed char> isg;
};
static void build_three_tables(const Plan& P, ThreeTables& T) {
  const int h = std::max(P.npairs_max, 1);
  const size_t NP = (size_t)P.nsteps * h;
  T.vcols.assign(NP * 6 * kMaxPivot, -1);
  T.vm.assign(NP * 6, 0);
  T.n1.assign(NP, 0);
  T.n2.assign(NP, 0);
  T.icolR.assign(NP * 3 * 2 * kMaxPivot, -1);
  T.icolG.assign(NP * 3 * 2 * kMaxPivot, -1);
  T.isg.assign(NP * 3 * 2 * kMaxPivot, 0);
  T.im.assign(NP * 3 * 2, 0);
  T.inf.assign(NP * 3 * 2, 0);
  for (int t = 0; t < P.nsteps; t++)
    for (int k = 0; k < P.count[t]; k++) {
      const size_t pr = (size_t)t * h + k;
      const int bi = P.pblocks[pr * 2], bj = P.pblocks[pr * 2 + 1];
      const int nI = P.off[bi + 1] - P.off[bi], nJ = P.off[bj + 1] - P.off[bj];
      const int a1 = (nI + 1) / 2, b1 = (nJ + 1) / 2;
      T.n1[pr] = nI;
      T.n2[pr] = nJ;
      // local column l (0 .. nI + nJ - 1): physical column and sign
      auto phys = [&](int l) { return P.colmap[l < nI ? P.off[bi] + l : P.off[bj] + l - nI]; };
      auto sign = [&](int l) { return P.sgn[l < nI ? P.off[bi] + l : P.off[bj] + l - nI]; };
      // local ranges [lo, hi) of I1, I2, J1, J2
      const int rg[4][2] = {{0, a1}, {a1, nI}, {nI, nI + b1}, {nI + b1, nI + nJ}};
      auto fill = [&](int* cols, int* mm, int* nf, signed char* sg, int colbase, bool phys_cols, int x, int y) {
        int c = 0;
        for (int l = rg[x][0]; l < rg[x][1]; l++, c++) {
          cols[c] = phys_cols ? phys(l) : colbase + l;
          if (sg) sg[c] = sign(l);
        }
        if (nf) *nf = c;
        for (int l = rg[y][0]; l < rg[y][1]; l++, c++) {
          cols[c] = phys_cols ? phys(l) : colbase + l;
          if (sg) sg[c] = sign(l);
        }
        *mm = c;
      };
      const int sub[6][2] = {{0, 1}, {2, 3}, {0, 2}, {0, 3}, {1, 2}, {1, 3}};
      for (int v = 0; v < 6; v++)
        fill(&T.vcols[(pr * 6 + v) * kMaxPivot], &T.vm[pr * 6 + v], nullptr, nullptr, 0, true, sub[v][0],
             sub[v][1]);
      const int inner[3][2][2] = {{{0, 1}, {2, 3}}, {{0, 2}, {1, 3}}, {{0, 3}, {1, 2}}};
      for (int s = 0; s < 3; s++)
        for (int q = 0; q < 2; q++) {
          const size_t e = (((size_t)t * 3 + s) * h + k) * 2 + q;
          fill(&T.icolR[e * kMaxPivot], &T.im[e], &T.inf[e], &T.isg[e * kMaxPivot], k * 2 * kMaxPivot, false,
               inner[s][q][0], inner[s][q][1]);
          int mm = 0;
          fill(&T.icolG[e * kMaxPivot], &mm, nullptr, nullptr, 0, true, inner[s][q][0], inner[s][q][1]);
        }
    }
}

// The library's own non-blocking stream on the current device: solves run on
// it (a HIP graph cannot be captured on the legacy default stream), ordered
// after the caller's stream on entry; on scope exit the caller's stream is
// ordered after everything the solve enqueued.
static hipStream_t lib_stream() {
  static hipStream_t s[64] = {};
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  if (!s[dev & 63]) ck(hipStreamCreateWithFlags(&s[dev & 63], hipStreamNonBlocking), "hipStreamCreate");
  return s[dev & 63];
}

constexpr int kMaxStepGroups = 8;

struct StreamJoin {
  hipStream_t caller, lib;
  hipEvent_t ev = nullptr;
  StreamJoin(hipStream_t c, hipStream_t l) : caller(c), lib(l) {
    if (caller == lib) return;
    ck(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
    ck(hipEventRecord(ev, caller), "event");
    ck(hipStreamWaitEvent(lib, ev, 0), "wait event");
  }
  ~StreamJoin() {
    if (ev == nullptr) return;
    (void)hipEventRecord(ev, lib);
    (void)hipStreamWaitEvent(caller, ev, 0);
    (void)hipEventDestroy(ev);
  }
};

// Block width chosen per (dtype, size bucket) by timing two sweeps of each
// candidate on the first problem of that bucket (see tune_block_width).
// value: block width * 2 + inner mode (0 block-oriented, 1 full diagonalisation)
static std::map<std::pair<int, int>, int> g_tuned_bw;
static int size_bucket(int n) {
  int b = 0;
  while ((64 << b) < n && b < 12) b++;
  return b;  // 0: n <= 64, 1: <= 128, 2: <= 256, ...
}
static int tune_block_width(int dtype, void* G, const signed char* J, int n, int ldg, hipStream_t stream,
                            bool wide, bool modes);
// wide: 64 (three-level pivots) is a candidate too (single solves; the batched
// form takes at most 32); modes: the full-diagonalisation variant too (single
// solves that leave the inner mode to the library).  Cached per (dtype, wide,
// modes, size bucket).  Returns block width * 2 + inner mode.
static int tuned_block_width(int dtype, void* G, const signed char* J, int n, int ldg, hipStream_t stream,
                             bool wide = false, bool modes = false) {
  modes = modes && n <= 1024;  // the candidate set is what keys the cache
  const auto key = std::make_pair(dtype + (wide ? 2 : 0) + (modes ? 4 : 0), size_bucket(n));
  auto it = g_tuned_bw.find(key);
  if (it == g_tuned_bw.end() && !wide) {
    // a choice among more candidates that did not pick width 64 is the choice
    // among these
    auto w = g_tuned_bw.find(std::make_pair(dtype + 2 + (modes ? 4 : 0), size_bucket(n)));
    if (w != g_tuned_bw.end() && (w->second >> 1) != 64) it = g_tuned_bw.emplace(key, w->second).first;
  }
  if (it == g_tuned_bw.end())
    it = g_tuned_bw.emplace(key, tune_block_width(dtype, G, J, n, ldg, stream, wide, modes)).first;
  return it->second;
}

// noalloc: the workspace is the fixed device scratch, the work runs eagerly on
// the caller's stream (no library stream, events, graphs or block-width tuning:
// each of those allocates), and a solve whose workspace exceeds the scratch
// throws ScratchTooSmall before any device work.
// m_rows: rows of G (0: square, m = n); a rectangular G (m > n, full column
// rank) is the factor of a singular H of rank n (Section 2.2).
static int solve_one(int dtype, void* Gv, const signed char* J, int n, int ldg, double* lambda, void* Vv,
                     int ldv, double tol, int max_sweeps, const jj_opts& o, jj_info* info, bool graphs_ok = true,
                     bool noalloc = false, int m_rows = 0) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = m_rows > 0 ? m_rows : n;
  const int cplx = dtype == JJ_C128;
  double* G = (double*)Gv;
  double* V = (double*)Vv;
  if (noalloc) graphs_ok = false;
  hipStream_t stream = noalloc ? (hipStream_t)o.stream : lib_stream();
  StreamJoin join(noalloc ? stream : (hipStream_t)o.stream, stream);
  // block width: the caller's, else tuned for large problems (first use of a
  // size bucket), else 32
  // (widths above 32 make three-level pivots: plain FP64, block-oriented, no
  // diagonal pass, one step at a time; other option sets take 32).  The inner
  // mode: the caller's, or (inner_mode < 0) tuned with the width where the
  // width is tuned, else block-oriented.
  int imode = o.inner_mode;
  const bool three_ok = o.precision == 0 && o.diag_pass == 0 && imode <= 0 && o.step_groups <= 1;
  int nt = o.block_width > 0 ? std::min(o.block_width, three_ok ? 2 * kMaxBlock : kMaxBlock) : 32;
  if (o.block_width <= 0 && graphs_ok && m == n && n >= 1024) {
    const int tv = tuned_block_width(dtype, Gv, J, n, ldg, stream, three_ok, imode < 0);
    nt = tv >> 1;
    if (imode < 0) imode = tv & 1;
  }
  if (imode < 0) imode = 0;
  const int inner_max = o.inner_max_sweeps > 0 ? o.inner_max_sweeps : 12;
  if (tol <= 0.0) tol = (double)m * std::ldexp(1.0, -53);
  if (max_sweeps <= 0) max_sweeps = 100;

  Plan P = make_plan(n, J, nt, o.strategy);
  const int h = std::max(P.npairs_max, 1);
  int bmax = 0;
  for (int l = 0; l < P.nbl; l++) bmax = std::max(bmax, P.off[l + 1] - P.off[l]);
  const bool three = P.nsteps > 0 && 2 * bmax > kMaxPivot;
  ThreeTables T3;
  int nch3 = 1, rows_g3 = 64, rows_u3 = 64;
  if (three) {
    build_three_tables(P, T3);
    // the six sub-pivot Gram blocks of a step: about 1024 workgroups
    nch3 = std::max(1, std::min(std::min((1024 + 6 * h - 1) / (6 * h), (m + 63) / 64), kMaxChunks));
    rows_g3 = ((m + nch3 - 1) / nch3 + 63) / 64 * 64;
    nch3 = (m + rows_g3 - 1) / rows_g3;
    rows_u3 = ((long long)2 * h * ((m + 255) / 256) < 512) ? 64 : 256;
  }
  const size_t NP3 = three ? (size_t)P.nsteps * h : 0;
  // chunking of the row dimension for the Gram and update kernels
  int nch = std::max(1, std::min(std::min((1024 + h - 1) / h, (m + 63) / 64), kMaxChunks));
  int rows_g = ((m + nch - 1) / nch + 63) / 64 * 64;
  nch = (m + rows_g - 1) / rows_g;
  int rows_u = 256;
  if ((long long)h * ((m + 255) / 256) < 512) rows_u = 64;

  std::vector<int> dcols, dm, dnf;
  std::vector<signed char> dsg;
  build_diag_tables(P, dcols, dsg, dm, dnf);
  // pivot slots: the pairs of a step, or every block for the diagonal pass
  const int nb_piv = o.diag_pass != 0 ? std::max(h, P.nbl) : h;

  // workspace layout
  const size_t tab = (size_t)std::max(P.nsteps, 1) * h * kMaxPivot;
  size_t need = 0;
  {
    Carver c{nullptr};
    c.take<int>(tab);
    c.take<signed char>(tab);
    c.take<int>((size_t)std::max(P.nsteps, 1) * h);
    c.take<int>((size_t)std::max(P.nsteps, 1) * h);
    c.take<int>((size_t)P.nbl * kMaxPivot);
    c.take<signed char>((size_t)P.nbl * kMaxPivot);
    c.take<int>(P.nbl);
    c.take<int>(P.nbl);
    c.take<int>(n);
    c.take<signed char>(n);
    c.take<double>((size_t)nb_piv * nch * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
    c.take<double>((size_t)nb_piv * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
    c.take<int>(nb_piv);
    c.take<int>((size_t)std::max(P.nsteps, 1) * h + P.nbl);
    c.take<SweepStats>(1);
    c.take<double>(n);
    c.take<int>(n);
    if (three) {
      c.take<int>(NP3 * 6 * kMaxPivot);
      c.take<int>(NP3 * 6);
      c.take<int>(NP3);
      c.take<int>(NP3);
      c.take<int>(NP3 * 6 * kMaxPivot);
      c.take<int>(NP3 * 6 * kMaxPivot);
      c.take<signed char>(NP3 * 6 * kMaxPivot);
      c.take<int>(NP3 * 6);
      c.take<int>(NP3 * 6);
      c.take<double>((size_t)6 * h * nch3 * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
      c.take<double>((size_t)h * kMaxPivot3 * kMaxPivot3 * (cplx ? 2 : 1));
      c.take<double>((size_t)2 * h * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
      c.take<double>((size_t)2 * h * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
      c.take<int>((size_t)2 * h);
    }
    need = c.off + 256;
  }
  if (noalloc && need > kScratchBytes) throw ScratchTooSmall{need};
  Carver c{noalloc ? scratch_base() : arena_get(need)};
  int* d_cols = c.take<int>(tab);
  signed char* d_sg = c.take<signed char>(tab);
  int* d_m = c.take<int>((size_t)std::max(P.nsteps, 1) * h);
  int* d_nf = c.take<int>((size_t)std::max(P.nsteps, 1) * h);
  int* d_dcols = c.take<int>((size_t)P.nbl * kMaxPivot);
  signed char* d_dsg = c.take<signed char>((size_t)P.nbl * kMaxPivot);
  int* d_dm = c.take<int>(P.nbl);
  int* d_dnf = c.take<int>(P.nbl);
  int* d_colmap = c.take<int>(n);
  signed char* d_sgn = c.take<signed char>(n);
  double* d_part = c.take<double>((size_t)nb_piv * nch * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
  double* d_W = c.take<double>((size_t)nb_piv * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
  int* d_rot = c.take<int>(nb_piv);
  // mixed sweeps: per (step, pair), then per diagonal block, 1 once the pair's
  // FP32 Gram block could not be factored (its Gram block is FP64 from then on)
  int* d_promote = c.take<int>((size_t)std::max(P.nsteps, 1) * h + P.nbl);
  int* d_promote_diag = d_promote + (size_t)std::max(P.nsteps, 1) * h;
  SweepStats* d_st = c.take<SweepStats>(1);
  double* d_d = c.take<double>(n);
  int* d_rank = c.take<int>(n);
  // three-level pivots: sub-pivot and inner tables, Gram partials, R slots
  int *d_vcols = nullptr, *d_vm = nullptr, *d_n1 = nullptr, *d_n2 = nullptr, *d_icolR = nullptr,
      *d_icolG = nullptr, *d_im = nullptr, *d_inf = nullptr, *d_irot = nullptr;
  signed char* d_isg = nullptr;
  double *d_vpart = nullptr, *d_RW = nullptr, *d_ipart = nullptr, *d_iW = nullptr;
  if (three) {
    d_vcols = c.take<int>(NP3 * 6 * kMaxPivot);
    d_vm = c.take<int>(NP3 * 6);
    d_n1 = c.take<int>(NP3);
    d_n2 = c.take<int>(NP3);
    d_icolR = c.take<int>(NP3 * 6 * kMaxPivot);
    d_icolG = c.take<int>(NP3 * 6 * kMaxPivot);
    d_isg = c.take<signed char>(NP3 * 6 * kMaxPivot);
    d_im = c.take<int>(NP3 * 6);
    d_inf = c.take<int>(NP3 * 6);
    d_vpart = c.take<double>((size_t)6 * h * nch3 * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
    d_RW = c.take<double>((size_t)h * kMaxPivot3 * kMaxPivot3 * (cplx ? 2 : 1));
    d_ipart = c.take<double>((size_t)2 * h * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
    d_iW = c.take<double>((size_t)2 * h * kMaxPivot * kMaxPivot * (cplx ? 2 : 1));
    d_irot = c.take<int>((size_t)2 * h);
    auto up = [&](void* dst, const void* src, size_t bytes) {
      ck(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream), "H2D");
    };
    up(d_vcols, T3.vcols.data(), T3.vcols.size() * sizeof(int));
    up(d_vm, T3.vm.data(), T3.vm.size() * sizeof(int));
    up(d_n1, T3.n1.data(), T3.n1.size() * sizeof(int));
    up(d_n2, T3.n2.data(), T3.n2.size() * sizeof(int));
    up(d_icolR, T3.icolR.data(), T3.icolR.size() * sizeof(int));
    up(d_icolG, T3.icolG.data(), T3.icolG.size() * sizeof(int));
    up(d_isg, T3.isg.data(), T3.isg.size());
    up(d_im, T3.im.data(), T3.im.size() * sizeof(int));
    up(d_inf, T3.inf.data(), T3.inf.size() * sizeof(int));
  }

  // The plan's tables lie back to back in the workspace (pair tables, diagonal-
  // pass tables, column map and signs): they go up in one copy from a host
  // image of that span (the alignment gaps and tables not used are zero).  The
  // image outlives the copy: it is freed when the solve returns, after the
  // stream has been synchronised.
  std::vector<char> img;
  {
    char* lo = reinterpret_cast<char*>(d_cols);
    const size_t span = static_cast<size_t>(reinterpret_cast<char*>(d_sgn + n) - lo);
    img.assign(span, 0);
    auto put = [&](const void* dst, const void* src, size_t bytes) {
      if (bytes) std::memcpy(img.data() + (reinterpret_cast<const char*>(dst) - lo), src, bytes);
    };
    if (P.nsteps > 0 && !three) {
      put(d_cols, P.cols.data(), P.cols.size() * sizeof(int));
      put(d_sg, P.sgp.data(), P.sgp.size());
      put(d_m, P.m.data(), P.m.size() * sizeof(int));
      put(d_nf, P.nfirst.data(), P.nfirst.size() * sizeof(int));
    }
    put(d_dcols, dcols.data(), dcols.size() * sizeof(int));
    put(d_dsg, dsg.data(), dsg.size());
    put(d_dm, dm.data(), dm.size() * sizeof(int));
    put(d_dnf, dnf.data(), dnf.size() * sizeof(int));
    put(d_colmap, P.colmap.data(), n * sizeof(int));
    put(d_sgn, P.sgn.data(), n);
    ck(hipMemcpyAsync(lo, img.data(), span, hipMemcpyHostToDevice, stream), "H2D");
  }

  Profiler prof;
  prof.on = o.profile != 0 && !noalloc;
  prof.s = stream;
  std::memset(&prof.acc, 0, sizeof(prof.acc));

  SweepStats hst;
  size_t e0 = prof.mark();
  launch_reset_stats(d_st, stream);
  launch_check_finite(G, ldg, m, n, cplx, d_st, stream);
  launch_fill_int(d_promote, (int)((size_t)std::max(P.nsteps, 1) * h + P.nbl), 0, stream);
  prof.done(JJ_K_OTHER, e0, 0);
  ck(hipGetLastError(), "launch");
  ck(hipMemcpyAsync(&hst, d_st, sizeof(hst), hipMemcpyDeviceToHost, stream), "D2H");
  ck(hipStreamSynchronize(stream), "sync");
  prof.flush();
  if (hst.nonfinite) {
    if (info) {
      info->status = JJ_NONFINITE;
      info->sweeps = 0;
    }
    return JJ_NONFINITE;
  }

  auto gram64 = cplx ? launch_gram_c128 : launch_gram_f64;
  auto pivot = cplx ? launch_pivot_c128 : launch_pivot_f64;
  auto update = cplx ? launch_update_c128 : launch_update_f64;

  // Mixed precision: sweeps run with the FP32-MFMA Gram until a sweep's largest
  // scaled off-diagonal falls below mixed_switch; those sweeps use a rotation
  // threshold above FP32 rounding noise and never declare convergence.
  bool mixed = o.precision == 1;
  const double mix_switch = o.mixed_switch > 0.0 ? o.mixed_switch : 0.1;
  const double tol_mix = std::max(tol, std::ldexp(1.0, -20));
  int mixed_sweeps = 0, mixed_resolved = 0;
  int status = JJ_NOT_CONVERGED, sweep = 0;
  long long piv_rot = 0;
  double last_off = 0.0;
  bool breakdown = false;
  if (P.nbl < 2) status = JJ_OK;
  // One sweep: stats reset, the optional diagonal pass, then every step of the
  // pairing (Gram partials, pivot solves, update).  Profiled solves launch it
  // eagerly with per-kernel events; otherwise each variant (precision, diagonal
  // pass) is captured once per solve as a HIP graph and replayed per sweep.
  // Gram block and pivot solve of the pairs in pl.  In a mixed sweep the Gram
  // block is formed on FP32 MFMA, except for the pairs flagged in promote
  // (their FP32 block could not be factored in an earlier sweep: its scaled
  // condition is beyond FP32, e.g. nearly parallel columns), which are formed
  // and solved in FP64; a pivot whose FP32 block cannot be factored is left
  // for this sweep and flagged.
  auto gram_pivot = [&](bool use_mix, const PivotList& pl, double* part, double* W, int* rot, int* promote,
                        int mode, int imax, const std::function<void()>& after_first = nullptr) {
    size_t k0 = prof.arm();
    if (use_mix)
      launch_gram_sel(cplx != 0, G, ldg, m, pl, nch, rows_g, part, stream, Batch(), promote);
    else
      gram64(G, ldg, m, pl, nch, rows_g, part, stream, Batch(), nullptr);
    prof.done_kernel(JJ_K_GRAM, k0, pl.count);
    if (after_first) after_first();
    k0 = prof.arm();
    pivot(part, nch, m, rows_g, pl, use_mix ? tol_mix : tol, tol, imax, mode, use_mix, W, rot, d_st, stream, Batch(),
          use_mix ? promote : nullptr, nullptr, G, ldg);
    prof.done_kernel(JJ_K_PIVOT, k0, pl.count);
  };
  // steps whose pivots all have kMaxPivot columns: their update launches the
  // instance without per-column bounds
  std::vector<char> full_step(P.nsteps, 0);
  if (!P.m.empty())
    for (int t = 0; t < P.nsteps; t++) {
      bool f = P.count[t] > 0;
      for (int k = 0; k < P.count[t]; k++) f = f && P.m[(size_t)t * h + k] == kMaxPivot;
      full_step[t] = f;
    }
  auto enqueue_sweep = [&](bool use_mix, bool diag) {
    size_t k0 = prof.mark();
    launch_reset_stats(d_st, stream);
    prof.done(JJ_K_OTHER, k0, 0);
    if (diag) {
      PivotList dl{d_dcols, d_dsg, d_dm, d_dnf, P.nbl};
      gram_pivot(use_mix, dl, d_part, d_W, d_rot, d_promote_diag, 0, inner_max);
      k0 = prof.arm();
      update(G, ldg, m, dl, d_W, d_rot, rows_u, stream, Batch(), 0);
      prof.done_kernel(JJ_K_UPDATE, k0, 0);
    }
    for (int t = 0; t < P.nsteps && three; t++) {
      // three-level step (Section 5.3 with step 3 by the blocked method,
      // Algorithm 5.1): Gram blocks of the six sub-pivots of every pair, A_P =
      // R^* R, then the inner steps on R, each inner transformation applied to
      // R and to the pair's columns of G
      const int cnt = P.count[t];
      if (cnt == 0) continue;
      const size_t pr0 = (size_t)t * h;
      PivotList vl{d_vcols + pr0 * 6 * kMaxPivot, d_isg, d_vm + pr0 * 6, d_vm + pr0 * 6, 6 * cnt};
      k0 = prof.arm();
      gram64(G, ldg, m, vl, nch3, rows_g3, d_vpart, stream, Batch(), nullptr);
      prof.done_kernel(JJ_K_GRAM, k0, vl.count);
      k0 = prof.arm();
      launch_chol128(cplx != 0, d_vpart, nch3, m, rows_g3, d_n1 + pr0, d_n2 + pr0, cnt, d_RW, kMaxPivot3, t == 0,
                     d_st, stream);
      prof.done_kernel(JJ_K_PIVOT, k0, 0);
      for (int sidx = t == 0 ? 0 : 1; sidx < 3; sidx++) {
        const size_t base = ((size_t)t * 3 + sidx) * h * 2;
        PivotList ilR{d_icolR + base * kMaxPivot, d_isg + base * kMaxPivot, d_im + base, d_inf + base, 2 * cnt};
        PivotList ilG{d_icolG + base * kMaxPivot, d_isg + base * kMaxPivot, d_im + base, d_inf + base, 2 * cnt};
        k0 = prof.arm();
        gram64(d_RW, kMaxPivot3, kMaxPivot3, ilR, 1, kMaxPivot3, d_ipart, stream, Batch(), nullptr);
        prof.done_kernel(JJ_K_GRAM, k0, 0);
        k0 = prof.arm();
        pivot(d_ipart, 1, kMaxPivot3, kMaxPivot3, ilR, tol, tol, 1, sidx == 0 ? 0 : 1, 0, d_iW, d_irot, d_st, stream,
              Batch(), nullptr, nullptr, d_RW, kMaxPivot3);
        prof.done_kernel(JJ_K_PIVOT, k0, ilR.count);
        k0 = prof.arm();
        update(d_RW, kMaxPivot3, kMaxPivot3, ilR, d_iW, d_irot, 64, stream, Batch(), 0);
        prof.done_kernel(JJ_K_UPDATE, k0, 0);
        k0 = prof.arm();
        update(G, ldg, m, ilG, d_iW, d_irot, rows_u3, stream, Batch(), 0);
        prof.done_kernel(JJ_K_UPDATE, k0, 0);
      }
    }
    for (int t = 0; t < P.nsteps && !three; t++) {
      PivotList pl{d_cols + (size_t)t * h * kMaxPivot, d_sg + (size_t)t * h * kMaxPivot, d_m + (size_t)t * h,
                   d_nf + (size_t)t * h, P.count[t]};
      pl.full = full_step[t];
      if (pl.count == 0) continue;
      // Block-oriented variant (Section 5.3): the first step of a sweep makes one
      // full pass over its pivots (covering every diagonal block), the other
      // steps one pass over the off-diagonal block only.  With two blocks the
      // single pivot is the whole matrix, and it is diagonalised in full
      // (Section 3.3) instead of one pass per sweep.
      const bool block_oriented = imode == 0 && P.nbl > 2;
      const int mode = (block_oriented && t > 0) ? 1 : 0;  // kernel mode 1: off-diagonal pass only
      const int imax = block_oriented ? 1 : inner_max;
      gram_pivot(use_mix, pl, d_part, d_W, d_rot, d_promote + (size_t)t * h, mode, imax);
      k0 = prof.arm();
      update(G, ldg, m, pl, d_W, d_rot, rows_u, stream, Batch(), 0);
      prof.done_kernel(JJ_K_UPDATE, k0, 0);
    }
  };
  // Dataflow form of a sweep.  The pairs of each step are split into G
  // contiguous groups (tasks: Gram, pivot solve, update of the group's pairs).
  // The sweep is captured in the sequential order on one stream, which makes a
  // chain of kernel nodes; the chain edges between tasks are then replaced by
  // the true dependencies: a task follows the tasks that last touched its
  // blocks.  Groups of consecutive steps then overlap in the graph (a group's
  // latency-bound pivot solves run beside other groups' Gram and update
  // kernels), and every task still reads exactly the data the sequential order
  // gives it, so the results are those of the eager sweep.
  const int wsz = cplx ? 2 : 1;
  const int ngrp = (o.step_groups <= 1 || h < 8 || three) ? 1 : std::min(o.step_groups, std::min(h / 4, kMaxStepGroups));
  struct Task {
    hipGraphNode_t first, last;
    std::vector<int> deps;
  };
  auto last_node = [&]() -> hipGraphNode_t {
    hipStreamCaptureStatus cs;
    unsigned long long id = 0;
    hipGraph_t cg = nullptr;
    const hipGraphNode_t* leaf = nullptr;
    size_t nleaf = 0;
    ck(hipStreamGetCaptureInfo_v2(stream, &cs, &id, &cg, &leaf, &nleaf), "capture info");
    if (cs != hipStreamCaptureStatusActive || nleaf != 1) ck(hipErrorUnknown, "capture: not a single chain");
    return leaf[0];
  };
  // captures the sequential sweep and returns its tasks (root node in *reset)
  auto capture_sweep_tasks = [&](bool use_mix, bool diag, hipGraphNode_t* reset, std::vector<Task>& tasks) {
    launch_reset_stats(d_st, stream);
    *reset = last_node();
    std::vector<int> owner(P.nbl, -1);  // last task to touch each block
    auto run_task = [&](const std::vector<int>& blocks, PivotList pl, size_t s0, int mode, int imax, int* promote) {
      Task tk;
      for (int b : blocks)
        if (owner[b] >= 0) tk.deps.push_back(owner[b]);
      std::sort(tk.deps.begin(), tk.deps.end());
      tk.deps.erase(std::unique(tk.deps.begin(), tk.deps.end()), tk.deps.end());
      double* part = d_part + s0 * nch * kMaxPivot * kMaxPivot * wsz;
      double* W = d_W + s0 * kMaxPivot * kMaxPivot * wsz;
      int* rot = d_rot + s0;
      gram_pivot(use_mix, pl, part, W, rot, promote + s0, mode, imax, [&]() { tk.first = last_node(); });
      update(G, ldg, m, pl, W, rot, rows_u, stream, Batch(), 0);
      tk.last = last_node();
      for (int b : blocks) owner[b] = (int)tasks.size();
      tasks.push_back(std::move(tk));
    };
    if (diag) {
      const int q = (P.nbl + ngrp - 1) / ngrp;
      for (int g = 0; g < ngrp; g++) {
        const int s0 = g * q, cnt = std::min(P.nbl, s0 + q) - s0;
        if (cnt <= 0) continue;
        std::vector<int> blocks;
        for (int l = s0; l < s0 + cnt; l++) blocks.push_back(l);
        PivotList dl{d_dcols + (size_t)s0 * kMaxPivot, d_dsg + (size_t)s0 * kMaxPivot, d_dm + s0, d_dnf + s0, cnt};
        run_task(blocks, dl, s0, 0, inner_max, d_promote_diag);
      }
    }
    const bool block_oriented = imode == 0 && P.nbl > 2;
    const int imax = block_oriented ? 1 : inner_max;
    for (int t = 0; t < P.nsteps; t++) {
      const int count = P.count[t];
      const int q = (count + ngrp - 1) / ngrp;
      const int mode = (block_oriented && t > 0) ? 1 : 0;
      for (int g = 0; g < ngrp; g++) {
        const int s0 = g * q, cnt = std::min(count, s0 + q) - s0;
        if (cnt <= 0) continue;
        std::vector<int> blocks;
        for (int k = s0; k < s0 + cnt; k++) {
          blocks.push_back(P.pblocks[((size_t)t * h + k) * 2]);
          blocks.push_back(P.pblocks[((size_t)t * h + k) * 2 + 1]);
        }
        const size_t base = (size_t)t * h + s0;
        PivotList pl{d_cols + base * kMaxPivot, d_sg + base * kMaxPivot, d_m + base, d_nf + base, cnt};
        run_task(blocks, pl, s0, mode, imax, d_promote + (size_t)t * h);
      }
    }
  };
  // chain edges between consecutive tasks -> dependency edges
  auto rewire = [&](hipGraph_t g, hipGraphNode_t reset, const std::vector<Task>& tasks) {
    for (size_t i = 0; i < tasks.size(); i++) {
      const hipGraphNode_t prev = i == 0 ? reset : tasks[i - 1].last;
      ck(hipGraphRemoveDependencies(g, &prev, &tasks[i].first, 1), "remove edge");
      if (tasks[i].deps.empty()) {
        ck(hipGraphAddDependencies(g, &reset, &tasks[i].first, 1), "add edge");
      } else {
        for (int d : tasks[i].deps) ck(hipGraphAddDependencies(g, &tasks[d].last, &tasks[i].first, 1), "add edge");
      }
    }
  };
  SweepGraphs graphs;
  // At most kMaxPivot columns and rows (two blocks: a single pivot holding the
  // whole matrix): the non-blocked process on G itself in one pivot launch
  // (Algorithm 3.2, inner sweeps until one applies no rotation, capped by
  // max_sweeps), no update.  The Gram block and its Cholesky factor serve only
  // the full-rank test of the blocked steps.  sweeps counts the inner sweeps.
  const bool direct = P.nbl == 2 && P.nsteps == 1 && m == n && n <= kMaxPivot && !mixed && o.diag_pass == 0;
  if (direct) {
    PivotList pl{d_cols, d_sg, d_m, d_nf, P.count[0]};
    gram_pivot(false, pl, d_part, d_W, d_rot, nullptr, 3, max_sweeps);
    ck(hipGetLastError(), "launch");
    ck(hipMemcpyAsync(&hst, d_st, sizeof(hst), hipMemcpyDeviceToHost, stream), "D2H");
    ck(hipStreamSynchronize(stream), "sync");
    prof.flush();
    sweep = (int)hst.inner_sweeps;
    piv_rot = hst.rotations > 0 ? 1 : 0;
    prof.acc.rotations += (long long)hst.rotations;
    prof.acc.inner_sweeps += (long long)hst.inner_sweeps;
    prof.acc.pivot_cols += (long long)hst.pivot_cols;
    prof.acc.pivot_cols3 += (long long)hst.pivot_cols3;
    if (hst.breakdown)
      breakdown = true;
    else if (hst.pivots_rotated == 0)
      status = JJ_OK;
  }
  while (!direct && P.nbl >= 2 && sweep < max_sweeps) {
    sweep++;
    const bool use_mix = mixed;
    const bool diag = o.diag_pass == 2 || (o.diag_pass == 1 && sweep == 1);
    if (prof.on || !graphs_ok) {
      enqueue_sweep(use_mix, diag);
    } else {
      hipGraphExec_t& ex = graphs.at(use_mix, diag);
      if (ex == nullptr) {
        hipGraph_t g = nullptr;
        hipGraphNode_t reset = nullptr;
        std::vector<Task> tasks;
        ck(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
          if (ngrp > 1)
            capture_sweep_tasks(use_mix, diag, &reset, tasks);
          else
            enqueue_sweep(use_mix, diag);
        } catch (...) {
          (void)hipStreamEndCapture(stream, &g);
          if (g != nullptr) (void)hipGraphDestroy(g);
          throw;
        }
        ck(hipStreamEndCapture(stream, &g), "end capture");
        if (ngrp > 1) {
          try {
            rewire(g, reset, tasks);
          } catch (...) {
            (void)hipGraphDestroy(g);
            throw;
          }
        }
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        ck(ie, "instantiate");
      }
      ck(hipGraphLaunch(ex, stream), "graph launch");
    }
    ck(hipGetLastError(), "launch");
    ck(hipMemcpyAsync(&hst, d_st, sizeof(hst), hipMemcpyDeviceToHost, stream), "D2H");
    ck(hipStreamSynchronize(stream), "sync");
    prof.flush();
    double off;
    std::memcpy(&off, &hst.max_off_bits, sizeof(off));
    last_off = off;
    piv_rot += hst.pivots_rotated;
    prof.acc.units[JJ_K_UPDATE] += hst.pivots_rotated;
    prof.acc.rotations += (long long)hst.rotations;
    prof.acc.inner_sweeps += (long long)hst.inner_sweeps;
    prof.acc.pivot_cols += (long long)hst.pivot_cols;
    prof.acc.pivot_cols3 += (long long)hst.pivot_cols3;
    if (hst.breakdown) {
      breakdown = true;
      break;
    }
    if (o.history != nullptr && sweep <= o.history_len) o.history[sweep - 1] = off;
    if (use_mix) {
      // leave FP32 Gram blocks once they are accurate enough to finish in FP64
      // or once no pivot rotates (pivots whose FP32 block could not be
      // factored were re-solved from FP64 blocks within their step)
      mixed_sweeps++;
      mixed_resolved += hst.soft_fail;
      if (off < mix_switch || hst.pivots_rotated == 0) mixed = false;
      continue;
    }
    if (hst.pivots_rotated == 0) {
      status = JJ_OK;
      break;
    }
  }

  e0 = prof.mark();
  launch_reset_stats(d_st, stream);
  prof.done(JJ_K_OTHER, e0, 0);
  e0 = prof.mark();
  launch_finalize(G, ldg, m, n, cplx, d_colmap, d_sgn, d_d, d_rank, lambda, V, ldv, d_st, stream);
  prof.done(JJ_K_FINAL, e0, n);
  ck(hipGetLastError(), "launch");
  ck(hipMemcpyAsync(&hst, d_st, sizeof(hst), hipMemcpyDeviceToHost, stream), "D2H");
  ck(hipStreamSynchronize(stream), "sync");
  prof.flush();
  if (prof.on) {
    prof.acc.n = n;
    prof.acc.nblocks = P.nbl;
    prof.acc.block_width = P.nbl >= 1 && P.off.size() > 1 ? P.off[1] - P.off[0] : 0;
    prof.acc.sweeps = sweep;
    prof.acc.dtype = dtype;
    prof.acc.valid = 1;
    g_last_prof = prof.acc;
    g_have_prof = true;
  }
  if (breakdown || hst.zero_col) status = JJ_BREAKDOWN;

  if (info) {
    info->status = status;
    info->sweeps = sweep;
    info->block_width = P.nbl >= 1 ? (P.off.size() > 1 ? P.off[1] - P.off[0] : 0) : 0;
    info->nblocks = P.nbl;
    info->pivots_rotated = piv_rot;
    info->final_offdiag = last_off;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->mixed_sweeps = mixed_sweeps;
    info->mixed_resolved = mixed_resolved;
    info->inner_mode = imode;
  }
  return status;
}


// ---------------------------------------------------------------------------
// Batched solves.  All problems advance together: one launch per kernel kind
// covers the current step of every active problem (slots map statically to
// (problem, pair)); each problem keeps its own step / sweep counters and
// convergence test on the device (k_batch_advance), so a round of steps needs
// no host decision and is captured once in a HIP graph and replayed until no
// problem is active.  Real and complex problems use their own launches.
// ---------------------------------------------------------------------------

// Autotuner: block width per (dtype, size bucket), chosen by timing two
// candidate widths on a copy of the first problem of the bucket (two sweeps
// each) and cached for the process.  Each candidate first runs one untimed
// sweep: the first solves of a process grow the workspace cache, and that
// cost, charged to whichever candidate ran first, outweighed two sweeps of a
// small problem and picked the slower width.


static int tune_block_width(int dtype, void* G, const signed char* J, int n, int ldg, hipStream_t stream,
                            bool wide, bool modes) {
  const int w = dtype == JJ_C128 ? 2 : 1;
  if (n <= 64) return 32 * 2;  // one pivot holds the whole problem for either width
  const size_t gsz = (size_t)n * n * w * sizeof(double);
  double *Gc = nullptr, *lam = nullptr, *V = nullptr;
  ck(hipMalloc((void**)&Gc, gsz), "hipMalloc tune");
  ck(hipMalloc((void**)&lam, n * sizeof(double)), "hipMalloc tune");
  ck(hipMalloc((void**)&V, gsz), "hipMalloc tune");
  hipEvent_t e0, e1;
  ck(hipEventCreate(&e0), "event");
  ck(hipEventCreate(&e1), "event");
  // Up to n = 2048 each candidate runs a whole solve (time to solution: the
  // candidates need different sweep counts); above, two sweeps (a solve there
  // takes from 0.2 s to seconds, and the measured sweep counts of the widths
  // differ by a few percent).  The full-diagonalisation variant needs far fewer
  // sweeps at a far higher cost per sweep, so it is a candidate only where
  // whole solves are timed, up to n = 1024.
  const bool whole = n <= 2048;
  std::vector<std::pair<int, int>> cand = {{32, 0}, {16, 0}};
  if (wide) cand.push_back({64, 0});
  if (modes && n <= 1024) {
    cand.push_back({32, 1});
    cand.push_back({16, 1});
  }
  int best = 32 * 2;
  float best_ms = 1e30f;
  for (const auto& c : cand) {  // untimed: workspace growth and first launches
    ck(hipMemcpy2DAsync(Gc, (size_t)n * w * sizeof(double), G, (size_t)ldg * w * sizeof(double),
                        (size_t)n * w * sizeof(double), n, hipMemcpyDeviceToDevice, stream),
       "copy tune");
    jj_opts o;
    jjacobi_default_opts(&o);
    o.stream = stream;
    o.block_width = c.first;
    o.inner_mode = c.second;
    solve_one(dtype, Gc, J, n, n, lam, V, n, 0.0, 1, o, nullptr, false);
  }
  for (const auto& c : cand) {
    ck(hipMemcpy2DAsync(Gc, (size_t)n * w * sizeof(double), G, (size_t)ldg * w * sizeof(double),
                        (size_t)n * w * sizeof(double), n, hipMemcpyDeviceToDevice, stream),
       "copy tune");
    jj_opts o;
    jjacobi_default_opts(&o);
    o.stream = stream;
    o.block_width = c.first;
    o.inner_mode = c.second;
    ck(hipEventRecord(e0, stream), "event");
    solve_one(dtype, Gc, J, n, n, lam, V, n, 0.0, whole ? 0 : 2, o, nullptr, whole);
    ck(hipEventRecord(e1, stream), "event");
    ck(hipEventSynchronize(e1), "event");
    float ms = 0.f;
    ck(hipEventElapsedTime(&ms, e0, e1), "event");
    if (ms < best_ms) {
      best_ms = ms;
      best = c.first * 2 + c.second;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(Gc);
  hipFree(lam);
  hipFree(V);
  return best;
}


struct GroupTables {
  std::vector<int> cols, m, nfirst, slot_prob, slot_k;
  std::vector<signed char> sg;
  int slots = 0, nmax = 0;
};

static int solve_batch(int count, const int* dtype, void* const* G, const signed char* const* J, const int* n,
                       const int* ldg, double* const* lambda, void* const* V, const int* ldv, double tol,
                       int max_sweeps, const jj_opts& o, jj_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t caller = (hipStream_t)o.stream;
  if (max_sweeps <= 0) max_sweeps = 100;

  // block width per problem: fixed by the caller, or tuned per (dtype, size bucket)
  std::vector<int> bw(count);
  for (int i = 0; i < count; i++) {
    if (o.block_width > 0) {
      bw[i] = std::min(o.block_width, kMaxBlock);
      continue;
    }
    bw[i] = tuned_block_width(dtype[i], G[i], J[i], n[i], ldg[i], caller) >> 1;
  }

  // per-problem plans; tables concatenated per dtype group
  std::vector<Plan> plans;
  plans.reserve(count);
  GroupTables grp[2];
  std::vector<int> tab_base(count, 0), npairs(count, 0), nsteps(count, 0), width(count), cm_off(count + 1, 0);
  std::vector<int> colmap_all;
  std::vector<signed char> sgn_all;
  for (int i = 0; i < count; i++) {
    plans.push_back(make_plan(n[i], J[i], bw[i], o.strategy));
    const Plan& P = plans.back();
    const int g = dtype[i] == JJ_C128 ? 1 : 0;
    width[i] = g ? 2 : 1;
    cm_off[i + 1] = cm_off[i] + n[i];
    colmap_all.insert(colmap_all.end(), P.colmap.begin(), P.colmap.end());
    sgn_all.insert(sgn_all.end(), P.sgn.begin(), P.sgn.end());
    if (P.nbl < 2 || P.nsteps == 0) continue;
    GroupTables& T = grp[g];
    const int h = P.npairs_max;
    // steps with fewer pairs (modulus pairing) keep m = 0 entries: such slots do nothing
    tab_base[i] = (int)T.m.size();
    npairs[i] = h;
    nsteps[i] = P.nsteps;
    T.cols.insert(T.cols.end(), P.cols.begin(), P.cols.end());
    T.sg.insert(T.sg.end(), P.sgp.begin(), P.sgp.end());
    T.m.insert(T.m.end(), P.m.begin(), P.m.end());
    T.nfirst.insert(T.nfirst.end(), P.nfirst.begin(), P.nfirst.end());
    for (int k = 0; k < h; k++) {
      T.slot_prob.push_back(i);
      T.slot_k.push_back(k);
    }
    T.slots += h;
    T.nmax = std::max(T.nmax, n[i]);
  }

  // device workspace
  int rows_g[2], nch_u[2];
  for (int g = 0; g < 2; g++) {
    rows_g[g] = std::max(64, (grp[g].nmax + 63) / 64 * 64);  // one Gram chunk per slot
    nch_u[g] = std::max(1, (grp[g].nmax + 255) / 256);
  }
  Carver c{nullptr};
  auto layout = [&](Carver& cv, bool fill, std::vector<void*>& ptrs) {
    auto take = [&](size_t bytes) {
      void* p = cv.take<char>(bytes);
      if (fill) ptrs.push_back(p);
      return p;
    };
    for (int g = 0; g < 2; g++) {
      const GroupTables& T = grp[g];
      const size_t S = std::max(T.slots, 1);
      take(std::max<size_t>(T.cols.size(), 1) * sizeof(int));
      take(std::max<size_t>(T.sg.size(), 1));
      take(std::max<size_t>(T.m.size(), 1) * sizeof(int));
      take(std::max<size_t>(T.nfirst.size(), 1) * sizeof(int));
      take(S * sizeof(int));                                          // slot_prob
      take(S * sizeof(int));                                          // slot_k
      take(S * kMaxPivot * kMaxPivot * (g + 1) * sizeof(double));     // partials (one chunk)
      take(S * kMaxPivot * kMaxPivot * (g + 1) * sizeof(double));     // W
      take(S * sizeof(int));                                          // rotflag
    }
    take(count * sizeof(double*));  // gptr
    for (int k = 0; k < 9; k++) take(count * sizeof(int));  // ldg nrow width npairs nsteps step sweep active status
    take(count * sizeof(int));      // tab_base
    take(count * sizeof(SweepStats));
    take(count * sizeof(double));   // final_off
    take(count * sizeof(double));   // tol
    take(count * sizeof(int));      // bad
    take(count * sizeof(int));      // zero_col
    take((count + 1) * sizeof(int));  // cm_off
    take(std::max<size_t>(colmap_all.size(), 1) * sizeof(int));
    take(std::max<size_t>(sgn_all.size(), 1));
    take(count * sizeof(double*));  // lambda ptrs
    take(count * sizeof(double*));  // V ptrs
    take(count * sizeof(int));      // ldv
    take(std::max<size_t>(colmap_all.size(), 1) * sizeof(double));  // dwork
    take(std::max<size_t>(colmap_all.size(), 1) * sizeof(int));     // rkwork
    take(sizeof(int));              // active count
    take(count * sizeof(int));      // prec (1: mixed sweeps)
    take(count * sizeof(int));      // mixed sweeps
  };
  std::vector<void*> ptrs;
  layout(c, false, ptrs);
  Carver cv{arena_get(c.off + 256)};
  layout(cv, true, ptrs);
  size_t pi = 0;
  struct DevGroup {
    int *cols, *m, *nfirst, *slot_prob, *slot_k, *rot;
    signed char* sg;
    double *part, *W;
  } dg[2];
  for (int g = 0; g < 2; g++) {
    dg[g].cols = (int*)ptrs[pi++];
    dg[g].sg = (signed char*)ptrs[pi++];
    dg[g].m = (int*)ptrs[pi++];
    dg[g].nfirst = (int*)ptrs[pi++];
    dg[g].slot_prob = (int*)ptrs[pi++];
    dg[g].slot_k = (int*)ptrs[pi++];
    dg[g].part = (double*)ptrs[pi++];
    dg[g].W = (double*)ptrs[pi++];
    dg[g].rot = (int*)ptrs[pi++];
  }
  double** d_gptr = (double**)ptrs[pi++];
  int* d_ldg = (int*)ptrs[pi++];
  int* d_nrow = (int*)ptrs[pi++];
  int* d_width = (int*)ptrs[pi++];
  int* d_npairs = (int*)ptrs[pi++];
  int* d_nsteps = (int*)ptrs[pi++];
  int* d_step = (int*)ptrs[pi++];
  int* d_sweep = (int*)ptrs[pi++];
  int* d_active = (int*)ptrs[pi++];
  int* d_status = (int*)ptrs[pi++];
  int* d_tab_base = (int*)ptrs[pi++];
  SweepStats* d_st = (SweepStats*)ptrs[pi++];
  double* d_final_off = (double*)ptrs[pi++];
  double* d_tol = (double*)ptrs[pi++];
  int* d_bad = (int*)ptrs[pi++];
  int* d_zero = (int*)ptrs[pi++];
  int* d_cm_off = (int*)ptrs[pi++];
  int* d_colmap = (int*)ptrs[pi++];
  signed char* d_sgn = (signed char*)ptrs[pi++];
  double** d_lam = (double**)ptrs[pi++];
  double** d_V = (double**)ptrs[pi++];
  int* d_ldv = (int*)ptrs[pi++];
  double* d_dwork = (double*)ptrs[pi++];
  int* d_rkwork = (int*)ptrs[pi++];
  int* d_active_count = (int*)ptrs[pi++];
  int* d_prec = (int*)ptrs[pi++];
  int* d_msw = (int*)ptrs[pi++];

  hipStream_t s = lib_stream();
  hipEvent_t ev;
  ck(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  ck(hipEventRecord(ev, caller), "event");
  ck(hipStreamWaitEvent(s, ev, 0), "wait event");

  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (bytes) ck(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "H2D batch");
  };
  for (int g = 0; g < 2; g++) {
    const GroupTables& T = grp[g];
    up(dg[g].cols, T.cols.data(), T.cols.size() * sizeof(int));
    up(dg[g].sg, T.sg.data(), T.sg.size());
    up(dg[g].m, T.m.data(), T.m.size() * sizeof(int));
    up(dg[g].nfirst, T.nfirst.data(), T.nfirst.size() * sizeof(int));
    up(dg[g].slot_prob, T.slot_prob.data(), T.slot_prob.size() * sizeof(int));
    up(dg[g].slot_k, T.slot_k.data(), T.slot_k.size() * sizeof(int));
  }
  std::vector<double*> gp(count), lp(count), vp(count);
  std::vector<int> zeros(count, 0), ldg_v(count), n_v(count), ldv_v(count);
  for (int i = 0; i < count; i++) {
    gp[i] = (double*)G[i];
    lp[i] = lambda[i];
    vp[i] = (double*)V[i];
    ldg_v[i] = ldg[i];
    n_v[i] = n[i];
    ldv_v[i] = ldv[i];
  }
  up(d_gptr, gp.data(), count * sizeof(double*));
  up(d_ldg, ldg_v.data(), count * sizeof(int));
  up(d_nrow, n_v.data(), count * sizeof(int));
  up(d_width, width.data(), count * sizeof(int));
  up(d_npairs, npairs.data(), count * sizeof(int));
  up(d_nsteps, nsteps.data(), count * sizeof(int));
  up(d_step, zeros.data(), count * sizeof(int));
  up(d_sweep, zeros.data(), count * sizeof(int));
  up(d_status, zeros.data(), count * sizeof(int));
  up(d_tab_base, tab_base.data(), count * sizeof(int));
  up(d_bad, zeros.data(), count * sizeof(int));
  up(d_zero, zeros.data(), count * sizeof(int));
  std::vector<SweepStats> st0(count);
  std::memset(st0.data(), 0, count * sizeof(SweepStats));
  up(d_st, st0.data(), count * sizeof(SweepStats));
  std::vector<double> off0(count, 0.0);
  up(d_final_off, off0.data(), count * sizeof(double));
  up(d_cm_off, cm_off.data(), (count + 1) * sizeof(int));
  up(d_colmap, colmap_all.data(), colmap_all.size() * sizeof(int));
  up(d_sgn, sgn_all.data(), sgn_all.size());
  up(d_lam, lp.data(), count * sizeof(double*));
  up(d_V, vp.data(), count * sizeof(double*));
  up(d_ldv, ldv_v.data(), count * sizeof(int));

  // non-finite inputs are reported (status 3) and left out
  launch_batch_check_finite(count, d_gptr, d_ldg, d_nrow, d_width, d_bad, s);
  ck(hipGetLastError(), "launch");
  std::vector<int> bad(count);
  ck(hipMemcpyAsync(bad.data(), d_bad, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipStreamSynchronize(s), "sync");
  std::vector<int> active(count, 0), status(count, 0);
  int nactive = 0;
  for (int i = 0; i < count; i++) {
    if (bad[i]) status[i] = JJ_NONFINITE;
    active[i] = (!bad[i] && nsteps[i] > 0) ? 1 : 0;
    nactive += active[i];
  }
  up(d_active, active.data(), count * sizeof(int));
  up(d_status, status.data(), count * sizeof(int));
  up(d_active_count, &nactive, sizeof(int));
  // mixed precision (reading as for single solves): FP32-Gram sweeps per problem
  const bool mixed = o.precision == 1;
  const double mix_switch = o.mixed_switch > 0.0 ? o.mixed_switch : 0.1;
  std::vector<int> prec0(count, mixed ? 1 : 0), msw0(count, 0);
  up(d_prec, prec0.data(), count * sizeof(int));
  up(d_msw, msw0.data(), count * sizeof(int));

  // rotation threshold per problem: tol, or n * 2^-53 by default
  std::vector<double> ptol(count);
  for (int i = 0; i < count; i++) ptol[i] = tol > 0.0 ? tol : (double)n[i] * std::ldexp(1.0, -53);
  up(d_tol, ptol.data(), count * sizeof(double));
  const double btol = 0.0;  // unused: the pivot solver reads the per-problem value
  const bool block_oriented = o.inner_mode <= 0;
  const int pmode = block_oriented ? 2 : 0;
  const int imax = block_oriented ? 1 : (o.inner_max_sweeps > 0 ? o.inner_max_sweeps : 12);

  Batch bt[2];
  for (int g = 0; g < 2; g++) {
    bt[g].slot_prob = dg[g].slot_prob;
    bt[g].slot_k = dg[g].slot_k;
    bt[g].tab_base = d_tab_base;
    bt[g].npairs = d_npairs;
    bt[g].step = d_step;
    bt[g].active = d_active;
    bt[g].gptr = d_gptr;
    bt[g].ldg = d_ldg;
    bt[g].nrow = d_nrow;
    bt[g].st = d_st;
    bt[g].tol = d_tol;
    bt[g].prec = mixed ? d_prec : nullptr;
  }
  auto one_step = [&]() {
    for (int g = 0; g < 2; g++) {
      if (grp[g].slots == 0) continue;
      PivotList pl{dg[g].cols, dg[g].sg, dg[g].m, dg[g].nfirst, grp[g].slots};
      if (!mixed)
        (g ? launch_gram_c128 : launch_gram_f64)(nullptr, 0, 0, pl, 1, rows_g[g], dg[g].part, s, bt[g], nullptr);
      else  // one launch: FP64 for the problems in FP64 sweeps, FP32 MFMA for the others
        launch_gram_sel(g == 1, nullptr, 0, 0, pl, 1, rows_g[g], dg[g].part, s, bt[g], nullptr);
    }
    for (int g = 0; g < 2; g++) {
      if (grp[g].slots == 0) continue;
      PivotList pl{dg[g].cols, dg[g].sg, dg[g].m, dg[g].nfirst, grp[g].slots};
      (g ? launch_pivot_c128 : launch_pivot_f64)(dg[g].part, 1, 0, rows_g[g], pl, btol, btol, imax, pmode, 0, dg[g].W,
                                                 dg[g].rot, nullptr, s, bt[g], nullptr, nullptr, nullptr, 0);
    }
    for (int g = 0; g < 2; g++) {
      if (grp[g].slots == 0) continue;
      PivotList pl{dg[g].cols, dg[g].sg, dg[g].m, dg[g].nfirst, grp[g].slots};
      (g ? launch_update_c128 : launch_update_f64)(nullptr, 0, 0, pl, dg[g].W, dg[g].rot, 256, s, bt[g], nch_u[g]);
    }
    launch_batch_advance(count, d_nsteps, d_step, d_sweep, d_active, d_status, d_st, d_final_off, max_sweeps,
                         d_active_count, mixed ? d_prec : nullptr, d_msw, mix_switch, s);
  };

  // a round of steps captured once, replayed until no problem is active
  int max_steps = 0;
  for (int i = 0; i < count; i++) max_steps = std::max(max_steps, nsteps[i]);
  const int kRound = 8;
  const long long step_cap = (long long)max_sweeps * std::max(max_steps, 1) + kRound;
  int left = nactive;
  if (left > 0) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto capture = [&]() {
      if (exec != nullptr) (void)hipGraphExecDestroy(exec);
      if (graph != nullptr) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
      ck(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
      for (int r = 0; r < kRound; r++) one_step();
      ck(hipStreamEndCapture(s, &graph), "end capture");
      ck(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
    };
    capture();
    // Slot compaction: once the active problems fall to 3/5 of those the slot
    // lists were built for, the lists are rebuilt from the active problems
    // only and the round is captured again, so that finished problems stop
    // taking workgroups (each slot's W_P, partials and flags live only within a
    // step, so slots can be renumbered between rounds).
    int basis = left;
    std::vector<int> act(count);
    for (long long done = 0; left > 0 && done < step_cap; done += kRound) {
      ck(hipGraphLaunch(exec, s), "graph launch");
      ck(hipMemcpyAsync(&left, d_active_count, sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
      ck(hipStreamSynchronize(s), "sync");
      if (left > 0 && 5LL * left <= 3LL * basis) {
        ck(hipMemcpyAsync(act.data(), d_active, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
        ck(hipStreamSynchronize(s), "sync");
        for (int g = 0; g < 2; g++) {
          GroupTables& T = grp[g];
          std::vector<int> sp, sk;
          for (size_t q = 0; q < T.slot_prob.size(); q++)
            if (act[T.slot_prob[q]]) {
              sp.push_back(T.slot_prob[q]);
              sk.push_back(T.slot_k[q]);
            }
          T.slots = (int)sp.size();
          up(dg[g].slot_prob, sp.data(), sp.size() * sizeof(int));
          up(dg[g].slot_k, sk.data(), sk.size() * sizeof(int));
          ck(hipStreamSynchronize(s), "sync");
        }
        basis = left;
        capture();
      }
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
  }

  launch_batch_finalize(count, d_gptr, d_ldg, d_nrow, d_width, d_colmap, d_cm_off, d_sgn, d_lam, d_V, d_ldv, d_dwork,
                        d_rkwork, d_zero, s);
  ck(hipGetLastError(), "launch");
  std::vector<int> zero(count), sweeps(count), msw(count);
  std::vector<double> foff(count);
  ck(hipMemcpyAsync(status.data(), d_status, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipMemcpyAsync(active.data(), d_active, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipMemcpyAsync(zero.data(), d_zero, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipMemcpyAsync(sweeps.data(), d_sweep, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipMemcpyAsync(foff.data(), d_final_off, count * sizeof(double), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipMemcpyAsync(msw.data(), d_msw, count * sizeof(int), hipMemcpyDeviceToHost, s), "D2H");
  ck(hipStreamSynchronize(s), "sync");
  hipEventDestroy(ev);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = 0;
  for (int i = 0; i < count; i++) {
    int st = status[i];
    if (active[i]) st = JJ_NOT_CONVERGED;  // step cap reached
    if (st == JJ_OK && zero[i]) st = JJ_BREAKDOWN;
    worst = std::max(worst, st);
    if (info) {
      std::memset(&info[i], 0, sizeof(jj_info));
      info[i].status = st;
      info[i].sweeps = sweeps[i];
      info[i].block_width = plans[i].nbl >= 1 && plans[i].off.size() > 1 ? plans[i].off[1] - plans[i].off[0] : 0;
      info[i].nblocks = plans[i].nbl;
      info[i].final_offdiag = foff[i];
      info[i].seconds = secs;
      info[i].mixed_sweeps = msw[i];
    }
  }
  return worst;
}

// Front end (Section 2.2, eq. 2.5): H (device, n x n, lower triangle read) ->
// G (device, n x n, ld ldg: the first r columns, the others zeroed), J and r on
// the host.  A step is a pivot-choice launch and an update launch; the n + 1
// steps are enqueued without host decisions (steps past the end return at
// once).  Returns 0, or JJ_NONFINITE.
static int bp_factor_dev(int dtype, const void* H, int n, int ldh, double* G, int ldg, signed char* J, int* rank,
                         double tol, hipStream_t stream) {
  const int w = dtype == JJ_C128 ? 2 : 1;
  if (tol <= 0.0) tol = (double)n * std::ldexp(1.0, -53);
  size_t need = 0;
  {
    Carver c{nullptr};
    c.take<double>((size_t)n * n * w);
    c.take<double>((size_t)n * 2 * w);
    c.take<BPPartial>(kBpGroups);
    c.take<BPState>(1);
    c.take<int>(n);
    c.take<int>(n);
    c.take<double>((size_t)2 * n);
    c.take<signed char>(n);
    need = c.off + 256;
  }
  Carver c{arena_get(need)};
  double* A = c.take<double>((size_t)n * n * w);
  double* pcol = c.take<double>((size_t)n * 2 * w);
  BPPartial* part = c.take<BPPartial>(kBpGroups);
  BPState* st = c.take<BPState>(1);
  int* perm = c.take<int>(n);
  int* piv = c.take<int>(n);
  double* dblk = c.take<double>((size_t)2 * n);
  signed char* Jd = c.take<signed char>(n);
  ck(hipMemcpy2DAsync(A, (size_t)n * w * sizeof(double), H, (size_t)ldh * w * sizeof(double),
                      (size_t)n * w * sizeof(double), n, hipMemcpyDeviceToDevice, stream),
     "copy H");
  launch_bp_init(st, perm, n, stream);
  launch_bp_update(A, n, w == 2, pcol, st, part, stream);  // the first search (no update yet)
  for (int step = 0; step <= n; step++) {
    launch_bp_select(A, n, w == 2, tol, pcol, st, part, perm, piv, dblk, stream);
    launch_bp_update(A, n, w == 2, pcol, st, part, stream);
  }
  launch_bp_build_g(A, n, w == 2, st, perm, piv, dblk, G, ldg, Jd, stream);
  ck(hipGetLastError(), "launch");
  BPState hst;
  ck(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, stream), "D2H");
  ck(hipMemcpyAsync(J, Jd, n, hipMemcpyDeviceToHost, stream), "D2H");
  ck(hipStreamSynchronize(stream), "sync");
  *rank = hst.nonfinite ? 0 : hst.rank;
  return hst.nonfinite ? JJ_NONFINITE : JJ_OK;
}

static int check_args(int dtype, const void* G, const signed char* J, int n, int ldg, const double* lambda,
                      const void* V, int ldv) {
  if (dtype != JJ_F64 && dtype != JJ_C128) return -1;
  if (n < 0) return -4;
  if (n == 0) return 0;
  if (!G) return -2;
  if (!J) return -3;
  if (ldg < std::max(1, n)) return -5;
  if (!lambda) return -6;
  if (!V) return -7;
  if (ldv < std::max(1, n)) return -8;
  for (int i = 0; i < n; i++)
    if (J[i] != 1 && J[i] != -1) return -3;
  return 0;
}

}  // namespace jj

using namespace jj;

extern "C" {

void jjacobi_default_opts(jj_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block_width = 0;  // library choice (tuned where it matters)
  o->inner_max_sweeps = 12;
  o->inner_mode = -1;  // library choice
  o->mixed_switch = 0.1;
}

int jjacobi_solve_ex(int dtype, void* G, const signed char* J, int n, int ldg, double* lambda, void* V, int ldv,
                     double tol, int max_sweeps, const jj_opts* opts, jj_info* info) {
  int a = check_args(dtype, G, J, n, ldg, lambda, V, ldv);
  if (a < 0) {
    if (info) info->status = a;
    return a;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    return solve_one(dtype, G, J, n, ldg, lambda, V, ldv, tol, max_sweeps, o, info);
  } catch (const HipFail&) {
    if (info) info->status = JJ_HIP_ERROR;
    return JJ_HIP_ERROR;
  }
}

int jjacobi_solve_noalloc(int dtype, void* G, const signed char* J, int n, int ldg, double* lambda, void* V,
                          int ldv, double tol, int max_sweeps, const jj_opts* opts, jj_info* info) {
  int a = check_args(dtype, G, J, n, ldg, lambda, V, ldv);
  if (a < 0) {
    if (info) info->status = a;
    return a;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    return solve_one(dtype, G, J, n, ldg, lambda, V, ldv, tol, max_sweeps, o, info, false, true);
  } catch (const ScratchTooSmall& e) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "the solve needs %zu bytes of device scratch; the fixed array holds %zu",
                  e.need, kScratchBytes);
    g_last_error = msg;
    if (info) info->status = JJ_SCRATCH_TOO_SMALL;
    return JJ_SCRATCH_TOO_SMALL;
  } catch (const HipFail&) {
    if (info) info->status = JJ_HIP_ERROR;
    return JJ_HIP_ERROR;
  }
}

int jjacobi_solve_rect(int dtype, void* G, const signed char* J, int m, int n, int ldg, double* lambda, void* V,
                       int ldv, double tol, int max_sweeps, const jj_opts* opts, jj_info* info) {
  int a = 0;
  if (dtype != JJ_F64 && dtype != JJ_C128)
    a = -1;
  else if (n < 0)
    a = -5;
  else if (m < n)
    a = -4;
  else if (n > 0) {
    if (!G)
      a = -2;
    else if (!J)
      a = -3;
    else if (ldg < m)
      a = -6;
    else if (!lambda)
      a = -7;
    else if (!V)
      a = -8;
    else if (ldv < m)
      a = -9;
    for (int i = 0; a == 0 && i < n; i++)
      if (J[i] != 1 && J[i] != -1) a = -3;
  }
  if (a < 0) {
    if (info) info->status = a;
    return a;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    return solve_one(dtype, G, J, n, ldg, lambda, V, ldv, tol, max_sweeps, o, info, true, false, m);
  } catch (const HipFail&) {
    if (info) info->status = JJ_HIP_ERROR;
    return JJ_HIP_ERROR;
  }
}

int jjacobi_factor(int dtype, const void* H, int n, int ldh, void* G, int ldg, signed char* J, int* rank, double tol,
                   const jj_opts* opts) {
  if (dtype != JJ_F64 && dtype != JJ_C128) return -1;
  if (n < 0) return -3;
  if (!rank) return -8;
  *rank = 0;
  if (n == 0) return 0;
  if (!H) return -2;
  if (ldh < n) return -4;
  if (!G) return -5;
  if (ldg < n) return -6;
  if (!J) return -7;
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    hipStream_t stream = lib_stream();
    StreamJoin join((hipStream_t)o.stream, stream);
    return bp_factor_dev(dtype, H, n, ldh, (double*)G, ldg, J, rank, tol, stream);
  } catch (const HipFail&) {
    return JJ_HIP_ERROR;
  }
}

int jjacobi_eigh(int dtype, void* H, int n, int ldh, double* lambda, void* V, int ldv, double tol, int max_sweeps,
                 const jj_opts* opts, jj_info* info) {
  if (dtype != JJ_F64 && dtype != JJ_C128) return -1;
  if (n < 0) return -3;
  if (info) std::memset(info, 0, sizeof(*info));
  if (n == 0) return 0;
  if (!H) return -2;
  if (ldh < n) return -4;
  if (!lambda) return -5;
  if (!V) return -6;
  if (ldv < n) return -7;
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    const int w = dtype == JJ_C128 ? 2 : 1;
    std::vector<signed char> J(n);
    int r = 0;
    int st;
    {
      hipStream_t stream = lib_stream();
      StreamJoin join((hipStream_t)o.stream, stream);
      // G overwrites H (H is copied into the workspace first)
      st = bp_factor_dev(dtype, H, n, ldh, (double*)H, ldh, J.data(), &r, 0.0, stream);
      if (st == JJ_OK && r < n)  // the zero eigenvalue (multiplicity n - r) at the end
        ck(hipMemsetAsync(lambda + r, 0, (size_t)(n - r) * sizeof(double), stream), "memset");
    }
    if (st != JJ_OK) {
      if (info) info->status = st;
      return st;
    }
    if (info) info->rank = r;
    if (r == 0) {
      // H = 0: every vector is an eigenvector; V = I
      hipStream_t stream = lib_stream();
      StreamJoin join((hipStream_t)o.stream, stream);
      launch_identity_tail(dtype == JJ_C128, (double*)V, n, ldv, 0, stream);
      ck(hipGetLastError(), "launch");
      ck(hipStreamSynchronize(stream), "sync");
      return JJ_OK;
    }
    st = solve_one(dtype, H, J.data(), r, ldh, lambda, V, ldv, tol, max_sweeps, o, info, true, false, n);
    if (info) info->rank = r;
    if (r < n && st <= JJ_NOT_CONVERGED) {
      // the eigenvectors of the zero eigenvalue: the complement of the r
      // eigenvectors, from the Householder QR of V[:, 0:r] (Section 2.2)
      hipStream_t stream = lib_stream();
      StreamJoin join((hipStream_t)o.stream, stream);
      Carver c{arena_get((size_t)2 * n * r * w * sizeof(double) + (size_t)r * sizeof(double) + 4096)};
      double* A = c.take<double>((size_t)n * r * w);
      double* Vh = c.take<double>((size_t)n * r * w);
      double* beta = c.take<double>(r);
      ck(hipMemcpy2DAsync(A, (size_t)n * w * sizeof(double), V, (size_t)ldv * w * sizeof(double),
                          (size_t)n * w * sizeof(double), r, hipMemcpyDeviceToDevice, stream),
         "copy U");
      launch_nullspace(dtype == JJ_C128, A, n, r, Vh, beta, (double*)V + (size_t)r * ldv * w, ldv, stream);
      ck(hipGetLastError(), "launch");
      ck(hipStreamSynchronize(stream), "sync");
    }
    return st;
  } catch (const HipFail&) {
    if (info) info->status = JJ_HIP_ERROR;
    return JJ_HIP_ERROR;
  }
}

int jjacobi_solve(double* G, const signed char* J, int n, int ldg, double* lambda, double* V, double tol,
                  int max_sweeps) {
  return jjacobi_solve_ex(JJ_F64, G, J, n, ldg, lambda, V, n, tol, max_sweeps, nullptr, nullptr);
}

int jjacobi_zsolve(void* G, const signed char* J, int n, int ldg, double* lambda, void* V, double tol,
                   int max_sweeps) {
  return jjacobi_solve_ex(JJ_C128, G, J, n, ldg, lambda, V, n, tol, max_sweeps, nullptr, nullptr);
}

int jjacobi_solve_batched(int count, const int* dtype, void* const* G, const signed char* const* J, const int* n,
                          const int* ldg, double* const* lambda, void* const* V, const int* ldv, double tol,
                          int max_sweeps, const jj_opts* opts, jj_info* info) {
  if (count < 0) return -1;
  if (count == 0) return 0;
  if (!dtype) return -2;
  if (!G) return -3;
  if (!J) return -4;
  if (!n) return -5;
  if (!ldg) return -6;
  if (!lambda) return -7;
  if (!V) return -8;
  if (!ldv) return -9;
  for (int k = 0; k < count; k++) {
    int a = check_args(dtype[k], G[k], J[k], n[k], ldg[k], lambda[k], V[k], ldv[k]);
    if (a < 0) return a;
  }
  jj_opts o;
  jjacobi_default_opts(&o);
  if (opts) o = *opts;
  std::lock_guard<std::mutex> lk(g_mutex);
  try {
    return solve_batch(count, dtype, G, J, n, ldg, lambda, V, ldv, tol, max_sweeps, o, info);
  } catch (const HipFail&) {
    if (info)
      for (int k = 0; k < count; k++) info[k].status = JJ_HIP_ERROR;
    return JJ_HIP_ERROR;
  }
}

const char* jjacobi_status_string(int status) {
  switch (status) {
    case 0:
      return "converged";
    case 1:
      return "not converged within max_sweeps";
    case 2:
      return "numerical breakdown: G is numerically rank deficient";
    case 3:
      return "non-finite input";
    case 4:
      return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
    case 5:
      return g_last_error.empty() ? "the solve needs more device scratch than jjacobi_solve_noalloc holds"
                                  : g_last_error.c_str();
    default:
      return status < 0 ? "invalid argument" : "unknown status";
  }
}

void jjacobi_release_workspace(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return;
  for (hipEvent_t e : Profiler::pool()) hipEventDestroy(e);
  Profiler::pool().clear();
  for (int d = 0; d < 64; d++)
    if (g_arena[d].base) {
      if (hipSetDevice(d) == hipSuccess) hipFree(g_arena[d].base);
      g_arena[d].base = nullptr;
      g_arena[d].cap = 0;
    }
  hipSetDevice(cur);
}

int jjacobi_last_profile(jj_profile* out) {
  if (!out || !g_have_prof) return -1;
  *out = g_last_prof;
  return 0;
}

// Host planning helpers exported for the CPU tests (no HIP calls).
int jjx_plan_nblocks(int n, int nt) { return plan_nblocks(n, nt); }
void jjx_plan_offsets(int n, int nbl, int* off) { plan_offsets(n, nbl, off); }
void jjx_plan_round_robin(int nbl, int* pairs) { plan_round_robin(nbl, pairs); }
int jjx_plan_modulus(int nbl, int* pairs, int* counts) { return plan_modulus(nbl, pairs, counts); }
void jjx_plan_sign_order(int n, const signed char* J, int* colmap) { plan_sign_order(n, J, colmap); }
int jjx_check_args(int dtype, const void* G, const signed char* J, int n, int ldg, const double* lambda,
                   const void* V, int ldv) {
  return check_args(dtype, G, J, n, ldg, lambda, V, ldv);
}

}  // extern "C"
