// kern.hpp -- device state and kernels of the branch-and-bound sweep.
//
// One sweep (Sec. 3.1, one iteration; Sec. 3.2, partition with variable cycling):
//   k_select       (one workgroup) insert the previous sweep's surviving
//                  children (cutoff with that sweep's final GUB, first-order
//                  test), stop test on [GLB, GUB], pick the live box with the
//                  smallest (lower bound, insertion number), rebuild its row from
//                  its parent row and child index, fix its m split coordinates.
//                  Large lists are scanned first by k_select_part.
//   k_bound<FAM,W> W wavefronts per child: F over the child, the first-order
//                  test, then (unless F.lo already exceeds the running GUB) the
//                  upper bound of f at the child midpoint -> atomicMin on GUB.
// Live boxes are kept compactly, as the paper's memory-limited list does
// (Sec. 3.2: an index, the iteration it came from, the cycling index and the
// lower bound): a key holds the lower bound, an insertion number, the row of
// the selected parent it was cut from and its child index.  The rows of the
// selected parents (one per sweep, 16 n bytes) stay in HBM.
#pragma once
#include "fam.hpp"

namespace ibb {

constexpr int kWave = 64;

// Everything a Params or State pointer reaches is device (global) memory.
// Accesses through G(p) compile to global loads and stores: LDS waits do not
// wait for them (accesses through generic pointers count against both).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}
// a record (a multiple of 8 bytes) read from device memory with global loads
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  static_assert(sizeof(T) % 8 == 0, "whole 8-byte words");
  T v;
  const gptr<const uint64_t> src = G(reinterpret_cast<const uint64_t*>(p));
  uint64_t* dst = reinterpret_cast<uint64_t*>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 8); ++k) dst[k] = src[k];
  return v;
}
constexpr int kBoundWaves = 4;            // waves per workgroup in the bound kernels
constexpr int kMaxSplit = 16;             // M <= 16
constexpr int kSelThreads = 256;
constexpr int kSelSingleThreads = 1024;   // the one-workgroup selection
constexpr int kSweepThreads = 512;        // persistent sweeps (room for 256 registers per lane)
constexpr int kSelIbThreads = 512;        // per-sweep selection with incremental bounds (likewise)
constexpr int kMaxSelBlocks = 1024;
constexpr int64_t kPersistentMaxKeys = (int64_t)1 << 18;   // lists one workgroup scans about as fast as a grid
constexpr int64_t kPersistentGrowth = (int64_t)1 << 17;      // keys a persistent launch may add (sets its sweeps)

// STOP_CAPACITY: the next sweep would pass the row or key capacity the host sized
// the arrays for (the host grows them before every chunk, so this only guards)
// STOP_INTERNAL: the selection counted live keys but found none to take (a guard)
// STOP_MEMORY: never set on the device; a run the server stopped at its memory
// budget ends with STOP_SWEEPS and reports this code instead
enum StopCode { RUNNING = 0, STOP_CONVERGED = 1, STOP_SWEEPS = 2, STOP_LIVE = 3, STOP_EMPTY = 4, STOP_HOST = 5,
                STOP_CAPACITY = 6, STOP_INTERNAL = 7, STOP_MEMORY = 8 };

// A bound that came out NaN says nothing about f: as a lower bound it counts as
// -inf (the box is kept and can never be cut off), as an upper bound as +inf (it
// never lowers GUB).  Validated inputs do not produce NaN; this keeps rigour and
// keeps every index the selection derives from the keys in range if one did.
__device__ __forceinline__ double lo_or_ninf(double v) { return v == v ? v : -__builtin_inf(); }
__device__ __forceinline__ double hi_or_inf(double v) { return v == v ? v + 0.0 : __builtin_inf(); }

// one box selected in a sweep that takes K > 1 boxes: its insertion number, the
// row its real endpoints were written to, its cycling index and split mask
struct SelRec {
  int64_t seq;
  int32_t row, cyc;
  uint32_t mask, pad;
};
constexpr int kMaxSelectK = 1024;         // K <= 1024 boxes per sweep
constexpr int kMaxSamples = 16;           // diagonal samples per child
// piece tables of one sweep (four pieces per split coordinate): at most
// kTabRows affected terms (combinations of the pieces of their one or two
// coordinates) and kTabRows affected derivative coordinates (pieces of up to
// three coordinates)
constexpr int kTabRows = 48;
constexpr int kTabEntry = 2 + kMaxSamples;   // F (-lo, hi), then the sample upper bounds
constexpr int kTabDoubles = kTabRows * 16 * kTabEntry + 2 + kMaxSamples + 1 + kMaxSplit * 4;
constexpr int kTabInts = 4 + kTabRows * (1 + 2) + kTabRows * (1 + 3) + kTabRows * 64;

struct KselBuf;

// the generic family: an expression tape (layout of the encoding in ibb.h)
constexpr int kTapeMaxOps = 32;   // ops per program
constexpr int kTapeMaxRed = 8;    // reductions
struct TapeOp {
  int32_t code, a, b, pad;
  double lo, hi;                  // the constant [lo, hi] of code 0
};
struct TapeRed {
  int32_t kind, start, stop;      // 0 sum, 1 product; i in [start, stop)
  int32_t first, nops;            // its program: op[first .. first + nops)
  int32_t pad;
};
struct TapeDev {
  int32_t K, Q, C, sc_first;      // the scalar program: op[sc_first .. sc_first + Q)
  int32_t nprod, pad;             // product reductions (each needs n workspace intervals per box)
  TapeRed red[kTapeMaxRed];
  TapeOp op[kTapeMaxOps * (kTapeMaxRed + 1)];
};

struct Params {
  int32_t family, n, m, nch;              // nch = 2^m children per selected box
  double tol_f, tol_x;
  int64_t max_sweeps, max_live;
  const CoefSep* sep;                     // [n] (separable families)
  const CoefChain* chain;                 // [n] (CHAIN; entry n-1 is zero)
  int32_t prec32;                         // 1: the FP32 filter may run (the sweep's State.use32 decides)
  int32_t incremental;                    // 1: children are bounded by the selection workgroup from the
                                          //    parent's shared terms (no bound kernel)
  const CoefSep32* sep32;                 // [n] float enclosures of the coefficients (filter only)
  const CoefChain32* chain32;             // [n]
  const double* nl;                       // [n] -l
  const double* u;                        // [n]  u
  // live-box keys
  double* key_flo;
  int64_t* key_seq;
  int32_t* key_ref;                       // row of the parent the box was cut from
  int32_t* key_r;                         // child index, or -1: the box is that row itself
  double* key_wmax;                       // widest side of the box (rounded up)
  int64_t key_cap;
  // rows of selected boxes, stored as (-lo, hi)
  double* hist_n;
  double* hist_h;
  int32_t* hist_cyc;                      // cycling index of the row
  uint32_t* hist_mask;                    // bit j: coordinate (cyc + j) mod n is split
  double* hist_mid;                       // [row][kMaxSplit] split points
  int64_t hist_cap;
  // per-sweep children
  double* ch_flo;
  uint8_t* ch_flag;                       // 0 not formed, 1 fails the first-order test, 2 candidate,
                                          // 3 discarded by the FP32 filter
  double* ch_wmax;
  // select partials
  double* part_flo;
  int64_t* part_idx;
  double* part_wmax;
  int64_t* part_cnt;
  // trace
  double* tr_gub;
  int64_t* tr_nsurv;
  int64_t* tr_nlive;
  int64_t* tr_sel;
  int64_t trace_cap;
  // K boxes per sweep (K > 1: the selected boxes are listed in sel_tab by rank,
  // box p of sweep t has row 1 + t K + p, its children are records p nch + c)
  int32_t select_k, pad_k;
  SelRec* sel_tab;                        // [select_k]
  // the schedule of the paper's experiments: pieces = 4 cuts each split
  // coordinate into four (nch = 4^m children), nsamp > 0 samples every child at
  // nsamp points of its diagonal (cs[s]: the double nearest (s + 1) / (nsamp + 1))
  int32_t pieces, nsamp;
  double cs[kMaxSamples];
  double* hist_cut;                       // [row][kMaxSplit][3] cut points of 4-piece rows
  double* tab;                            // the sweep's piece tables (kTabDoubles)
  int32_t* tabi;                          // their index part (kTabInts)
  KselBuf* ksel;                          // K > 1: the selection's buffer for long lists
  int32_t* ins_cnt;                       // four pieces: survivors and formed records per insertion
                                          // workgroup ([2][kMaxSelBlocks])
  // term cache (one box per sweep, incremental bounds, large n): for every row,
  // the terms its children share (F's enclosure and the midpoint bound of each
  // term no split coordinate of the row touches), [row][3][n]; a selected box
  // takes those of its parent row that its own cut leaves unchanged
  double* tcache;                         // null: no cache
  double* ibsum;                          // with the cache, the sweep on several workgroups: the 64
                                          // slot sums of F's endpoints and of the midpoint bound
                                          // [3][64], the separable families' tables of the split
                                          // halves, the widest unsplit side per block of coordinates
  int32_t* hist_par;                      // [row] the row the box was cut from (-1: none)
  // the generic family
  const TapeDev* tape;                    // null for the fixed families
  const double* tcols;                    // [C][n] coefficient columns
  I* tws;                                 // [children][nprod][n] right products of the product reductions
};

struct State {
  uint64_t gub_key;                       // ordered key of GUB
  int64_t n_keys, next_seq, sweeps, evaluated, ub_evaluated, n_live;
  double glb, wmax;
  int32_t stop;
  int32_t pending;                        // children of the last selected box await insertion
  uint32_t sel_done, bound_done;
  int32_t sel_row, sel_cyc;
  uint32_t sel_mask;
  int64_t sel_seq;
  double sel_mid[kMaxSplit];
  // FP32 filter: GUB when the sweep's bound kernel starts (the filter's cutoff,
  // so that its decisions do not depend on the order of the GUB updates), the
  // switch for the next sweep, back-off after sweeps where it pruned too little
  double gub_start;
  int32_t use32, p32_fails;
  int64_t p32_resume, fp32_pruned, fp32_sweeps;
  int32_t sel_count, pad_sel;             // K > 1: boxes selected by the last selection
  int32_t sel_ref, sel_r;                 // K = 1: the selected key's parent row and child index
  // K > 1 on long lists, the radix selection between its launches: the bits fixed
  // so far (ks_prefix, above bit ks_shift), how many boxes are still to be taken
  // at the bound, whether the bound is settled (ks_done) and whether every live
  // key up to it is taken (ks_whole; else the bound is one key value with ties)
  uint64_t ks_prefix;
  int32_t ks_shift, ks_need, ks_done, ks_whole;
};

// K > 1 on long lists: the current digit's histogram, the ticket that finds the
// last workgroup of a histogram launch, and the candidates gathered below the bound
struct KselBuf {
  uint32_t hist[256];
  uint32_t ticket, ncand;
  double cf[kMaxSelectK];
  int32_t ci[kMaxSelectK];
};

// ordered key of a lower bound for the K > 1 selection, the two zeros made one
// (-0 + 0 is +0 when rounding up), so that equal bounds tie whatever their sign
__device__ __forceinline__ uint64_t skey(double x) { return okey(x + 0.0); }

// bisection point: 0.5 lo + 0.5 hi rounded up, kept inside [lo, hi]
__device__ __forceinline__ double midpoint(I x) {
  double m = mul_neg(0.5, x.n) + 0.5 * x.h;
  m = dmax(m, neg(x.n));
  return dmin(m, x.h);
}

// read access to the rows of boxes -------------------------------------------

// a box given as real endpoints lo[i], hi[i]
struct PlainRow {
  const double* lo;
  const double* hi;
  __device__ __forceinline__ I get(int i) const { return I{neg(lo[i]), hi[i]}; }
};

// (a + b) mod n for a, b in [0, n): one compare instead of an integer division.
__device__ __forceinline__ int add_mod(int a, int b, int n) {
  const int s = a + b;
  return s >= n ? s - n : s;
}

// child r of a stored row: coordinate (cyc + j) mod n takes the upper half
// [mid_j, hi] when bit j of r is set and the lower half [lo, mid_j] otherwise
struct ChildRow {
  const double* pn;
  const double* ph;
  const double* mid;
  int n, m, cyc;
  uint32_t mask, r;
  __device__ __forceinline__ I get(int i) const {
    I x{G(pn)[i], G(ph)[i]};
    int j = i - cyc;
    if (j < 0) j += n;
    if (j < m && ((mask >> j) & 1u)) {
      const double md = G(mid)[j];
      if ((r >> j) & 1u) x.n = neg(md); else x.h = md;
    }
    return x;
  }
};

// Write row `src` (a child of a stored row) to dn/dh.  The loads of U strides are
// issued before their stores: the stores may alias the loads as far as the
// compiler knows, so a load after a store would wait for it.  Returns the
// widest side (rounded up) this thread wrote among the coordinates outside the
// window of m coordinates from wstart (those no cut of the new row touches).
template <int NT, int U = (NT >= 1024 ? 2 : 8), class Row>
__device__ __forceinline__ double build_row(const Row& src, double* dn, double* dh, int n, int wstart, int m) {
  double wb = 0.0;
  auto outside = [&](int i) {
    int j = i - wstart;
    if (j < 0) j += n;
    return j >= m;
  };
  int i = threadIdx.x;
  for (; i + (U - 1) * NT < n; i += U * NT) {
    I x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = src.get(i + u * NT);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      G(dn)[i + u * NT] = x[u].n;
      G(dh)[i + u * NT] = x[u].h;
      if (outside(i + u * NT)) wb = dmax(wb, x[u].n + x[u].h);
    }
  }
  for (; i < n; i += NT) {
    const I x = src.get(i);
    G(dn)[i] = x.n;
    G(dh)[i] = x.h;
    if (outside(i)) wb = dmax(wb, x.n + x.h);
  }
  return wb;
}

// child r of a stored row cut into four pieces per split coordinate: coordinate
// (cyc + j) mod n takes piece (r >> 2j) & 3 of [lo, c_1, c_2, c_3, hi]
struct ChildRow4 {
  const double* pn;
  const double* ph;
  const double* cut;   // [kMaxSplit][3]
  int n, m, cyc;
  uint32_t mask, r;
  __device__ __forceinline__ I get(int i) const {
    I x{G(pn)[i], G(ph)[i]};
    int j = i - cyc;
    if (j < 0) j += n;
    if (j < m && ((mask >> j) & 1u)) {
      const int d = (int)((r >> (2 * j)) & 3u);
      if (d > 0) x.n = neg(G(cut)[3 * j + d - 1]);
      if (d < 3) x.h = G(cut)[3 * j + d];
    }
    return x;
  }
};

// the cut points of [lo, hi] = (-x.n, x.h) into four pieces: lo + w I, w =
// (hi - lo) / 4, I = 1, 2, 3, every operation rounded up (the kernels run in
// round-up mode), each kept inside [previous cut, hi]; true when every piece has
// positive width
__device__ __forceinline__ bool cuts4(I x, double* c) {
  const double w = (x.h + x.n) * 0.25;
  double prev = neg(x.n);
  bool ok = true;
  for (int q = 0; q < 3; ++q) {
    double v = w * (double)(q + 1) - x.n;
    v = dmin(dmax(v, prev), x.h);
    ok = ok && prev < v;
    c[q] = v;
    prev = v;
  }
  return ok && prev < x.h;
}

// coordinate of a diagonal sample of [lo, hi] = (-x.n, x.h): lo + (hi - lo) c,
// each operation rounded up, kept inside [lo, hi]
__device__ __forceinline__ double diag_coord(I x, double c) {
  const double v = (x.h + x.n) * c - x.n;
  return dmin(dmax(v, neg(x.n)), x.h);
}

// wave-level helpers ---------------------------------------------------------

__device__ __forceinline__ double wave_max(double v) {
  for (int h = 32; h >= 1; h >>= 1) v = dmax(v, __shfl_xor(v, h, kWave));
  return v;
}

// Canonical sum: lane s holds slot s (terms s, s+64, ... summed left to right);
// slots are folded with strides 32, 16, ..., 1, slot s absorbing slot s + h.
__device__ __forceinline__ I fold_slots(I acc, int lane) {
  for (int h = 32; h >= 1; h >>= 1) {
    const double on = __shfl_down(acc.n, h, kWave);
    const double oh = __shfl_down(acc.h, h, kWave);
    if (lane < h) acc = add(acc, I{on, oh});
  }
  return I{__shfl(acc.n, 0, kWave), __shfl(acc.h, 0, kWave)};
}
__device__ __forceinline__ double fold_slots_hi(double acc, int lane) {
  for (int h = 32; h >= 1; h >>= 1) {
    const double o = __shfl_down(acc, h, kWave);
    if (lane < h) acc = acc + o;
  }
  return __shfl(acc, 0, kWave);
}

// wave sum of single-precision intervals (fixed order, any lane holds the result)
__device__ __forceinline__ J fold32(J acc, int lane) {
  for (int h = 32; h >= 1; h >>= 1) {
    const float on = __shfl_down(acc.n, h, kWave);
    const float oh = __shfl_down(acc.h, h, kWave);
    if (lane < h) acc = add32(acc, J{on, oh});
  }
  return J{__shfl(acc.n, 0, kWave), __shfl(acc.h, 0, kWave)};
}

// FP32 filter, coordinate i of a box: its term of f (CHAIN: term i, zero for the
// last coordinate) and the first-order test on its gradient component
template <int FAM, class Row>
__device__ __forceinline__ void filter32_coord(const Params& P, const Row& X, int i, J& t, bool& mono,
                                               double* Gout = nullptr) {
  const int n = P.n;
  const I x = X.get(i);
  J G;
  if (FAM != FAM_CHAIN) {
    sep_box32<FAM>(P.sep32[i], to32(x), t, G);
  } else {
    const bool has_prev = i > 0, has_next = i + 1 < n;
    const J x32 = to32(x);
    const J xp = has_prev ? to32(X.get(i - 1)) : x32;
    const J xn = has_next ? to32(X.get(i + 1)) : x32;
    t = has_next ? chain_term32(P.chain32[i], x32, xn) : J{0.0f, 0.0f};
    G = chain_grad32(P.chain32[has_prev ? i - 1 : i], P.chain32[i], xp, x32, xn, has_prev, has_next);
  }
  mono |= (G.n < 0.0f && x.n != P.nl[i]) || (G.h < 0.0f && x.h != P.u[i]);
  if (Gout) { Gout[2 * i] = (double)neg32(G.n); Gout[2 * i + 1] = (double)G.h; }
}

// F, first-order test and widest side of one box, by one wavefront
template <int FAM, class Row>
__device__ __forceinline__ void bound_box(const Params& P, const Row& X, int lane, I& F, bool& mono,
                                          double& wmax, double* Gout) {
  const int n = P.n;
  I acc{0.0, 0.0};
  bool mo = false;
  double wm = 0.0;
  if (FAM != FAM_CHAIN) {
    for (int i = lane; i < n; i += kWave) {
      const I x = X.get(i);
      I t, G;
      sep_box<FAM>(P.sep[i], x, t, G);
      acc = add(acc, t);
      mo |= (G.n < 0.0 && x.n != P.nl[i]) || (G.h < 0.0 && x.h != P.u[i]);
      wm = dmax(wm, x.n + x.h);
      if (Gout) { Gout[2 * i] = neg(G.n); Gout[2 * i + 1] = G.h; }
    }
  } else {
    for (int i = lane; i < n; i += kWave) {
      const I xi = X.get(i);
      const bool has_prev = i > 0, has_next = i + 1 < n;
      const I xp = has_prev ? X.get(i - 1) : xi;
      const I xn = has_next ? X.get(i + 1) : xi;
      if (has_next) {
        I R, E;
        acc = add(acc, chain_term(P.chain[i], xi, xn, R, E));
      }
      const I G = chain_grad(P.chain[has_prev ? i - 1 : i], P.chain[i], xp, xi, xn, has_prev, has_next);
      mo |= (G.n < 0.0 && xi.n != P.nl[i]) || (G.h < 0.0 && xi.h != P.u[i]);
      wm = dmax(wm, xi.n + xi.h);
      if (Gout) { Gout[2 * i] = neg(G.n); Gout[2 * i + 1] = G.h; }
    }
  }
  F = fold_slots(acc, lane);
  mono = __any(mo);
  wmax = wave_max(wm);
}

// upper bound of f at the box midpoint, by one wavefront
template <int FAM, class Row>
__device__ __forceinline__ double point_ub(const Params& P, const Row& X, int lane) {
  const int n = P.n;
  double acc = 0.0;
  if (FAM != FAM_CHAIN) {
    for (int i = lane; i < n; i += kWave) acc = acc + sep_point_hi<FAM>(P.sep[i], midpoint(X.get(i)));
  } else {
    for (int i = lane; i + 1 < n; i += kWave) {
      I R, E;
      const I t = chain_term(P.chain[i], point(midpoint(X.get(i))), point(midpoint(X.get(i + 1))), R, E);
      acc = acc + t.h;
    }
  }
  return fold_slots_hi(acc, lane);
}

}  // namespace ibb
