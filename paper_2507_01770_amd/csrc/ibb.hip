// ibb.hip -- libibb: kernels, host driver and the C ABI declared in include/ibb.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <type_traits>
#include <string>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "ibb.h"
#include "kern.hpp"
#include "tape.hpp"

using namespace ibb;

// ===========================================================================
// kernels
// ===========================================================================

// per-coordinate coefficient records; [c pi k b] = [RD(c PI_LO k), RU(c PI_HI k)] * b
__global__ void k_setup_sep(int n, int family, const double* __restrict__ coef, CoefSep* __restrict__ out,
                            CoefSep32* __restrict__ out32) {
  round_up_mode();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CoefSep r;
  r.a = coef[i];
  r.b = coef[n + i];
  r.k = coef[2 * n + i];
  r.c = coef[3 * n + i];
  // PI_LO < pi < PI_HI, adjacent doubles; the factor 2 is exact
  const double pl = hexd(0x400921fb54442d18ull), ph = hexd(0x400921fb54442d19ull);
  const double sc = family == FAM_SEP_COS ? 2.0 : 1.0;
  const I pk{mul_neg(sc * pl, r.k), (sc * ph) * r.k};
  r.pkb = mul(pk, point(r.b));
  out[i] = r;
  if (out32) {
    CoefSep32 q;
    q.a = to32(point(r.a));
    q.b = to32(point(r.b));
    q.c = to32(point(r.c));
    q.pkb = to32(r.pkb);
    q.k = (float)r.k;        // exact: the filter is enabled only for k <= 2^24
    q.hk = 0.5f * q.k;
    q.pad0 = q.pad1 = 0.0f;
    out32[i] = q;
  }
}

__global__ void k_setup_chain(int n, const double* __restrict__ coef, CoefChain* __restrict__ out,
                              CoefChain32* __restrict__ out32) {
  round_up_mode();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  CoefChain r;
  r.al = i < n - 1 ? coef[i] : 0.0;
  r.be = i < n - 1 ? coef[(n - 1) + i] : 0.0;
  out[i] = r;
  if (out32) out32[i] = CoefChain32{to32(point(r.al)), to32(point(r.be))};
}

// ---------------------------------------------------------------------------
// The generic family (an expression tape): every child bounded in full by one
// thread (the terms of f are not a sum of per-coordinate terms in general, so
// there are no shared terms to reuse), the records written for the next
// selection, GUB lowered by the smallest sample upper bound of the workgroup.

// the root box (the first key) and GUB from its midpoint (no sample with the
// diagonal samples of the paper's schedule)
__global__ __launch_bounds__(kWave) void k_tape_root(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  const Params P = *PP;
  if (threadIdx.x != 0) return;
  const ChildRow X{P.hist_n, P.hist_h, P.hist_mid, P.n, P.m, 0, 0u, 0u};
  bool mo = false;
  const I F = tape_box<ChildRow, false>(*P.tape, P.tcols, P.n, X, P.nl, P.u, P.tws, mo, nullptr);
  const PointRow<ChildRow> M{X, -1.0};
  bool unused = false;
  const double u = tape_box<PointRow<ChildRow>, false>(*P.tape, P.tcols, P.n, M, P.nl, P.u, P.tws, unused, nullptr).h;
  double wm = 0.0;
  for (int i = 0; i < P.n; ++i) { const I x = X.get(i); wm = dmax(wm, x.n + x.h); }
  S->gub_key = okey(P.nsamp > 0 ? __builtin_inf() : hi_or_inf(u));
  P.key_flo[0] = lo_or_ninf(neg(F.n));
  P.key_seq[0] = 0;
  P.key_ref[0] = 0;
  P.key_r[0] = -1;
  P.key_wmax[0] = wm;
  P.hist_cyc[0] = 0;
  P.hist_mask[0] = 0u;
  S->n_keys = 1;
  S->next_seq = 1;
  S->sweeps = 0;
  S->evaluated = 1;
  S->ub_evaluated = 1;
  S->n_live = 1;
  S->stop = RUNNING;
  S->pending = 0;
  S->sel_done = 0u;
  S->bound_done = 0u;
}

// F, the first-order test and the record of every child of the selected box,
// one thread each (PIECES = 2: bisection; PIECES = 4: the paper's four pieces);
// the children's sample bounds are k_tape_samples' (the midpoint, or P.nsamp
// diagonal points)
template <int PIECES>
__global__ __launch_bounds__(256) void k_tape_children(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  const Params& P = *PP;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = P.n, m = P.m;
  const int64_t row = S->sel_row;
  const int cyc = S->sel_cyc;
  const uint32_t mask = S->sel_mask;
  const bool in = g < P.nch;
  bool formed = in;
  if (PIECES == 2) {
    formed = in && ((uint32_t)g & ~mask) == 0u;
  } else {
    for (int j = 0; j < m; ++j)
      if (((g >> (2 * j)) & 3) && !((mask >> j) & 1u)) formed = false;
  }
  if (formed) {
    using Row = typename std::conditional<PIECES == 4, ChildRow4, ChildRow>::type;
    const Row X{P.hist_n + row * n, P.hist_h + row * n,
                PIECES == 4 ? P.hist_cut + row * (3 * kMaxSplit) : P.hist_mid + row * kMaxSplit, n, m, cyc, mask,
                (uint32_t)g};
    I* ws = P.tws ? P.tws + (int64_t)g * P.tape->nprod * n : nullptr;
    bool mo = false;
    // GUB at this sweep's selection, never below the sweep's final GUB: a child
    // whose lower bound exceeds it is not inserted, so its first-order test is
    // not needed (its record still counts as formed)
    const double gub0 = S->gub_start;
    const I F = tape_box<Row, true>(*P.tape, P.tcols, n, X, P.nl, P.u, ws, mo, nullptr, gub0);
    double wm = 0.0;
    for (int i = 0; i < n; ++i) { const I x = X.get(i); wm = dmax(wm, x.n + x.h); }
    P.ch_flo[g] = lo_or_ninf(neg(F.n));
    P.ch_wmax[g] = wm;
    P.ch_flag[g] = mo ? 1 : 2;
  } else if (in) {
    P.ch_flag[g] = 0;
  }
}

// The sample upper bounds of the same children (their diagonal points, or the
// midpoint), one thread per child, and the workgroup's smallest into GUB.  A
// kernel of its own: point values need no tangents or adjoints, so it holds
// about half the registers of the pass above and runs twice the wavefronts.
// A child whose lower bound (written by the pass above) exceeds GUB is skipped:
// every sample bound of a point of its box is at least that lower bound, so it
// could not lower GUB.
template <int PIECES>
__global__ __launch_bounds__(256) void k_tape_samples(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  const Params& P = *PP;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = P.n, m = P.m;
  const int64_t row = S->sel_row;
  const int cyc = S->sel_cyc;
  const uint32_t mask = S->sel_mask;
  const bool in = g < P.nch;
  bool formed = in;
  if (PIECES == 2) {
    formed = in && ((uint32_t)g & ~mask) == 0u;
  } else {
    for (int j = 0; j < m; ++j)
      if (((g >> (2 * j)) & 3) && !((mask >> j) & 1u)) formed = false;
  }
  double ub = __builtin_inf();
  // GUB at this sweep's selection (not the running one, which other workgroups
  // lower meanwhile: the count of bounds evaluated stays the same on every run)
  if (formed && P.ch_flo[g] > S->gub_start) formed = false;   // counted as not evaluated
  if (formed) {
    using Row = typename std::conditional<PIECES == 4, ChildRow4, ChildRow>::type;
    const Row X{P.hist_n + row * n, P.hist_h + row * n,
                PIECES == 4 ? P.hist_cut + row * (3 * kMaxSplit) : P.hist_mid + row * kMaxSplit, n, m, cyc, mask,
                (uint32_t)g};
    bool unused = false;
    if (P.nsamp > 0) {
      for (int s = 0; s < P.nsamp; ++s) {
        const PointRow<Row> D{X, P.cs[s]};
        ub = dmin(ub, hi_or_inf(tape_box<PointRow<Row>, false>(*P.tape, P.tcols, n, D, P.nl, P.u, nullptr, unused,
                                                               nullptr).h));
      }
    } else {
      const PointRow<Row> M{X, -1.0};
      ub = hi_or_inf(tape_box<PointRow<Row>, false>(*P.tape, P.tcols, n, M, P.nl, P.u, nullptr, unused, nullptr).h);
    }
  }
  // the workgroup's smallest sample bound into GUB (only when it is lower)
  __shared__ double s_u[256 / kWave];
  __shared__ int s_n[256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  double um = ub;
  int cnt = formed ? 1 : 0;
  for (int h = 32; h >= 1; h >>= 1) {
    um = dmin(um, __shfl_xor(um, h, kWave));
    cnt += __shfl_xor(cnt, h, kWave);
  }
  if (lane == 0) { s_u[wid] = um; s_n[wid] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mn = s_u[0];
    int tot = s_n[0];
    for (int k = 1; k < 256 / kWave; ++k) { mn = dmin(mn, s_u[k]); tot += s_n[k]; }
    if (tot > 0) {
      const unsigned long long key = okey(mn);
      if (key < __hip_atomic_load(&S->gub_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)&S->gub_key, key);
      atomicAdd((unsigned long long*)&S->ub_evaluated, (unsigned long long)tot);
    }
  }
}

// bound nb boxes given by their real endpoints, one thread each (ibb_eval_boxes)
__global__ __launch_bounds__(256) void k_eval_tape(const Params* __restrict__ PP, int64_t nb,
                                                   const double* __restrict__ lo, const double* __restrict__ hi,
                                                   double* __restrict__ F, double* __restrict__ ub,
                                                   uint8_t* __restrict__ mono, double* __restrict__ G, I* ws) {
  round_up_mode();
  const Params P = *PP;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  const int n = P.n;
  const PlainRow X{lo + b * n, hi + b * n};
  bool mo = false;
  I* w = ws ? ws + b * P.tape->nprod * n : nullptr;
  const I f = tape_box<PlainRow, true>(*P.tape, P.tcols, n, X, P.nl, P.u, w, mo, G ? G + b * 2 * n : nullptr);
  bool unused = false;
  const PointRow<PlainRow> M{X, -1.0};
  const double u = tape_box<PointRow<PlainRow>, false>(*P.tape, P.tcols, n, M, P.nl, P.u, w, unused, nullptr).h;
  F[2 * b] = neg(f.n);
  F[2 * b + 1] = f.h;
  ub[b] = u;
  mono[b] = mo ? 1 : 0;
}

// a[i] = -a[i] (exact), for the lower bounds held negated
__global__ void k_negate(int n, double* __restrict__ a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = neg(a[i]);
}

// bound nb boxes given by their real endpoints (one wavefront per box)
template <int FAM>
__global__ __launch_bounds__(kWave* kBoundWaves) void k_eval_boxes(const Params* __restrict__ PP, int64_t nb,
                                                                  const double* __restrict__ lo,
                                                                  const double* __restrict__ hi,
                                                                  double* __restrict__ F, double* __restrict__ ub,
                                                                  uint8_t* __restrict__ mono,
                                                                  double* __restrict__ G) {
  round_up_mode();
  const Params P = *PP;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t b = (int64_t)blockIdx.x * kBoundWaves + (threadIdx.x >> 6);
  if (b >= nb) return;
  const PlainRow X{lo + b * P.n, hi + b * P.n};
  I Fb;
  bool mo;
  double wm;
  bound_box<FAM>(P, X, lane, Fb, mo, wm, G ? G + b * 2 * P.n : nullptr);
  const double u = point_ub<FAM>(P, X, lane);
  if (lane == 0) {
    F[2 * b] = neg(Fb.n);
    F[2 * b + 1] = Fb.h;
    ub[b] = u;
    mono[b] = mo ? 1 : 0;
  }
}

// the FP32 filter's bounds of nb boxes: F and the first-order test in single
// precision over the FP32-enclosing box, the midpoint upper bound in FP64
template <int FAM>
__global__ __launch_bounds__(kWave* kBoundWaves) void k_eval_boxes32(const Params* __restrict__ PP, int64_t nb,
                                                                    const double* __restrict__ lo,
                                                                    const double* __restrict__ hi,
                                                                    double* __restrict__ F, double* __restrict__ ub,
                                                                    uint8_t* __restrict__ mono,
                                                                    double* __restrict__ G) {
  round_up_mode();
  const Params P = *PP;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t b = (int64_t)blockIdx.x * kBoundWaves + (threadIdx.x >> 6);
  if (b >= nb) return;
  const PlainRow X{lo + b * P.n, hi + b * P.n};
  J a32{0.0f, 0.0f};
  bool m32 = false;
  for (int i = lane; i < P.n; i += kWave) {
    J t;
    filter32_coord<FAM>(P, X, i, t, m32, G ? G + b * 2 * P.n : nullptr);
    a32 = add32(a32, t);
  }
  const J F32 = fold32(a32, lane);
  const bool mo = __any(m32);
  const double u = point_ub<FAM>(P, X, lane);
  if (lane == 0) {
    F[2 * b] = (double)neg32(F32.n);
    F[2 * b + 1] = (double)F32.h;
    ub[b] = u;
    mono[b] = mo ? 1 : 0;
  }
}

// root box: key 0, GUB from its midpoint
template <int FAM>
__global__ __launch_bounds__(kWave) void k_root(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  const Params P = *PP;
  const int lane = threadIdx.x;
  const ChildRow X{P.hist_n, P.hist_h, P.hist_mid, P.n, P.m, 0, 0u, 0u};
  I F;
  bool mo;
  double wm;
  bound_box<FAM>(P, X, lane, F, mo, wm, nullptr);
  const double u = point_ub<FAM>(P, X, lane);
  if (lane == 0) {
    // with diagonal samples (the paper's schedule) nothing is sampled before the
    // first sweep, which samples the subregions of the whole domain: GUB = +inf
    S->gub_key = okey(P.nsamp > 0 ? __builtin_inf() : hi_or_inf(u));
    P.key_flo[0] = lo_or_ninf(neg(F.n));
    P.key_seq[0] = 0;
    P.key_ref[0] = 0;
    P.key_r[0] = -1;
    P.key_wmax[0] = wm;
    P.hist_cyc[0] = 0;
    P.hist_mask[0] = 0u;
    S->n_keys = 1;
    S->next_seq = 1;
    S->sweeps = 0;
    S->evaluated = 1;
    S->ub_evaluated = 1;
    S->n_live = 1;
    S->stop = RUNNING;
    S->pending = 0;
    S->sel_done = 0u;
    S->bound_done = 0u;
  }
}

// candidate order of the selection: smaller lower bound, then smaller insertion
// number.  Keys are appended in insertion order and every compaction keeps their
// order, so a key's index in the list orders keys as its insertion number does:
// the scan compares indices and never loads the numbers.
struct Cand {
  double f;
  int64_t idx;
};
__device__ __forceinline__ bool better(const Cand& a, const Cand& b) {  // a before b
  return a.f < b.f || (a.f == b.f && a.idx < b.idx);
}
// running reduction of the selection scan: best key, widest box, live count
struct SelAcc {
  Cand best;
  double wm;
  int64_t cnt;
};
__device__ __forceinline__ SelAcc sel_merge(SelAcc a, const SelAcc& b) {
  if (better(b.best, a.best)) a.best = b.best;
  a.wm = dmax(a.wm, b.wm);
  a.cnt += b.cnt;
  return a;
}
__device__ __forceinline__ SelAcc sel_empty() { return SelAcc{Cand{__builtin_inf(), INT64_MAX}, 0.0, 0}; }

// reduce over a workgroup of NT threads; the result is returned to every thread
template <int NT>
__device__ __forceinline__ SelAcc sel_block_reduce(SelAcc v) {
  for (int h = 32; h >= 1; h >>= 1) {
    SelAcc o;
    o.best.f = __shfl_xor(v.best.f, h, kWave);
    o.best.idx = (int64_t)__shfl_xor((long long)v.best.idx, h, kWave);
    o.wm = __shfl_xor(v.wm, h, kWave);
    o.cnt = (int64_t)__shfl_xor((long long)v.cnt, h, kWave);
    v = sel_merge(v, o);
  }
  __shared__ SelAcc part[NT / kWave];
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  SelAcc r = part[0];
  for (int k = 1; k < NT / kWave; ++k) r = sel_merge(r, part[k]);
  return r;
}

// Insert the survivors of the previous sweep's children (lower bound <= the
// final GUB of that sweep, first-order test passed), in child order, and fold
// them into the running selection.  One workgroup of NT threads: each wavefront
// takes a contiguous range of the records (the ranges in wavefront order keep
// child order) and walks it in rounds of 64 consecutive records, one per lane,
// so every load of a round is coalesced; a ballot places a round's survivors.
template <int NT>
__device__ __forceinline__ void insert_children(const Params& P, State* S, double gub, SelAcc& acc) {
  constexpr int NW = NT / kWave;
  __shared__ int w_ins[NW], w_form[NW], w_n32[NW];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // K > 1: the records of the K parents, parent-major (record p nch + c)
  const bool multi = P.select_k > 1;
  const int nrec = multi ? S->sel_count * P.nch : P.nch;
  const int per_w = (nrec + NW - 1) / NW;
  const int r0 = min(nrec, wid * per_w), r1 = min(nrec, r0 + per_w);
  int wsurv = 0, nformed = 0, n32 = 0;
  for (int b = r0; b < r1; b += kWave) {
    const int k = b + lane;
    bool sv = false;
    if (k < r1) {
      const uint8_t fl = P.ch_flag[k];
      nformed += fl != 0;
      n32 += fl == 3;
      sv = fl == 2 && !(P.ch_flo[k] > gub);
    }
    wsurv += __popcll(__ballot(sv));
  }
  for (int h = 32; h >= 1; h >>= 1) {
    nformed += __shfl_xor(nformed, h, kWave);
    n32 += __shfl_xor(n32, h, kWave);
  }
  __shared__ int w_tot[3];
  __syncthreads();   // the LDS arrays may still be read by a previous call
  if (lane == 0) { w_ins[wid] = wsurv; w_form[wid] = nformed; w_n32[wid] = n32; }
  __syncthreads();
  if (wid == 0) {    // exclusive prefix of the wavefront totals, and the sums
    const int v = lane < NW ? w_ins[lane] : 0;
    int f = lane < NW ? w_form[lane] : 0, q = lane < NW ? w_n32[lane] : 0, x = v;
    for (int h = 1; h < kWave; h <<= 1) {
      const int o = __shfl_up(x, h, kWave);
      if (lane >= h) x += o;
    }
    for (int h = 32; h >= 1; h >>= 1) {
      f += __shfl_xor(f, h, kWave);
      q += __shfl_xor(q, h, kWave);
    }
    if (lane < NW) w_ins[lane] = x - v;
    if (lane == kWave - 1) w_tot[0] = x;
    if (lane == 0) { w_tot[1] = f; w_tot[2] = q; }
  }
  __syncthreads();
  const int before = w_ins[wid], total = w_tot[0], formed = w_tot[1], s_n32 = w_tot[2];
  const int64_t base = S->n_keys;
  const int64_t seq0 = S->next_seq;
  const int row = S->sel_row;
  int64_t o = base + before;   // the wavefront's next key
  SelAcc a = sel_empty();
  for (int b = r0; b < r1; b += kWave) {
    const int k = b + lane;
    double f = 0.0;
    bool sv = false;
    if (k < r1) {
      f = P.ch_flo[k];
      sv = P.ch_flag[k] == 2 && !(f > gub);
    }
    const unsigned long long bal = __ballot(sv);
    if (sv) {
      const int64_t ok = o + __popcll(bal & below);
      P.key_flo[ok] = f;
      P.key_seq[ok] = seq0 + (ok - base);
      P.key_ref[ok] = multi ? P.sel_tab[k >> P.m].row : row;
      P.key_r[ok] = multi ? (k & (P.nch - 1)) : k;
      const double w = P.ch_wmax[k];
      P.key_wmax[ok] = w;
      a.cnt++;
      a.wm = dmax(a.wm, w);
      const Cand cd{f, ok};
      if (better(cd, a.best)) a.best = cd;
    }
    o += __popcll(bal);
  }
  a = sel_block_reduce<NT>(a);
  acc = sel_merge(acc, a);
  if (threadIdx.x == 0) {
    const int64_t t = S->sweeps;
    if (t < P.trace_cap) {
      P.tr_gub[t] = gub;
      P.tr_nsurv[t] = total;
      P.tr_sel[t] = S->sel_seq;
    }
    S->n_keys = base + total;
    S->next_seq = seq0 + total;
    S->evaluated += formed;
    S->sweeps = t + 1;
    S->pending = 0;
    if (P.prec32) {
      // FP32 filter switch, from counts only (so the same for every run): keep it
      // while it discards at least half of the children; after a sweep where it
      // discarded less, turn it off for 2, 4, ..., 64 sweeps; turn it on when at
      // least half of an FP64 sweep's children were discarded
      if (S->use32) {
        S->fp32_sweeps += 1;
        S->fp32_pruned += s_n32;
        if (2 * s_n32 < formed) {
          S->use32 = 0;
          S->p32_fails = min(S->p32_fails + 1, 6);
          S->p32_resume = t + 1 + (1 << S->p32_fails);
        }
      } else if (t + 1 >= S->p32_resume && formed > 0 && 2 * (formed - total) >= formed) {
        S->use32 = 1;
      }
    }
  }
  __syncthreads();
}

// The same insertion on many workgroups, for the 4^m records of the paper's
// schedule (one box per sweep, FP64): workgroup b takes the contiguous records
// [b R, (b + 1) R) and, as insert_children does within its workgroup, each
// wavefront a contiguous part of those, walked 64 consecutive records at a time.
// k_ins_count counts each workgroup's survivors; k_ins_scatter places them after
// those of the workgroups before it (so keys stay in child order); k_ins_finish
// (one workgroup) updates the counters, so that the selection's scan that
// follows finds the new keys with everything else and inserts nothing itself.
// All three do nothing unless children are pending.
__device__ __forceinline__ void ins_range(int nrec, int& r0, int& r1) {
  const int per_b = (nrec + (int)gridDim.x - 1) / (int)gridDim.x;
  const int b0 = min(nrec, (int)blockIdx.x * per_b), b1 = min(nrec, b0 + per_b);
  constexpr int NW = kSelThreads / kWave;
  const int wid = threadIdx.x >> 6;
  const int per_w = (b1 - b0 + NW - 1) / NW;
  r0 = min(b1, b0 + wid * per_w);
  r1 = min(b1, r0 + per_w);
}
__global__ __launch_bounds__(kSelThreads) void k_ins_count(const Params* __restrict__ PP, State* __restrict__ S) {
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  const double gub = okey_inv(S->gub_key);
  int r0, r1;
  ins_range(P.nch, r0, r1);
  const int lane = threadIdx.x & (kWave - 1);
  int surv = 0, formed = 0;
  for (int b = r0; b < r1; b += kWave) {
    const int k = b + lane;
    bool sv = false;
    if (k < r1) {
      const uint8_t fl = P.ch_flag[k];
      formed += fl != 0;
      sv = fl == 2 && !(P.ch_flo[k] > gub);
    }
    surv += __popcll(__ballot(sv));
  }
  for (int h = 32; h >= 1; h >>= 1) formed += __shfl_xor(formed, h, kWave);
  __shared__ int s_s[kSelThreads / kWave], s_f[kSelThreads / kWave];
  if (lane == 0) { s_s[threadIdx.x >> 6] = surv; s_f[threadIdx.x >> 6] = formed; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int ts = 0, tf = 0;
    for (int w = 0; w < kSelThreads / kWave; ++w) { ts += s_s[w]; tf += s_f[w]; }
    P.ins_cnt[blockIdx.x] = ts;
    P.ins_cnt[kMaxSelBlocks + blockIdx.x] = tf;
  }
}
__global__ __launch_bounds__(kSelThreads) void k_ins_scatter(const Params* __restrict__ PP, State* __restrict__ S) {
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  const double gub = okey_inv(S->gub_key);
  const int64_t base = S->n_keys, seq0 = S->next_seq;   // k_ins_finish changes them afterwards
  const int row = S->sel_row;
  constexpr int NW = kSelThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // survivors of the workgroups before this one, and of this one's wavefronts before this one
  __shared__ int s_before, s_w[NW];
  if (wid == 0) {
    int x = 0;
    for (int q = lane; q < (int)blockIdx.x; q += kWave) x += P.ins_cnt[q];
    for (int h = 32; h >= 1; h >>= 1) x += __shfl_xor(x, h, kWave);
    if (lane == 0) s_before = x;
  }
  int r0, r1;
  ins_range(P.nch, r0, r1);
  int wsurv = 0;
  for (int b = r0; b < r1; b += kWave) {
    const int k = b + lane;
    const bool sv = k < r1 && P.ch_flag[k] == 2 && !(P.ch_flo[k] > gub);
    wsurv += __popcll(__ballot(sv));
  }
  if (lane == 0) s_w[wid] = wsurv;
  __syncthreads();
  int64_t o = base + s_before;
  for (int w = 0; w < wid; ++w) o += s_w[w];
  for (int b = r0; b < r1; b += kWave) {
    const int k = b + lane;
    double f = 0.0;
    bool sv = false;
    if (k < r1) {
      f = P.ch_flo[k];
      sv = P.ch_flag[k] == 2 && !(f > gub);
    }
    const unsigned long long bal = __ballot(sv);
    if (sv) {
      const int64_t ok = o + __popcll(bal & below);
      P.key_flo[ok] = f;
      P.key_seq[ok] = seq0 + (ok - base);
      P.key_ref[ok] = row;
      P.key_r[ok] = k;
      P.key_wmax[ok] = P.ch_wmax[k];
    }
    o += __popcll(bal);
  }
}
// the counters after the insertion (nb: the workgroups of the two kernels above)
__global__ __launch_bounds__(kWave) void k_ins_finish(const Params* __restrict__ PP, State* __restrict__ S, int nb) {
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  const int lane = threadIdx.x;
  int ts = 0, tf = 0;
  for (int q = lane; q < nb; q += kWave) {
    ts += P.ins_cnt[q];
    tf += P.ins_cnt[kMaxSelBlocks + q];
  }
  for (int h = 32; h >= 1; h >>= 1) {
    ts += __shfl_xor(ts, h, kWave);
    tf += __shfl_xor(tf, h, kWave);
  }
  if (lane == 0) {
    const int64_t t = S->sweeps;
    if (t < P.trace_cap) {
      P.tr_gub[t] = okey_inv(S->gub_key);
      P.tr_nsurv[t] = ts;
      P.tr_sel[t] = S->sel_seq;
    }
    S->n_keys += ts;
    S->next_seq += ts;
    S->evaluated += tf;
    S->sweeps = t + 1;
    S->pending = 0;
  }
}

// One workgroup: stop test on [GLB, GUB]; if running, remove the best key from the
// list and build its row (child r of row ref) and the split points of that row.
// *wb (if given) receives this thread's widest written side outside the new
// row's window (see build_row).
template <int NT, int PIECES = 2>
__device__ __forceinline__ bool select_finish(const Params& P, State* S, const SelAcc& tot, double gub,
                                              double* wb = nullptr, bool build = true) {
  __shared__ int32_t go;
  if (threadIdx.x == 0) {
    const Cand b = tot.best;
    const int64_t t = S->sweeps;
    if (t > 0 && t - 1 < P.trace_cap) P.tr_nlive[t - 1] = tot.cnt;
    S->n_live = tot.cnt;
    S->glb = b.f;
    S->wmax = tot.wm;
    int32_t stop = RUNNING;
    if (tot.cnt == 0) stop = STOP_EMPTY;
    else if (b.idx < 0 || b.idx >= S->n_keys) stop = STOP_INTERNAL;
    else if (gub - b.f <= P.tol_f && (P.tol_x <= 0.0 || tot.wm < P.tol_x)) stop = STOP_CONVERGED;
    else if (t >= P.max_sweeps) stop = STOP_SWEEPS;
    else if (P.max_live > 0 && tot.cnt > P.max_live) stop = STOP_LIVE;
    else if (t + 1 >= P.hist_cap || S->n_keys + P.nch > P.key_cap) stop = STOP_CAPACITY;
    if (stop) S->stop = stop;
    go = stop == RUNNING;
    if (go) {
      P.key_flo[b.idx] = __builtin_inf();     // removed from the list
      S->sel_seq = P.key_seq[b.idx];
      S->gub_start = gub;
      S->pending = 1;                         // the bound kernel will produce children
    }
  }
  __syncthreads();
  if (!go) return false;
  const int64_t row = S->sweeps + 1;
  const int32_t ref = P.key_ref[tot.best.idx];
  const int32_t r = P.key_r[tot.best.idx];
  const int n = P.n;
  const int pcyc = P.hist_cyc[ref];
  using Row = typename std::conditional<PIECES == 4, ChildRow4, ChildRow>::type;
  const Row src{P.hist_n + (int64_t)ref * n, P.hist_h + (int64_t)ref * n,
                PIECES == 4 ? P.hist_cut + (int64_t)ref * (3 * kMaxSplit) : P.hist_mid + (int64_t)ref * kMaxSplit,
                n, P.m, pcyc, r >= 0 ? P.hist_mask[ref] : 0u, r >= 0 ? (uint32_t)r : 0u};
  const int cyc = r >= 0 ? add_mod(pcyc, P.m, n) : pcyc;   // m <= n
  if (build) {   // else k_ib_rowterms builds the row on several workgroups
    const double w = build_row<NT>(src, P.hist_n + row * n, P.hist_h + row * n, n, cyc, P.m);
    if (wb) *wb = w;
  }
  if (threadIdx.x < (unsigned)kWave) {
    const int j = threadIdx.x;
    bool ok = false;
    if (j < P.m) {
      const int d = add_mod(cyc, j, n);
      const I x = src.get(d);                 // same values as the row just written
      if (PIECES == 4) {                      // the four pieces of Eqs. (10)-(11)
        double c[3];
        ok = cuts4(x, c);
        for (int q = 0; q < 3; ++q) P.hist_cut[row * (3 * kMaxSplit) + 3 * j + q] = c[q];
      } else {
        const double md = midpoint(x);
        ok = neg(x.n) < md && md < x.h;
        P.hist_mid[row * kMaxSplit + j] = md;
        S->sel_mid[j] = md;
      }
    }
    const unsigned long long bal = __ballot(ok);
    if (j == 0) {
      const uint32_t mask = (uint32_t)bal & ((P.m >= 32) ? 0xffffffffu : ((1u << P.m) - 1u));
      P.hist_mask[row] = mask;
      P.hist_cyc[row] = cyc;
      if (P.hist_par) P.hist_par[row] = r >= 0 ? ref : -1;
      S->sel_ref = ref;
      S->sel_r = r;
      S->sel_mask = mask;
      S->sel_cyc = cyc;
      S->sel_row = (int32_t)row;
    }
  }
  return true;
}

// scan of keys [lo, hi) with lower bound <= GUB into a running selection (four
// keys per step, loaded together; the result does not depend on the order)
__device__ __forceinline__ void scan_key(const Params& P, double gub, bool need_w, int64_t i, double f, SelAcc& a) {
  if (!(f <= gub)) return;   // removed (+inf) or above GUB
  a.cnt++;
  if (need_w) a.wm = dmax(a.wm, P.key_wmax[i]);
  const Cand c{f, i};
  if (better(c, a.best)) a.best = c;
}
__device__ __forceinline__ void scan_keys(const Params& P, double gub, int64_t i0, int64_t i1, int64_t stride,
                                          SelAcc& a) {
  const bool need_w = P.tol_x > 0.0;
  int64_t i = i0;
  for (; i + 3 * stride < i1; i += 4 * stride) {
    const double f0 = P.key_flo[i], f1 = P.key_flo[i + stride], f2 = P.key_flo[i + 2 * stride],
                 f3 = P.key_flo[i + 3 * stride];
    scan_key(P, gub, need_w, i, f0, a);
    scan_key(P, gub, need_w, i + stride, f1, a);
    scan_key(P, gub, need_w, i + 2 * stride, f2, a);
    scan_key(P, gub, need_w, i + 3 * stride, f3, a);
  }
  for (; i < i1; i += stride) scan_key(P, gub, need_w, i, P.key_flo[i], a);
}

// The whole list by one workgroup, reduced over the workgroup (the result is
// returned to every thread).  Each thread visits its keys in increasing index,
// so keeping the first key with the smallest lower bound (strict <) keeps the
// smallest index among equal bounds; indices and counts are 32-bit here.  Pairs
// of keys come in 16-byte loads, eight pairs in flight per thread (one
// workgroup's scan is bound by load latency and per-key instructions).
struct OwnSel {   // one thread's part of the selection scan
  double bf, wm;
  int32_t bi, cnt;   // bi = INT32_MAX: no candidate
};
template <int NT>
__device__ __forceinline__ bool scan_own_ok(const Params& P, int64_t nk) {
  return nk < (int64_t)INT32_MAX && (reinterpret_cast<uintptr_t>(P.key_flo) & 15u) == 0u;
}
template <int NT>
__device__ __forceinline__ OwnSel scan_own(const Params& P, double gub, int64_t nk) {
  const bool need_w = P.tol_x > 0.0;
  double bf = __builtin_inf(), wm = 0.0;
  int32_t bi = INT32_MAX, cnt = 0;
  auto visit = [&](int32_t i, double f) {
    const bool live = f <= gub;
    cnt += live ? 1 : 0;
    if (live && f < bf) {
      bf = f;
      bi = i;
    }
    if (need_w && live) wm = dmax(wm, G(P.key_wmax)[i]);
  };
  const double2* f2 = reinterpret_cast<const double2*>(P.key_flo);
  const int32_t np = (int32_t)(nk >> 1);
  constexpr int U = 8;
  int32_t p = threadIdx.x;
  for (; p + (U - 1) * NT < np; p += U * NT) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = gload(f2 + p + u * NT);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      visit(2 * (p + u * NT), v[u].x);
      visit(2 * (p + u * NT) + 1, v[u].y);
    }
  }
  for (; p < np; p += NT) {
    const double2 v = gload(f2 + p);
    visit(2 * p, v.x);
    visit(2 * p + 1, v.y);
  }
  if ((nk & 1) && threadIdx.x == 0) visit((int32_t)(nk - 1), G(P.key_flo)[nk - 1]);
  return OwnSel{bf, wm, bi, cnt};
}
template <int NT>
__device__ __forceinline__ SelAcc reduce_own(const Params& P, OwnSel o) {
  const bool need_w = P.tol_x > 0.0;
  double bf = o.bf, wm = o.wm;
  int32_t bi = o.bi, cnt = o.cnt;
  for (int h = 32; h >= 1; h >>= 1) {
    const double of = __shfl_xor(bf, h, kWave);
    const int32_t oi = __shfl_xor(bi, h, kWave);
    if (of < bf || (of == bf && oi < bi)) {
      bf = of;
      bi = oi;
    }
    cnt += __shfl_xor(cnt, h, kWave);
    if (need_w) wm = dmax(wm, __shfl_xor(wm, h, kWave));
  }
  constexpr int NW = NT / kWave;
  __shared__ double s_f[NW], s_w[NW];
  __shared__ int32_t s_i[NW], s_c[NW];
  const int w = threadIdx.x >> 6;
  // (callers run at most one reduction per sweep, with barriers in between: no
  // thread still reads these when they are written again)
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_f[w] = bf;
    s_i[w] = bi;
    s_c[w] = cnt;
    s_w[w] = wm;
  }
  __syncthreads();
  SelAcc r = sel_empty();
  for (int k = 0; k < NW; ++k) {
    const Cand c{s_f[k], s_i[k] == INT32_MAX ? INT64_MAX : (int64_t)s_i[k]};
    if (better(c, r.best)) r.best = c;
    r.cnt += s_c[k];
    r.wm = dmax(r.wm, s_w[k]);
  }
  return r;
}
template <int NT>
__device__ __forceinline__ SelAcc scan_select_wg(const Params& P, double gub, int64_t nk) {
  if (!scan_own_ok<NT>(P, nk)) {
    SelAcc a = sel_empty();   // general form (lists past 2^31 keys, or 8-byte aligned keys)
    scan_keys(P, gub, threadIdx.x, nk, NT, a);
    return sel_block_reduce<NT>(a);
  }
  return reduce_own<NT>(P, scan_own<NT>(P, gub, nk));
}

// Large lists: each of `parts` workgroups scans every parts-th stretch of the keys
// and writes partial j.
__device__ __forceinline__ void select_part_body(const Params& P, State* S, int j, int parts) {
  const double gub = okey_inv(S->gub_key);
  SelAcc a = sel_empty();
  scan_keys(P, gub, (int64_t)j * kSelThreads + threadIdx.x, S->n_keys, (int64_t)parts * kSelThreads, a);
  a = sel_block_reduce<kSelThreads>(a);
  if (threadIdx.x == 0) {
    P.part_flo[j] = a.best.f;
    P.part_idx[j] = a.best.idx;
    P.part_wmax[j] = a.wm;
    P.part_cnt[j] = a.cnt;
  }
}
__global__ __launch_bounds__(kSelThreads) void k_select_part(const Params* __restrict__ PP, State* __restrict__ S) {
  if (S->stop) return;
  const Params P = *PP;
  select_part_body(P, S, blockIdx.x, gridDim.x);
}

// One workgroup per sweep: insert the previous sweep's survivors, take the
// smallest key over the list (its own scan, or the partials of k_select_part),
// test the stopping criteria and select the next box.  Kernel boundaries make
// the children written by k_bound and the partials visible: no device-scope
// fences are needed.
template <int NT, int PIECES = 2>
__device__ __forceinline__ bool select_body(const Params& P, State* S, int nparts, int host_stop,
                                            double* wb = nullptr, bool build = true) {
  const double gub = okey_inv(S->gub_key);
  // every thread reads the pending flag before the scan's barriers: thread 0 sets
  // it again in select_finish with no barrier in between, so a later read could see
  // the new value in some wavefronts and send them alone into insert_children
  const int32_t pending = S->pending;
  SelAcc a = sel_empty();
  if (nparts == 0) {
    a = scan_select_wg<NT>(P, gub, S->n_keys);
  } else {
    for (int k = threadIdx.x; k < nparts; k += NT) {
      const SelAcc o{Cand{P.part_flo[k], P.part_idx[k]}, P.part_wmax[k], P.part_cnt[k]};
      a = sel_merge(a, o);
    }
    a = sel_block_reduce<NT>(a);
  }
  if (pending) insert_children<NT>(P, S, gub, a);
  if (host_stop) {   // the host ends the run here (time limit): keep the inserted list
    if (threadIdx.x == 0) {
      const int64_t t = S->sweeps;
      if (t > 0 && t - 1 < P.trace_cap) P.tr_nlive[t - 1] = a.cnt;
      S->n_live = a.cnt;
      S->stop = STOP_HOST;
    }
    return false;
  }
  return select_finish<NT, PIECES>(P, S, a, gub, wb, build);
}

// ---------------------------------------------------------------------------
// Incremental bounds (an option): the children of the selected box share every
// term that involves none of its split coordinates.  The selection workgroup
// forms the canonical sum of those terms once (slot order, the affected terms
// left out) and a table of the affected terms for every combination of halves
// of the split coordinates they involve; a child is then bounded in one thread:
// F = base + its affected terms in increasing index, the midpoint upper bound
// likewise, the first-order test on the coordinates whose derivative involves a
// split coordinate (the parent passed it on every other one, with the same
// intervals), the widest side from the parent's unsplit sides.  GUB takes the
// minimum of the children's midpoint bounds (this workgroup is the only writer
// of the problem's GUB here).
//
// Tables: for an affected term a the halves of its coordinates (a; a and a + 1
// for the chained family) index 2 or 4 entries; for an affected derivative
// coordinate g of the chained family, the halves of g - 1, g, g + 1 index 8
// test results.  A coordinate that is not split has a single "half", the
// parent's interval, so its bit is taken as 0.
// The counters of a problem that its sweep workgroup keeps current itself while
// it runs (every thread holds the same copy).  The workgroup still writes each
// of them to the problem's State as before; the copy only spares it reading back
// from device memory what it has just written.
struct Hot {
  uint64_t gub_key;
  int64_t n_keys, next_seq, sweeps, n_live, evaluated, ub_evaluated;
};
// a value every lane holds alike, moved to scalar registers
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int64_t uni64(int64_t v) { return (int64_t)uni64((uint64_t)v); }
__device__ __forceinline__ Hot hot_load(const State* S) {
  const auto Sg = G(S);
  return Hot{uni64(Sg->gub_key), uni64(Sg->n_keys), uni64(Sg->next_seq), uni64(Sg->sweeps),
             uni64(Sg->n_live), uni64(Sg->evaluated), uni64(Sg->ub_evaluated)};
}
// the selected box: its row, cycling index, split mask and insertion number
struct Sel {
  int64_t row, seq;
  int32_t cyc;
  uint32_t mask;
};

constexpr int kIbChunkTerms = 2048;  // base terms evaluated by the workgroup between two barriers
// The sweep on several workgroups leaves in Params::ibsum: the 64 slot sums of F's
// two endpoints and of the midpoint bound [3][64]; for the separable families the
// table entries of each split index j and half b [kMaxSplit][2][4] (F's enclosure
// of the term, its midpoint bound, the first-order test as 0 or 1); the widest
// unsplit side of each block of coordinates.
constexpr int kIbTabOff = 3 * kWave;
constexpr int kIbWOff = kIbTabOff + kMaxSplit * 2 * 4;
constexpr int kTermCacheMinN = 1024;  // the term cache pays for its 24 n bytes per row from this n on
constexpr int kIbMaxTerms = kMaxSplit + 1;
constexpr int kIbCacheChildren = 1024;   // children whose bounds are kept in LDS between the two passes
constexpr int kIbMaxGrad = kMaxSplit + 2;
constexpr int kIbGroup = 6;              // table rows a child reads together (their LDS reads overlap)
constexpr int kIbSlots = 18;             // rows of each table: a multiple of kIbGroup, >= both maxima above
constexpr int kIbPreBits = 6;            // split positions folded into the prefix table (2^6 entries)
static_assert(kIbSlots % kIbGroup == 0 && kIbSlots >= kIbMaxTerms && kIbSlots >= kIbMaxGrad, "table rows");

template <int NT>
struct IbLds {
  static constexpr int CH = kIbChunkTerms / NT;   // terms per thread between two barriers
  double tfn[kIbChunkTerms], tfh[kIbChunkTerms], tu[kIbChunkTerms];
  double red[NT / kWave];
  int cnt[NT / kWave], ins[NT / kWave];
  double wred[NT / kWave];              // widest unsplit side per wavefront
  int naff, ngc;
  int aff[kIbSlots];                 // affected terms, increasing
  int aj[kIbSlots][2];                  // split index of the term's coordinates (-1: not split)
  double t_n[kIbSlots][4], t_h[kIbSlots][4], t_u[kIbSlots][4];
  double c_flo[kIbCacheChildren], c_wm[kIbCacheChildren];   // the children's bounds (nch <= kIbCacheChildren)
  int8_t c_keep[kIbCacheChildren];      // 1: first-order test passed
  int gc[kIbSlots];                  // CHAIN: affected derivative coordinates, increasing
  int gj[kIbSlots][3];                   // CHAIN: split index of g - 1, g, g + 1 (-1: not split / absent)
  int gmono[kIbSlots][8];                // first-order test failed, per combination of halves
  double w[kMaxSplit][2];               // width of each half of each split coordinate
  double w4[kMaxSplit / 4][16];         // widest split half over coordinates 4g..4g+3 for each 4 bits of c
  // prefix table: for each choice x of halves at the first kIbPreBits sorted
  // positions of the split window, F and the midpoint bound after the leading
  // terms that involve only those positions, and the first-order tests of the
  // leading derivative coordinates that do
  double pre_n[1 << kIbPreBits], pre_h[1 << kIbPreBits], pre_u[1 << kIbPreBits];
  int pre_mo[1 << kIbPreBits];
  int pre_terms, pre_grads, start;      // leading entries in the table; sorted position 0 is split index start
};

// the interval of coordinate i of the selected row for half b of split index j
__device__ __forceinline__ I ib_half(const double* rn, const double* rh, const double* mid, int i, int j, int b) {
  if (j < 0) return I{G(rn)[i], G(rh)[i]};
  const double md = G(mid)[j];
  return b ? I{neg(md), G(rh)[i]} : I{G(rn)[i], md};
}

// wb0 >= 0: this thread's widest side outside the split window, taken when the
// row was built (the base pass then reads the row only where it needs it);
// negative: the base pass forms the widest side itself.  presum: the base pass
// was done on several workgroups (k_ib_rowterms, k_ib_slots), which left the 64
// slot sums of F's endpoints and of the midpoint bound and the widest unsplit
// side of each of nblk coordinate blocks there.
template <int NT, int FAM>
__device__ __forceinline__ void ib_prepare(const Params& P, IbLds<NT>& L, const Sel& sel, double wb0 = -1.0,
                                           const double* presum = nullptr, int nblk = 0) {
  static_assert(NT % kWave == 0, "whole wavefronts");
  __syncthreads();   // the selected row and its split points were written by other threads
  const int n = P.n, m = P.m, lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  const int64_t row = sel.row;
  const int cyc = sel.cyc;
  const uint32_t mask = sel.mask;
  const double* rn = P.hist_n + (int64_t)row * n;
  const double* rh = P.hist_h + (int64_t)row * n;
  const double* mid = P.hist_mid + (int64_t)row * kMaxSplit;
  auto split_of = [&](int i) -> int {   // j if coordinate i is split, else -1
    if (i < 0 || i >= n) return -1;
    int j = i - cyc;
    if (j < 0) j += n;
    return (j < m && ((mask >> j) & 1u)) ? j : -1;
  };
  const int T = FAM == FAM_CHAIN ? n - 1 : n;

  // 1. lists of affected terms and derivative coordinates, in increasing index.
  //    Lane k of wavefront 0 takes the k-th smallest coordinate d of the split
  //    window; if d is split it adds the entries its predecessor in that order
  //    has not added (chained family: term d - 1 unless the predecessor is d - 1,
  //    term d unless d is the last coordinate; derivative coordinates up to d + 1
  //    beyond the predecessor's d' + 1).  An exclusive scan places them.
  if (wid == 0) {
    const int start = (n - cyc < m) ? n - cyc : 0;   // position 0: first j whose coordinate wrapped to the front
    const int k = lane;
    const int j = k < m ? add_mod(start, k, m) : 0;
    const bool sp = k < m && ((mask >> j) & 1u);
    const int d = sp ? add_mod(cyc, j, n) : 0;
    const unsigned long long below = __ballot(sp) & ((1ull << k) - 1ull);
    const int prev = below != 0ull ? add_mod(cyc, add_mod(start, 63 - __clzll(below), m), n) : -2;
    int nt = 0, ngr = 0, a0 = 0, g0 = 0;
    if (sp) {
      if (FAM == FAM_CHAIN) {
        const bool lo_new = d >= 1 && prev != d - 1;
        a0 = lo_new ? d - 1 : d;
        nt = (lo_new ? 1 : 0) + (d < T ? 1 : 0);
        const int last_g = prev >= 0 ? prev + 1 : -1;
        g0 = max(max(d - 1, last_g + 1), 0);
        const int g1 = min(d + 1, n - 1);
        ngr = g1 >= g0 ? g1 - g0 + 1 : 0;
      } else {
        a0 = d;
        nt = 1;
      }
    }
    int it = nt, ig = ngr;
    for (int h = 1; h < kWave; h <<= 1) {
      const int ot = __shfl_up(it, h, kWave), og = __shfl_up(ig, h, kWave);
      if (lane >= h) { it += ot; ig += og; }
    }
    const int pt = it - nt, pg = ig - ngr;   // at most kIbMaxTerms terms, kIbMaxGrad coordinates in all
    for (int e = 0; e < nt; ++e) {
      const int a = a0 + e;
      L.aff[pt + e] = a;
      L.aj[pt + e][0] = split_of(a);
      L.aj[pt + e][1] = FAM == FAM_CHAIN ? split_of(a + 1) : -1;
    }
    if (FAM == FAM_CHAIN)
      for (int e = 0; e < ngr; ++e) {
        const int g = g0 + e;
        L.gc[pg + e] = g;
        L.gj[pg + e][0] = split_of(g - 1);
        L.gj[pg + e][1] = split_of(g);
        L.gj[pg + e][2] = split_of(g + 1);
      }
    if (lane == kWave - 1) {
      L.naff = it;
      L.ngc = ig;
    }
  }
  __syncthreads();

  // 2. the tables (threads from the top down, so that they overlap the base sums
  //    of the first chunk when n is small; each kind of entry in wavefronts of
  //    its own, so that no wavefront runs two kinds one after the other) and the
  //    widths of the halves
  static_assert(NT >= 128 + 8 * kIbMaxGrad && 2 * kIbMaxTerms <= kWave && 4 * kIbMaxTerms <= 128,
                "one thread per table entry");
  {
    const int q = NT - 1 - (int)threadIdx.x;
    const int na = L.naff, ng = L.ngc;
    if (FAM != FAM_CHAIN) {                     // separable: F, midpoint bound, first-order test of each half
      const int part = q >> 6, r = q & (kWave - 1);
      if (part < 3 && r < 2 * na && presum) {   // formed by k_ib_rowterms (the same functions of the same halves)
        const int k = r >> 1, b = r & 1;
        const double* e = presum + kIbTabOff + (L.aj[k][0] * 2 + b) * 4;
        if (part == 0) {
          L.t_n[k][b] = G(e)[0];
          L.t_h[k][b] = G(e)[1];
        } else if (part == 1) {
          L.t_u[k][b] = G(e)[2];
        } else {
          L.gmono[k][b] = G(e)[3] != 0.0 ? 1 : 0;
        }
      } else if (part < 3 && r < 2 * na) {
        const int k = r >> 1, b = r & 1;
        const int a = L.aff[k];
        const I x = ib_half(rn, rh, mid, a, L.aj[k][0], b);
        if (part == 0) {
          const I t = sep_term<FAM>(gload(P.sep + a), x);
          L.t_n[k][b] = t.n;
          L.t_h[k][b] = t.h;
        } else if (part == 1) {
          L.t_u[k][b] = sep_point_hi<FAM>(gload(P.sep + a), midpoint(x));
        } else {
          I t, Gr;
          sep_box<FAM>(gload(P.sep + a), x, t, Gr);
          L.gmono[k][b] = (Gr.n < 0.0 && x.n != G(P.nl)[a]) || (Gr.h < 0.0 && x.h != G(P.u)[a]);
        }
      }
    } else if (q < 4 * na) {                    // chained: affected term, combination of halves
      const int k = q >> 2, cb = q & 3;
      const int a = L.aff[k];
      const int ja = L.aj[k][0], jb = L.aj[k][1];
      if ((ja >= 0 || !(cb & 1)) && (jb >= 0 || !(cb & 2))) {
        const I xa = ib_half(rn, rh, mid, a, ja, cb & 1);
        const I xb = ib_half(rn, rh, mid, a + 1, jb, (cb >> 1) & 1);
        I R, E;
        const CoefChain ca = gload(P.chain + a);
        const I t = chain_term(ca, xa, xb, R, E);
        L.t_n[k][cb] = t.n;
        L.t_h[k][cb] = t.h;
        L.t_u[k][cb] = chain_term(ca, point(midpoint(xa)), point(midpoint(xb)), R, E).h;
      }
    } else if (q >= 128 && q < 128 + 8 * ng) {  // chained: test per combination of halves of g - 1, g, g + 1
      const int k = (q - 128) >> 3, cb = (q - 128) & 7;
      const int g = L.gc[k];
      const int j0 = L.gj[k][0], j1 = L.gj[k][1], j2 = L.gj[k][2];
      int mo = 0;
      if ((j0 >= 0 || !(cb & 1)) && (j1 >= 0 || !(cb & 2)) && (j2 >= 0 || !(cb & 4))) {
        const bool has_prev = g > 0, has_next = g + 1 < n;
        const I xg = ib_half(rn, rh, mid, g, j1, (cb >> 1) & 1);
        const I xp = has_prev ? ib_half(rn, rh, mid, g - 1, j0, cb & 1) : xg;
        const I xq = has_next ? ib_half(rn, rh, mid, g + 1, j2, (cb >> 2) & 1) : xg;
        const I Gr = chain_grad(gload(P.chain + (has_prev ? g - 1 : g)), gload(P.chain + g), xp, xg, xq, has_prev, has_next);
        mo = (Gr.n < 0.0 && xg.n != G(P.nl)[g]) || (Gr.h < 0.0 && xg.h != G(P.u)[g]);
      }
      L.gmono[k][cb] = mo;
    }
  }
  if ((int)threadIdx.x < 2 * m) {              // widths of the halves
    const int j = threadIdx.x >> 1, b = threadIdx.x & 1;
    if ((mask >> j) & 1u) {
      const I x = ib_half(rn, rh, mid, add_mod(cyc, j, n), j, b);
      L.w[j][b] = x.n + x.h;
    }
  }

  // 3. base sums over the terms no split coordinate touches; widest unsplit side.
  //    With the term cache, a term that the parent row's cut left unchanged is the
  //    parent's (same intervals, same value), and every base term is kept for this
  //    row's own children.
  const bool wknown = wb0 >= 0.0;
  auto in_window = [&](int i) {
    int j = i - cyc;
    if (j < 0) j += n;
    return j < m;
  };
  I acc{0.0, 0.0};
  double uacc = 0.0, wb = wknown ? wb0 : 0.0;
  constexpr int CH = IbLds<NT>::CH;
  const int32_t par = P.tcache ? G(P.hist_par)[row] : -1;
  const int pcyc = par >= 0 ? G(P.hist_cyc)[par] : 0;
  const uint32_t pmask = par >= 0 ? G(P.hist_mask)[par] : 0u;
  auto cut_by_parent = [&](int i) -> bool {   // coordinate i differs from the parent row's
    if (i >= n) return false;
    int j = i - pcyc;
    if (j < 0) j += n;
    return j < m && ((pmask >> j) & 1u);
  };
  const double* ptc = par >= 0 ? P.tcache + (int64_t)par * 3 * n : nullptr;
  double* rtc = P.tcache ? P.tcache + row * 3 * n : nullptr;
  if (presum) {
    for (int k = (int)threadIdx.x; k < nblk; k += NT) wb = dmax(wb, G(presum)[kIbWOff + k]);
    if (wid == 0) {
      acc = I{G(presum)[lane], G(presum)[kWave + lane]};
      uacc = G(presum)[2 * kWave + lane];
    }
    // the chunk loop's barriers are skipped: this one orders the tables and
    // widths of step 2 (other wavefronts) before the prefix step reads them
    __syncthreads();
  }
  for (int c0 = 0; c0 < n && !presum; c0 += CH * NT) {
    // Every load of the chunk is issued before any term is formed or stored: the
    // stores into this row's cache may alias the loads as far as the compiler
    // knows, so loads left between them would each wait for the stores before.
    // kind: 0 split or past n, 1 width only (no base term), 2 the parent's cached
    // term, 3 formed here
    int kind[CH];
    I xr[CH];
    double pc[CH][3];
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int i = c0 + r * NT + (int)threadIdx.x;
      int k = 0;
      if (i < n && split_of(i) < 0) {
        k = 1;
        if (i < T && !(FAM == FAM_CHAIN && split_of(i + 1) >= 0))
          k = (ptc && !cut_by_parent(i) && !(FAM == FAM_CHAIN && cut_by_parent(i + 1))) ? 2 : 3;
      }
      kind[r] = k;
      if (k == 3 || (k && (!wknown || in_window(i)))) xr[r] = I{G(rn)[i], G(rh)[i]};
      if (k == 2) {
        pc[r][0] = G(ptc)[i];
        pc[r][1] = G(ptc)[n + i];
        pc[r][2] = G(ptc)[2 * n + i];
      }
    }
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int i = c0 + r * NT + (int)threadIdx.x;
      I t{0.0, 0.0};
      double u = 0.0;
      if (kind[r] >= 1 && (!wknown || in_window(i))) wb = dmax(wb, xr[r].n + xr[r].h);
      if (kind[r] == 2) {
        t = I{pc[r][0], pc[r][1]};
        u = pc[r][2];
      } else if (kind[r] == 3) {   // a term the parent's cut changed, or no cache: formed here
        if constexpr (FAM == FAM_CHAIN) {
          const I xn{G(rn)[i + 1], G(rh)[i + 1]};
          I R, E;
          const CoefChain ci = gload(P.chain + i);
          t = chain_term(ci, xr[r], xn, R, E);
          u = chain_term(ci, point(midpoint(xr[r])), point(midpoint(xn)), R, E).h;
        } else {
          const CoefSep ci = gload(P.sep + i);
          t = sep_term<FAM>(ci, xr[r]);
          u = sep_point_hi<FAM>(ci, midpoint(xr[r]));
        }
      }
      if (kind[r] >= 2 && rtc) {
        G(rtc)[i] = t.n;
        G(rtc)[n + i] = t.h;
        G(rtc)[2 * n + i] = u;
      }
      L.tfn[r * NT + threadIdx.x] = t.n;
      L.tfh[r * NT + threadIdx.x] = t.h;
      L.tu[r * NT + threadIdx.x] = u;
    }
    __syncthreads();
    // slot = lane: terms c0 + q*64 + lane in increasing order (rows past n hold
    // only zeros, and a zero added to a slot sum started at +0 changes no bit);
    // V rows are read before they are added, in the same order
    const int qn = min(CH * NT / kWave, (n - c0 + kWave - 1) / kWave);
    if (wid == 0) {
      constexpr int V = NT >= 1024 ? 2 : 8;   // registers: 128 per lane at 1024 threads
      int q = 0;
      for (; q + V <= qn; q += V) {
        double vn[V], vh[V], vu[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          vn[e] = L.tfn[(q + e) * kWave + lane];
          vh[e] = L.tfh[(q + e) * kWave + lane];
          vu[e] = L.tu[(q + e) * kWave + lane];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          acc = add(acc, I{vn[e], vh[e]});
          uacc = uacc + vu[e];
        }
      }
      for (; q < qn; ++q) {
        acc = add(acc, I{L.tfn[q * kWave + lane], L.tfh[q * kWave + lane]});
        uacc = uacc + L.tu[q * kWave + lane];
      }
    }
    __syncthreads();
  }
  if (wid == 0) {
    // the slot folds of F and of the midpoint bound (slot s absorbs s + h) and the widest side
    for (int h = 32; h >= 1; h >>= 1) {
      const double on = __shfl_down(acc.n, h, kWave), oh = __shfl_down(acc.h, h, kWave);
      const double ou = __shfl_down(uacc, h, kWave), ow = __shfl_xor(wb, h, kWave);
      if (lane < h) {
        acc = add(acc, I{on, oh});
        uacc = uacc + ou;
      }
      wb = dmax(wb, ow);
    }
    const I base{__shfl(acc.n, 0, kWave), __shfl(acc.h, 0, kWave)};
    const double base_u = __shfl(uacc, 0, kWave);
    if (lane == 0) L.wred[0] = wb;
    // the prefix table, lane x: bit p of x is the half at sorted position p; the
    // leading entries whose split coordinates all lie at positions below K
    const int start = (n - cyc < m) ? n - cyc : 0;
    const int K = min(m, kIbPreBits);
    auto pos = [&](int j) { return j < 0 ? -1 : (j >= start ? j - start : j - start + m); };
    const int na = L.naff, ng = L.ngc;
    const int le = min(lane, kIbSlots - 1);
    const bool tin = lane < na && max(pos(L.aj[le][0]), pos(L.aj[le][1])) < K;
    const int pre_t = min(__builtin_ctzll(~__ballot(tin)), kIbPreBits + 1);
    int pre_g = 0;
    if (FAM == FAM_CHAIN) {
      const bool gin = lane < ng && max(max(pos(L.gj[le][0]), pos(L.gj[le][1])), pos(L.gj[le][2])) < K;
      pre_g = min(__builtin_ctzll(~__ballot(gin)), kIbPreBits + 2);
    }
    const int x = lane;
    I F = base;
    double u = base_u;
    int mo = 0;
    // at most K + 1 terms and K + 2 derivative coordinates involve only positions
    // below K: their rows are read together, then added in order
    constexpr int kPreT = kIbPreBits + 1, kPreG = kIbPreBits + 2;
    {
      double tn[kPreT], th[kPreT], tu[kPreT];
      int gm[kPreT];
#pragma unroll
      for (int e = 0; e < kPreT; ++e) {
        const int er = min(e, kIbSlots - 1);
        const int pa = pos(L.aj[er][0]), pb = pos(L.aj[er][1]);
        const int cb = (pa >= 0 ? (x >> pa) & 1 : 0) | (pb >= 0 ? ((x >> pb) & 1) << 1 : 0);
        tn[e] = L.t_n[er][cb];
        th[e] = L.t_h[er][cb];
        tu[e] = L.t_u[er][cb];
        gm[e] = FAM != FAM_CHAIN ? L.gmono[er][cb] : 0;
      }
#pragma unroll
      for (int e = 0; e < kPreT; ++e)
        if (e < pre_t) {
          F = add(F, I{tn[e], th[e]});
          u = u + tu[e];
          mo |= gm[e];
        }
    }
    if (FAM == FAM_CHAIN) {
#pragma unroll
      for (int g = 0; g < kPreG; ++g) {
        const int gr = min(g, kIbSlots - 1);
        const int p0 = pos(L.gj[gr][0]), p1 = pos(L.gj[gr][1]), p2 = pos(L.gj[gr][2]);
        const int cb = (p0 >= 0 ? (x >> p0) & 1 : 0) | (p1 >= 0 ? ((x >> p1) & 1) << 1 : 0) |
                       (p2 >= 0 ? ((x >> p2) & 1) << 2 : 0);
        const int v = L.gmono[gr][cb];
        if (g < pre_g) mo |= v;
      }
    }
    L.pre_n[x] = F.n;
    L.pre_h[x] = F.h;
    L.pre_u[x] = u;
    L.pre_mo[x] = mo;
    if (x == 0) {
      L.pre_terms = pre_t;
      L.pre_grads = pre_g;
      L.start = start;
    }
  } else {
    wb = wave_max(wb);
    if (lane == 0) L.wred[wid] = wb;
    if (wid == 1) {   // L.w was written before the barriers above
      const int g = lane >> 4, nib = lane & 15;
      double w = 0.0;
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * g + b;
        if (j < m && ((mask >> j) & 1u)) w = dmax(w, L.w[j][(nib >> b) & 1]);
      }
      L.w4[g][nib] = w;
    }
  }
  __syncthreads();
}

// bit j of child c; 0 for j < 0 (the coordinate is not split)
__device__ __forceinline__ int child_bit(uint32_t c, int j) { return j >= 0 ? (int)((c >> (j & 31)) & 1u) : 0; }

// bounds of child c from the tables: lower bound, first-order test failed,
// widest side, midpoint upper bound.  Rows are read kIbGroup at a time (a row
// past the table's length is read but not used), then added in increasing order.
template <int NT, int FAM>
__device__ __forceinline__ void ib_child(const Params& P, const IbLds<NT>& L, uint32_t mask, int m, uint32_t c,
                                         double wbase, double& flo, bool& mo, double& wm, double& u) {
  // the table entry for c's halves at the first sorted positions (c rotated so
  // that bit p is sorted position p), then the remaining entries in order
  const int st = L.start;
  const uint32_t cr = ((c >> st) | (c << ((m - st) & 31))) & ((1u << m) - 1u);   // m <= 16; st = 0: c
  const uint32_t x = cr & ((1u << kIbPreBits) - 1u);
  I F{L.pre_n[x], L.pre_h[x]};
  u = L.pre_u[x];
  wm = wbase;
  mo = L.pre_mo[x] != 0;
  const int na = L.naff;
  for (int k0 = L.pre_terms; k0 < na; k0 += kIbGroup) {
    int cb[kIbGroup], kr[kIbGroup];
#pragma unroll
    for (int g = 0; g < kIbGroup; ++g) {
      kr[g] = min(k0 + g, kIbSlots - 1);   // rows past na are read but not used
      cb[g] = child_bit(c, L.aj[kr[g]][0]) | (child_bit(c, L.aj[kr[g]][1]) << 1);
    }
    double tn[kIbGroup], th[kIbGroup], tu[kIbGroup];
    int gm[kIbGroup];
#pragma unroll
    for (int g = 0; g < kIbGroup; ++g) {
      tn[g] = L.t_n[kr[g]][cb[g]];
      th[g] = L.t_h[kr[g]][cb[g]];
      tu[g] = L.t_u[kr[g]][cb[g]];
      gm[g] = FAM != FAM_CHAIN ? L.gmono[kr[g]][cb[g]] : 0;
    }
#pragma unroll
    for (int g = 0; g < kIbGroup; ++g)
      if (k0 + g < na) {
        F = add(F, I{tn[g], th[g]});
        u = u + tu[g];
        mo = mo || gm[g];
      }
  }
  if (FAM == FAM_CHAIN) {
    const int ng = L.ngc;
    for (int k0 = L.pre_grads; k0 < ng; k0 += kIbGroup) {
      int gm[kIbGroup];
#pragma unroll
      for (int g = 0; g < kIbGroup; ++g) {
        const int kr = min(k0 + g, kIbSlots - 1);
        const int cb = child_bit(c, L.gj[kr][0]) | (child_bit(c, L.gj[kr][1]) << 1) | (child_bit(c, L.gj[kr][2]) << 2);
        gm[g] = L.gmono[kr][cb];
      }
#pragma unroll
      for (int g = 0; g < kIbGroup; ++g)
        if (k0 + g < ng) mo = mo || gm[g];
    }
  }
  static_assert(kMaxSplit == 16, "four nibbles of the child index");
  wm = dmax(wm, dmax(dmax(L.w4[0][c & 15u], L.w4[1][(c >> 4) & 15u]), dmax(L.w4[2][(c >> 8) & 15u], L.w4[3][(c >> 12) & 15u])));
  flo = lo_or_ninf(neg(F.n));
}

// GUB = min(GUB, the children's midpoint bounds); returns the new GUB and the
// number of children formed to every thread (each thread reduces the
// wavefronts' partials itself: the same values in the same order)
template <int NT, int FAM>
__device__ __forceinline__ double ib_gub(const Params& P, State* S, IbLds<NT>& L, uint32_t mask, Hot& h,
                                         int& formed) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  double wbase = 0.0;   // widest unsplit side
  for (int k = 0; k < NT / kWave; ++k) wbase = dmax(wbase, L.wred[k]);
  double umin = __builtin_inf();
  int cnt = 0;
  const bool cache = P.nch <= kIbCacheChildren;
  for (int c = threadIdx.x; c < P.nch; c += NT) {
    if (((uint32_t)c & ~mask) != 0u) continue;
    double flo, wm, u;
    bool mo;
    ib_child<NT, FAM>(P, L, mask, P.m, (uint32_t)c, wbase, flo, mo, wm, u);
    if (cache) {
      L.c_flo[c] = flo;
      L.c_wm[c] = wm;
      L.c_keep[c] = mo ? 0 : 1;
    }
    umin = dmin(umin, hi_or_inf(u));
    ++cnt;
  }
  for (int h = 32; h >= 1; h >>= 1) {
    umin = dmin(umin, __shfl_xor(umin, h, kWave));
    cnt += __shfl_xor(cnt, h, kWave);
  }
  if (lane == 0) { L.red[wid] = umin; L.cnt[wid] = cnt; }
  __syncthreads();   // L.red and L.cnt are written again only in the next sweep, after more barriers
  double mn = L.red[0];
  int tot = L.cnt[0];
  for (int k = 1; k < NT / kWave; ++k) { mn = dmin(mn, L.red[k]); tot += L.cnt[k]; }
  const uint64_t key = okey(mn);
  const bool lower = tot > 0 && key < h.gub_key;
  if (threadIdx.x == 0) {
    if (lower) G(S)->gub_key = key;
    G(S)->ub_evaluated = h.ub_evaluated + tot;
  }
  if (lower) h.gub_key = uni64(key);
  h.ub_evaluated = uni64(h.ub_evaluated + tot);
  formed = tot;
  return okey_inv(h.gub_key);
}

// The survivors (first-order test passed, lower bound <= the new GUB) are
// appended right away, in child order, exactly as the next selection would
// insert them from child records (the full-bound path): no records round-trip
// through device memory
template <int NT, int FAM>
__device__ __forceinline__ void ib_children_insert(const Params& P, State* S, IbLds<NT>& L, const Sel& sel, Hot& h,
                                                   double wb0 = -1.0, const double* presum = nullptr,
                                                   int nblk = 0) {
  ib_prepare<NT, FAM>(P, L, sel, wb0, presum, nblk);
  int formed = 0;
  const double gub = ib_gub<NT, FAM>(P, S, L, sel.mask, h, formed);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  const uint32_t mask = sel.mask;
  const int64_t base = h.n_keys, seq0 = h.next_seq;
  const int row = (int)sel.row;
  int64_t done = 0;
  if (P.nch <= kIbCacheChildren) {
    // bounds cached in LDS: each thread takes cpt consecutive children, one scan
    // places them (children stay in child order)
    const int cpt = (P.nch + NT - 1) / NT;
    const int c0 = (int)threadIdx.x * cpt;
    int mine = 0;
    for (int k = 0; k < cpt; ++k) {
      const int c = c0 + k;
      mine += (c < P.nch && (((uint32_t)c & ~mask) == 0u) && L.c_keep[c] != 0 && !(L.c_flo[c] > gub)) ? 1 : 0;
    }
    int incl = mine;
    for (int h = 1; h < kWave; h <<= 1) {
      const int o = __shfl_up(incl, h, kWave);
      if (lane >= h) incl += o;
    }
    if (lane == kWave - 1) L.ins[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NT / kWave; ++k) {
      const int v = L.ins[k];
      before += k < wid ? v : 0;
      total += v;
    }
    int64_t o = before + incl - mine;
    for (int k = 0; k < cpt; ++k) {
      const int c = c0 + k;
      if (c < P.nch && (((uint32_t)c & ~mask) == 0u) && L.c_keep[c] != 0 && !(L.c_flo[c] > gub)) {
        G(P.key_flo)[base + o] = L.c_flo[c];
        G(P.key_seq)[base + o] = seq0 + o;
        G(P.key_ref)[base + o] = row;
        G(P.key_r)[base + o] = c;
        G(P.key_wmax)[base + o] = L.c_wm[c];
        ++o;
      }
    }
    done = total;
    __syncthreads();   // L.ins is rewritten by the next use
  }
  for (int c0 = 0; c0 < P.nch && P.nch > kIbCacheChildren; c0 += NT) {
    const int c = c0 + (int)threadIdx.x;
    double flo = 0.0, wm = 0.0, u;
    bool mo = true;
    const bool formed = c < P.nch && (((uint32_t)c & ~mask) == 0u);
    if (formed) {   // bounds not cached: formed again from the tables
      double wbase = 0.0;
      for (int k = 0; k < NT / kWave; ++k) wbase = dmax(wbase, L.wred[k]);
      ib_child<NT, FAM>(P, L, mask, P.m, (uint32_t)c, wbase, flo, mo, wm, u);
    }
    const int keep = formed && !mo && !(flo > gub);
    int incl = keep;
    for (int h = 1; h < kWave; h <<= 1) {
      const int o = __shfl_up(incl, h, kWave);
      if (lane >= h) incl += o;
    }
    if (lane == kWave - 1) L.ins[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NT / kWave; ++k) {
      const int v = L.ins[k];
      before += k < wid ? v : 0;
      total += v;
    }
    if (keep) {
      const int64_t o = done + before + incl - 1;
      G(P.key_flo)[base + o] = flo;
      G(P.key_seq)[base + o] = seq0 + o;
      G(P.key_ref)[base + o] = row;
      G(P.key_r)[base + o] = c;
      G(P.key_wmax)[base + o] = wm;
    }
    done += total;
    __syncthreads();   // L.ins is rewritten by the next round
  }
  const int64_t t = h.sweeps;
  if (threadIdx.x == 0) {
    if (t < P.trace_cap) {
      G(P.tr_gub)[t] = gub;
      G(P.tr_nsurv)[t] = done;
      G(P.tr_sel)[t] = sel.seq;
    }
    const auto Sg = G(S);
    Sg->n_keys = base + done;
    Sg->next_seq = seq0 + done;
    Sg->evaluated = h.evaluated + formed;
    Sg->sweeps = t + 1;
    Sg->pending = 0;
  }
  h.n_keys = uni64(base + done);
  h.next_seq = uni64(seq0 + done);
  h.evaluated = uni64(h.evaluated + formed);
  h.sweeps = t + 1;
}

// Up to `iters` whole sweeps with incremental bounds in one workgroup: the
// selection scans the list itself, the children are bounded, GUB updated and
// the survivors inserted.  Problems are independent, so one workgroup per
// problem loops without any grid-wide barrier.
// Stable in-place compaction of the keys by one workgroup: keys whose lower
// bound exceeds GUB (and removed keys, +inf) are dropped; the order, and so the
// insertion numbers and every later selection, are unchanged.  Each chunk of NT
// keys is read completely before any of it is written, and a key only moves to
// a lower index, so no key is overwritten before it has been read.
template <int NT>
__device__ __forceinline__ void compact_in_place(const Params& P, State* S, IbLds<NT>& L, Hot& h) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  const double gub = okey_inv(h.gub_key);
  const int64_t nk = h.n_keys;
  int64_t kept = 0;
  for (int64_t c0 = 0; c0 < nk; c0 += NT) {
    const int64_t i = c0 + threadIdx.x;
    double f = __builtin_inf(), w = 0.0;
    int64_t sq = 0;
    int32_t rf = 0, rr = 0;
    const bool in = i < nk;
    if (in) { f = G(P.key_flo)[i]; sq = G(P.key_seq)[i]; rf = G(P.key_ref)[i]; rr = G(P.key_r)[i]; w = G(P.key_wmax)[i]; }
    const int keep = in && f <= gub;
    int incl = keep;
    for (int h = 1; h < kWave; h <<= 1) {
      const int o = __shfl_up(incl, h, kWave);
      if (lane >= h) incl += o;
    }
    if (lane == kWave - 1) L.ins[wid] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NT / kWave; ++k) {
      const int v = L.ins[k];
      before += k < wid ? v : 0;
      total += v;
    }
    if (keep) {
      const int64_t o = kept + before + incl - 1;
      G(P.key_flo)[o] = f; G(P.key_seq)[o] = sq; G(P.key_ref)[o] = rf; G(P.key_r)[o] = rr; G(P.key_wmax)[o] = w;
    }
    kept += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) G(S)->n_keys = kept;
  h.n_keys = uni64(kept);
  __syncthreads();
}

// The selection of the persistent loop: the steps of select_body and
// select_finish for a list with no pending children, with the counters taken
// from the workgroup's own copy.  Every wavefront forms the split mask itself
// (the same ballot over the same values), so no thread waits to read it back.
template <int NT>
__device__ __forceinline__ bool select_ib(const Params& P, State* S, Hot& h, Sel& sel, double& wb) {
  const double gub = okey_inv(h.gub_key);
  // each thread fetches the row reference of its own candidate while the
  // workgroup reduces; the winner's thread passes it on through LDS
  __shared__ int32_t go, w_ref, w_r;
  __shared__ int64_t w_seq;
  SelAcc tot;
  bool pre = false;
  if (scan_own_ok<NT>(P, h.n_keys)) {
    const OwnSel own = scan_own<NT>(P, gub, h.n_keys);
    int32_t o_ref = 0, o_r = 0;
    int64_t o_seq = 0;
    if (own.bi != INT32_MAX) {
      o_ref = G(P.key_ref)[own.bi];
      o_r = G(P.key_r)[own.bi];
      o_seq = G(P.key_seq)[own.bi];
    }
    tot = reduce_own<NT>(P, own);
    if (own.bi != INT32_MAX && (int64_t)own.bi == tot.best.idx) {   // one thread: each key has one scanner
      w_ref = o_ref;
      w_r = o_r;
      w_seq = o_seq;
    }
    pre = true;
  } else {
    tot = scan_select_wg<NT>(P, gub, h.n_keys);
  }
  const int64_t t = h.sweeps, row = t + 1;
  const auto Sg = G(S);
  if (threadIdx.x == 0) {
    const Cand b = tot.best;
    if (t > 0 && t - 1 < P.trace_cap) G(P.tr_nlive)[t - 1] = tot.cnt;
    Sg->n_live = tot.cnt;
    Sg->glb = b.f;
    Sg->wmax = tot.wm;
    int32_t stop = RUNNING;
    if (tot.cnt == 0) stop = STOP_EMPTY;
    else if (b.idx < 0 || b.idx >= h.n_keys) stop = STOP_INTERNAL;
    else if (gub - b.f <= P.tol_f && (P.tol_x <= 0.0 || tot.wm < P.tol_x)) stop = STOP_CONVERGED;
    else if (t >= P.max_sweeps) stop = STOP_SWEEPS;
    else if (P.max_live > 0 && tot.cnt > P.max_live) stop = STOP_LIVE;
    else if (row >= P.hist_cap || h.n_keys + P.nch > P.key_cap) stop = STOP_CAPACITY;
    if (stop) Sg->stop = stop;
    go = stop == RUNNING;
    if (go) {
      G(P.key_flo)[b.idx] = __builtin_inf();     // removed from the list
      Sg->gub_start = gub;
      Sg->pending = 1;
    }
  }
  __syncthreads();
  h.n_live = uni64(tot.cnt);
  if (!go) return false;
  const int32_t ref = pre ? w_ref : G(P.key_ref)[tot.best.idx];
  const int32_t r = pre ? w_r : G(P.key_r)[tot.best.idx];
  const int64_t seq = pre ? w_seq : G(P.key_seq)[tot.best.idx];
  const int n = P.n;
  const int pcyc = G(P.hist_cyc)[ref];
  const ChildRow src{P.hist_n + (int64_t)ref * n, P.hist_h + (int64_t)ref * n, P.hist_mid + (int64_t)ref * kMaxSplit,
                     n, P.m, pcyc, r >= 0 ? G(P.hist_mask)[ref] : 0u, r >= 0 ? (uint32_t)r : 0u};
  const int cyc = r >= 0 ? add_mod(pcyc, P.m, n) : pcyc;   // m <= n
  wb = build_row<NT>(src, P.hist_n + row * n, P.hist_h + row * n, n, cyc, P.m);
  const int lane = threadIdx.x & (kWave - 1);
  bool ok = false;
  double md = 0.0;
  if (lane < P.m) {
    const I x = src.get(add_mod(cyc, lane, n));
    md = midpoint(x);
    ok = neg(x.n) < md && md < x.h;
  }
  const uint32_t mask = (uint32_t)__ballot(ok) & ((1u << P.m) - 1u);   // m <= 16
  if (threadIdx.x < (unsigned)kWave) {
    if (lane < P.m) {
      G(P.hist_mid)[row * kMaxSplit + lane] = md;
      Sg->sel_mid[lane] = md;
    }
    if (lane == 0) {
      G(P.hist_mask)[row] = mask;
      G(P.hist_cyc)[row] = cyc;
      if (P.hist_par) G(P.hist_par)[row] = r >= 0 ? ref : -1;
      Sg->sel_mask = mask;
      Sg->sel_cyc = cyc;
      Sg->sel_row = (int32_t)row;
      Sg->sel_seq = seq;
    }
  }
  sel.row = row;
  sel.seq = seq;
  sel.cyc = cyc;
  sel.mask = mask;
  return true;
}

// load the selection select_body left in the State (after a barrier)
__device__ __forceinline__ Sel sel_load(const State* S) {
  Sel sel;
  sel.row = (int64_t)__builtin_amdgcn_readfirstlane(S->sel_row);
  sel.seq = uni64(S->sel_seq);
  sel.cyc = __builtin_amdgcn_readfirstlane(S->sel_cyc);
  sel.mask = __builtin_amdgcn_readfirstlane(S->sel_mask);
  return sel;
}

template <int NT, int FAM>
__device__ __forceinline__ void sweeps_ib(const Params& P, State* S, IbLds<NT>& lds, int iters) {
  if (G(S)->stop) return;
  Hot h = hot_load(S);   // no children are pending here: the incremental sweep inserts its own
  for (int it = 0; it < iters; ++it) {
    // dead keys dominate the list: drop them before the scan
    if (h.n_keys > 4 * (h.n_live + P.nch) && h.n_keys > 4096) compact_in_place<NT>(P, S, lds, h);
    Sel sel;
    double wb;
    if (!select_ib<NT>(P, S, h, sel, wb)) return;   // stopped (the flag is set)
    ib_children_insert<NT, FAM>(P, S, lds, sel, h, wb);
    __syncthreads();   // keys written by other threads are read by the next selection
  }
}

template <int NT, int FAM>
__global__ __launch_bounds__(NT) void k_sweeps_ib(const Params* __restrict__ PP, State* __restrict__ S, int iters) {
  round_up_mode();
  __shared__ IbLds<NT> lds;
  sweeps_ib<NT, FAM>(*PP, S, lds, iters);   // parameters read where used: nothing held across the loop
}

template <int NT, int FAM>
__global__ __launch_bounds__(NT) void k_select_ib(const Params* __restrict__ PP, State* __restrict__ S, int nparts,
                                                  int host_stop) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  __shared__ IbLds<NT> lds;
  double wb;
  if (select_body<NT>(P, S, nparts, host_stop, &wb)) {
    __syncthreads();   // the selection was written to the State by wavefront 0
    Hot h = hot_load(S);
    ib_children_insert<NT, FAM>(P, S, lds, sel_load(S), h, wb);
  }
}

// The same sweep with the term cache on several workgroups (one box per sweep,
// n >= kIbPipeMinN): the O(n) work of one box (its row, its base terms) is what
// one workgroup is bound by there, and it splits without changing any sum:
//   k_ib_pick      the selection (select_body; on a long list after the
//                  partials of k_select_part) without the row;
//   k_ib_rowterms  one coordinate per thread: the row, each base term from the
//                  parent's cache or formed (ib_prepare's rules), into this
//                  row's cache, and each block's widest unsplit side; for the
//                  separable families one more workgroup forms the table
//                  entries of the split coordinates' halves;
//   k_ib_slots     the 64 slot sums of F's two endpoints and of the midpoint
//                  bound, one workgroup per sum: each slot adds its terms in
//                  increasing index, as the one-workgroup base pass does (the
//                  slots are independent chains);
//   k_ib_finish    ib_children_insert from those sums and tables (folds,
//                  prefix table, children, GUB, insertion).
// The results are those of the one-workgroup sweep bit for bit.
constexpr int kIbRowBlock = 256;   // coordinates per k_ib_rowterms workgroup, one per thread
static_assert(3 * 2 * kMaxSplit <= kIbRowBlock, "one thread per table entry of the split halves");
// below this n the extra launches cost more than spreading the O(n) pass saves
// (per sweep, one workgroup against several: n = 2048 28 against 30 us, 4096 36
// against 36, 6144 39 against 35)
constexpr int kIbPipeMinN = 5120;

template <int NT>
__global__ __launch_bounds__(NT) void k_ib_pick(const Params* __restrict__ PP, State* __restrict__ S, int nparts,
                                                int host_stop) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  (void)select_body<NT>(P, S, nparts, host_stop, nullptr, false);
}

// a base term of the selected row (the one-workgroup pass's kind 2 or 3): i is
// not cut in the row, has a term, and (chained family) its neighbour is not cut
struct IbRowView {
  int n, m, cyc, T;
  uint32_t mask;
  bool chain;
  __device__ __forceinline__ bool split(int i) const {
    if (i < 0 || i >= n) return false;
    int j = i - cyc;
    if (j < 0) j += n;
    return j < m && ((mask >> j) & 1u);
  }
  __device__ __forceinline__ bool base_term(int i) const {
    return i < n && !split(i) && i < T && !(chain && split(i + 1));
  }
};

template <int FAM>
__global__ __launch_bounds__(kIbRowBlock) void k_ib_rowterms(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  const int n = P.n, m = P.m;
  const int64_t row = S->sel_row;
  const int32_t ref = S->sel_ref, r = S->sel_r;
  const IbRowView V{n, m, S->sel_cyc, FAM == FAM_CHAIN ? n - 1 : n, S->sel_mask, FAM == FAM_CHAIN};
  const ChildRow src{P.hist_n + (int64_t)ref * n, P.hist_h + (int64_t)ref * n, P.hist_mid + (int64_t)ref * kMaxSplit,
                     n, m, P.hist_cyc[ref], r >= 0 ? P.hist_mask[ref] : 0u, r >= 0 ? (uint32_t)r : 0u};
  const int32_t par = G(P.hist_par)[row];
  const int pcyc = par >= 0 ? G(P.hist_cyc)[par] : 0;
  const uint32_t pmask = par >= 0 ? G(P.hist_mask)[par] : 0u;
  auto cut_by_parent = [&](int i) -> bool {
    if (i >= n) return false;
    int j = i - pcyc;
    if (j < 0) j += n;
    return j < m && ((pmask >> j) & 1u);
  };
  const double* ptc = par >= 0 ? P.tcache + (int64_t)par * 3 * n : nullptr;
  double* rtc = P.tcache + row * 3 * n;
  double* rn = P.hist_n + row * n;
  double* rh = P.hist_h + row * n;
  if (FAM != FAM_CHAIN && (int)blockIdx.x * kIbRowBlock >= n) {
    // the separable families' last workgroup: the table entries of the split
    // coordinates' halves, which the finishing workgroup would otherwise form
    // (ib_prepare's step 2) while the rest of it waits
    const int part = (int)threadIdx.x / (2 * kMaxSplit), q = (int)threadIdx.x % (2 * kMaxSplit);
    const int j = q >> 1, b = q & 1;
    if (part < 3 && j < m && ((S->sel_mask >> j) & 1u)) {
      const int a = add_mod(S->sel_cyc, j, n);
      const I xa = src.get(a);
      const double md = G(P.hist_mid)[row * kMaxSplit + j];
      const I x = b ? I{neg(md), xa.h} : I{xa.n, md};
      const CoefSep ci = gload(P.sep + a);
      double* e = P.ibsum + kIbTabOff + (j * 2 + b) * 4;
      if (part == 0) {
        const I t = sep_term<FAM>(ci, x);
        G(e)[0] = t.n;
        G(e)[1] = t.h;
      } else if (part == 1) {
        G(e)[2] = sep_point_hi<FAM>(ci, midpoint(x));
      } else {
        I t, Gr;
        sep_box<FAM>(ci, x, t, Gr);
        G(e)[3] = ((Gr.n < 0.0 && x.n != G(P.nl)[a]) || (Gr.h < 0.0 && x.h != G(P.u)[a])) ? 1.0 : 0.0;
      }
    }
    return;
  }
  // one coordinate per thread, every load issued before the stores (which the
  // compiler must assume may alias them)
  const int i = (int)blockIdx.x * kIbRowBlock + (int)threadIdx.x;
  double wb = 0.0;
  if (i < n) {
    const I x = src.get(i);
    const bool sp = V.split(i), bt = V.base_term(i);
    const bool reuse = bt && ptc && !cut_by_parent(i) && !(FAM == FAM_CHAIN && cut_by_parent(i + 1));
    I t{0.0, 0.0};
    double u = 0.0;
    if (reuse) {
      t = I{G(ptc)[i], G(ptc)[n + i]};
      u = G(ptc)[2 * n + i];
    } else if (bt) {
      if constexpr (FAM != FAM_CHAIN) {
        const CoefSep ci = gload(P.sep + i);
        t = sep_term<FAM>(ci, x);
        u = sep_point_hi<FAM>(ci, midpoint(x));
      } else {
        const I xn = src.get(i + 1);   // the next coordinate of this row
        I R, E;
        const CoefChain ci = gload(P.chain + i);
        t = chain_term(ci, x, xn, R, E);
        u = chain_term(ci, point(midpoint(x)), point(midpoint(xn)), R, E).h;
      }
    }
    G(rn)[i] = x.n;
    G(rh)[i] = x.h;
    if (!sp) wb = x.n + x.h;
    if (bt) {
      G(rtc)[i] = t.n;
      G(rtc)[n + i] = t.h;
      G(rtc)[2 * n + i] = u;
    }
  }
  wb = wave_max(wb);
  __shared__ double s_w[kIbRowBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x >> 6] = wb;
  __syncthreads();
  if (threadIdx.x == 0) {
    double w = s_w[0];
    for (int k = 1; k < kIbRowBlock / kWave; ++k) w = dmax(w, s_w[k]);
    G(P.ibsum)[kIbWOff + blockIdx.x] = w;
  }
}

// Workgroup w forms sum w (0: F's negated lower endpoint, 1: its upper
// endpoint, 2: the midpoint bound).  The column is staged in LDS a chunk at a
// time, every load of a chunk in flight together; then lane s of the first
// wavefront adds the terms s, s + 64, ... of the chunk in increasing index.
constexpr int kIbSlotsThreads = 1024;
constexpr int kIbSlotsChunk = 16384;   // 128 KB of LDS (gfx950 has 160 KB per CU)

__global__ __launch_bounds__(kIbSlotsThreads) void k_ib_slots(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  const int n = P.n;
  const bool chain = P.family == FAM_CHAIN;
  const IbRowView V{n, P.m, S->sel_cyc, chain ? n - 1 : n, S->sel_mask, chain};
  const int which = blockIdx.x, lane = threadIdx.x & (kWave - 1);
  const double* col = P.tcache + (int64_t)S->sel_row * 3 * n + (int64_t)which * n;
  __shared__ double buf[kIbSlotsChunk];
  constexpr int R = kIbSlotsChunk / kIbSlotsThreads;
  double acc = 0.0;
  for (int c0 = 0; c0 < n; c0 += kIbSlotsChunk) {
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = c0 + r * kIbSlotsThreads + (int)threadIdx.x;
      v[r] = V.base_term(i) ? G(col)[i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) buf[r * kIbSlotsThreads + threadIdx.x] = v[r];
    __syncthreads();
    if (threadIdx.x < kWave) {
      const int rows = (min(kIbSlotsChunk, n - c0) + kWave - 1) / kWave;   // rows past n hold zeros
      for (int q = 0; q < rows; ++q) acc = acc + buf[q * kWave + lane];
    }
    __syncthreads();
  }
  if (threadIdx.x < kWave) G(P.ibsum)[which * kWave + lane] = acc;
}

// nblk: the workgroups of k_ib_rowterms (each left its widest unsplit side)
template <int NT, int FAM>
__global__ __launch_bounds__(NT) void k_ib_finish(const Params* __restrict__ PP, State* __restrict__ S, int nblk) {
  round_up_mode();
  if (S->stop || !S->pending) return;
  const Params P = *PP;
  __shared__ IbLds<NT> lds;
  Hot h = hot_load(S);
  ib_children_insert<NT, FAM>(P, S, lds, sel_load(S), h, -1.0, P.ibsum, nblk);
}

// K > 1 with incremental bounds: workgroup p bounds the children of the box of
// rank p of the sweep's selection (its own base sums and tables, exactly as the
// K = 1 sweep forms them), writes their records p nch + c for the insertion in
// the next selection, and lowers GUB to the minimum of their midpoint bounds.
template <int NT, int FAM>
__global__ __launch_bounds__(NT) void k_ib_parents(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  const int pr = blockIdx.x;
  if (pr >= S->sel_count) return;
  const Params& P = *PP;
  __shared__ IbLds<NT> lds;
  const SelRec rec = P.sel_tab[pr];
  const Sel sel{rec.row, rec.seq, rec.cyc, rec.mask};
  ib_prepare<NT, FAM>(P, lds, sel);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  double wbase = 0.0;
  for (int k = 0; k < NT / kWave; ++k) wbase = dmax(wbase, lds.wred[k]);
  double umin = __builtin_inf();
  int cnt = 0;
  const int64_t g0 = (int64_t)pr * P.nch;
  for (int c = threadIdx.x; c < P.nch; c += NT) {
    if (((uint32_t)c & ~sel.mask) != 0u) {
      P.ch_flag[g0 + c] = 0;   // takes the upper half of a coordinate that cannot be split
      continue;
    }
    double flo, wm, u;
    bool mo;
    ib_child<NT, FAM>(P, lds, sel.mask, P.m, (uint32_t)c, wbase, flo, mo, wm, u);
    P.ch_flo[g0 + c] = flo;
    P.ch_wmax[g0 + c] = wm;
    P.ch_flag[g0 + c] = mo ? 1 : 2;
    umin = dmin(umin, hi_or_inf(u));
    ++cnt;
  }
  for (int h = 32; h >= 1; h >>= 1) {
    umin = dmin(umin, __shfl_xor(umin, h, kWave));
    cnt += __shfl_xor(cnt, h, kWave);
  }
  if (lane == 0) { lds.red[wid] = umin; lds.cnt[wid] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mn = lds.red[0];
    int tot = lds.cnt[0];
    for (int k = 1; k < NT / kWave; ++k) { mn = dmin(mn, lds.red[k]); tot += lds.cnt[k]; }
    if (tot > 0) {
      atomicMin((unsigned long long*)&S->gub_key, (unsigned long long)okey(mn));
      atomicAdd((unsigned long long*)&S->ub_evaluated, (unsigned long long)tot);
    }
  }
}

// ---------------------------------------------------------------------------
// The schedule of the paper's experiments (Sec. 4): the selected box's m cycled
// coordinates are cut into four equal pieces (Eqs. (8)-(11), digit j of the
// child index picks the piece of the j-th coordinate), 4^m children, each
// sampled at nsamp points of its diagonal.  Children are bounded incrementally:
// k_prep4 (one workgroup) forms, for the selected box, the canonical sums of the
// terms no split coordinate touches (F over the box and the upper bound at each
// of its diagonal points), and tables of the other terms and of the first-order
// test for every combination of pieces of the coordinates they involve;
// k_children4 (one thread per child, the whole chip) adds a child's table
// entries in increasing term index, takes the smallest sample bound into GUB
// and writes the child's record for the next selection to insert.

// offsets in the tables
constexpr int kTabBase = kTabRows * 16 * kTabEntry;   // doubles: base F (-lo, hi), base samples, wbase, widths
constexpr int kTiAff = 4, kTiAj = kTiAff + kTabRows, kTiGc = kTiAj + 2 * kTabRows, kTiGj = kTiGc + kTabRows,
              kTiGm = kTiGj + 3 * kTabRows;
static_assert(kTiGm + 64 * kTabRows <= kTabInts, "table layout");

template <int NT, int FAM>
__global__ __launch_bounds__(NT) void k_prep4(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  const Params& P = *PP;
  const int n = P.n, m = P.m, ns = P.nsamp;
  const int row = S->sel_row, cyc = S->sel_cyc;
  const uint32_t mask = S->sel_mask;
  const double* rn = P.hist_n + (int64_t)row * n;
  const double* rh = P.hist_h + (int64_t)row * n;
  const double* cut = P.hist_cut + (int64_t)row * (3 * kMaxSplit);
  const int T = FAM == FAM_CHAIN ? n - 1 : n;
  auto split_of = [&](int i) -> int {   // window index j if coordinate i is split, else -1
    if (i < 0 || i >= n) return -1;
    int j = i - cyc;
    if (j < 0) j += n;
    return (j < m && ((mask >> j) & 1u)) ? j : -1;
  };
  auto piece = [&](int i, int j, int d) -> I {   // coordinate i of the child with digit d on window index j
    if (j < 0) return I{G(rn)[i], G(rh)[i]};
    return I{d > 0 ? neg(G(cut)[3 * j + d - 1]) : G(rn)[i], d < 3 ? G(cut)[3 * j + d] : G(rh)[i]};
  };
  __shared__ int s_aff[kTabRows], s_aj[kTabRows][2], s_gc[kTabRows], s_gj[kTabRows][3];
  __shared__ int s_naff, s_ngc;
  if (threadIdx.x == 0) {
    // affected terms and derivative coordinates in increasing index (few: m <= 12)
    int ca[3 * kMaxSplit], cg[3 * kMaxSplit];
    int na = 0, ng = 0;
    for (int j = 0; j < m; ++j) {
      if (!((mask >> j) & 1u)) continue;
      const int d = add_mod(cyc, j, n);
      if (d < T) ca[na++] = d;
      if (FAM == FAM_CHAIN && d >= 1) ca[na++] = d - 1;
      cg[ng++] = d;
      if (FAM == FAM_CHAIN) {
        if (d >= 1) cg[ng++] = d - 1;
        if (d + 1 < n) cg[ng++] = d + 1;
      }
    }
    auto sort_unique = [](int* v, int k) {
      for (int a = 1; a < k; ++a)
        for (int b = a; b > 0 && v[b - 1] > v[b]; --b) { const int t = v[b]; v[b] = v[b - 1]; v[b - 1] = t; }
      int u = 0;
      for (int a = 0; a < k; ++a)
        if (u == 0 || v[u - 1] != v[a]) v[u++] = v[a];
      return u;
    };
    na = sort_unique(ca, na);
    ng = sort_unique(cg, ng);
    for (int a = 0; a < na; ++a) {
      s_aff[a] = ca[a];
      s_aj[a][0] = split_of(ca[a]);
      s_aj[a][1] = FAM == FAM_CHAIN ? split_of(ca[a] + 1) : -1;
      P.tabi[kTiAff + a] = ca[a];
      P.tabi[kTiAj + 2 * a] = s_aj[a][0];
      P.tabi[kTiAj + 2 * a + 1] = s_aj[a][1];
    }
    for (int k = 0; k < ng; ++k) {
      const int g = cg[k];
      s_gc[k] = g;
      s_gj[k][0] = FAM == FAM_CHAIN ? split_of(g - 1) : -1;
      s_gj[k][1] = split_of(g);
      s_gj[k][2] = FAM == FAM_CHAIN ? split_of(g + 1) : -1;
      P.tabi[kTiGc + k] = g;
      for (int q = 0; q < 3; ++q) P.tabi[kTiGj + 3 * k + q] = s_gj[k][q];
    }
    s_naff = na;
    s_ngc = ng;
    P.tabi[0] = na;
    P.tabi[1] = ng;
  }
  __syncthreads();
  const int na = s_naff, ng = s_ngc;
  // term tables: F over the pieces and the upper bound at each diagonal point
  for (int e = threadIdx.x; e < na * 16; e += NT) {
    const int a = e >> 4, cb = e & 15, d0 = cb & 3, d1 = cb >> 2;
    const int i = s_aff[a], j0 = s_aj[a][0], j1 = s_aj[a][1];
    if ((j0 < 0 && d0) || (j1 < 0 && d1)) continue;   // a combination no child has
    double* ent = P.tab + (a * 16 + cb) * kTabEntry;
    const I xa = piece(i, j0, d0);
    if (FAM != FAM_CHAIN) {
      const CoefSep c = gload(P.sep + i);
      const I t = sep_term<FAM>(c, xa);
      G(ent)[0] = t.n;
      G(ent)[1] = t.h;
      for (int q = 0; q < ns; ++q) G(ent)[2 + q] = sep_point_hi<FAM>(c, diag_coord(xa, P.cs[q]));
    } else {
      const I xb = piece(i + 1, j1, d1);
      const CoefChain c = gload(P.chain + i);
      I R, E;
      const I t = chain_term(c, xa, xb, R, E);
      G(ent)[0] = t.n;
      G(ent)[1] = t.h;
      for (int q = 0; q < ns; ++q)
        G(ent)[2 + q] = chain_term(c, point(diag_coord(xa, P.cs[q])), point(diag_coord(xb, P.cs[q])), R, E).h;
    }
  }
  // first-order test per combination of the pieces of g - 1, g, g + 1
  for (int e = threadIdx.x; e < ng * 64; e += NT) {
    const int k = e >> 6, cb = e & 63, d0 = cb & 3, d1 = (cb >> 2) & 3, d2 = cb >> 4;
    const int g = s_gc[k], j0 = s_gj[k][0], j1 = s_gj[k][1], j2 = s_gj[k][2];
    int mo = 0;
    if (!((j0 < 0 && d0) || (j1 < 0 && d1) || (j2 < 0 && d2))) {
      const I xg = piece(g, j1, d1);
      I Gr;
      if (FAM != FAM_CHAIN) {
        I t;
        sep_box<FAM>(gload(P.sep + g), xg, t, Gr);
      } else {
        const bool has_prev = g > 0, has_next = g + 1 < n;
        const I xp = has_prev ? piece(g - 1, j0, d0) : xg;
        const I xq = has_next ? piece(g + 1, j2, d2) : xg;
        Gr = chain_grad(gload(P.chain + (has_prev ? g - 1 : g)), gload(P.chain + g), xp, xg, xq, has_prev, has_next);
      }
      mo = (Gr.n < 0.0 && xg.n != G(P.nl)[g]) || (Gr.h < 0.0 && xg.h != G(P.u)[g]);
    }
    P.tabi[kTiGm + 64 * k + cb] = mo;
  }
  // canonical sums (slot i mod 64, slots in order, then the folds) of the terms
  // no split coordinate touches: F over the box and the bound at each diagonal
  // point of the box; the widest side among the coordinates not split
  constexpr int NE = 2 + kMaxSamples;
  __shared__ double sv[NT][NE];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  I acc{0.0, 0.0};
  double su[kMaxSamples];
#pragma unroll
  for (int q = 0; q < kMaxSamples; ++q) su[q] = 0.0;
  double wb = 0.0;
  for (int c0 = 0; c0 < n; c0 += NT) {
    const int i = c0 + (int)threadIdx.x;
    double v[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) v[q] = 0.0;
    if (i < n && split_of(i) < 0) {
      const I x{G(rn)[i], G(rh)[i]};
      wb = dmax(wb, x.n + x.h);
      if (i < T && !(FAM == FAM_CHAIN && split_of(i + 1) >= 0)) {
        if (FAM != FAM_CHAIN) {
          const CoefSep c = gload(P.sep + i);
          const I t = sep_term<FAM>(c, x);
          v[0] = t.n;
          v[1] = t.h;
#pragma unroll
          for (int q = 0; q < kMaxSamples; ++q)
            if (q < ns) v[2 + q] = sep_point_hi<FAM>(c, diag_coord(x, P.cs[q]));
        } else {
          const I xn{G(rn)[i + 1], G(rh)[i + 1]};
          const CoefChain c = gload(P.chain + i);
          I R, E;
          const I t = chain_term(c, x, xn, R, E);
          v[0] = t.n;
          v[1] = t.h;
#pragma unroll
          for (int q = 0; q < kMaxSamples; ++q)
            if (q < ns) v[2 + q] = chain_term(c, point(diag_coord(x, P.cs[q])), point(diag_coord(xn, P.cs[q])), R, E).h;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) sv[threadIdx.x][q] = v[q];
    __syncthreads();
    if (wid == 0) {   // lane s: terms c0 + r*64 + s in increasing order (zeros past n change no bit)
      const int rows = min(NT / kWave, (n - c0 + kWave - 1) / kWave);
      for (int r = 0; r < rows; ++r) {
        const int t = r * kWave + lane;
        acc = add(acc, I{sv[t][0], sv[t][1]});
#pragma unroll
        for (int q = 0; q < kMaxSamples; ++q)
          if (q < ns) su[q] = su[q] + sv[t][2 + q];
      }
    }
    __syncthreads();
  }
  __shared__ double s_wb[NT / kWave];
  wb = wave_max(wb);
  if (lane == 0) s_wb[wid] = wb;
  __syncthreads();
  if (wid == 0) {
    const I F = fold_slots(acc, lane);
    double* base = P.tab + kTabBase;
    if (lane == 0) { G(base)[0] = F.n; G(base)[1] = F.h; }
#pragma unroll
    for (int q = 0; q < kMaxSamples; ++q)
      if (q < ns) {   // uniform branch
        const double u = fold_slots_hi(su[q], lane);
        if (lane == 0) G(base)[2 + q] = u;
      }
    if (lane == 0) {
      double w = 0.0;
      for (int k = 0; k < NT / kWave; ++k) w = dmax(w, s_wb[k]);
      G(base)[2 + kMaxSamples] = w;
    }
    if (lane < 4 * m) {   // widths of the pieces of the split coordinates
      const int j = lane >> 2, d = lane & 3;
      double w = 0.0;
      if ((mask >> j) & 1u) {
        const I x = piece(add_mod(cyc, j, n), j, d);
        w = x.n + x.h;
      }
      G(base)[3 + kMaxSamples + 4 * j + d] = w;
    }
  }
}

// one thread per child of the selected box; the tables in LDS (dynamic: `rows`
// term rows of 16 combinations of 2 + nsamp doubles, then 3 m test rows of 64)
template <int FAM>
__global__ __launch_bounds__(256) void k_children4(const Params* __restrict__ PP, State* __restrict__ S, int rows) {
  round_up_mode();
  if (S->stop) return;
  const Params& P = *PP;
  extern __shared__ double sm[];
  const int na = G(P.tabi)[0], ng = G(P.tabi)[1], ns = P.nsamp, m = P.m;
  const uint32_t mask = S->sel_mask;
  const int E = 2 + ns;                              // doubles per table entry in LDS
  double* st = sm;                                   // [rows][16][E]
  int* sgm = reinterpret_cast<int*>(sm + rows * 16 * E);   // [3 m][64]
  __shared__ int s_aj[kTabRows][2], s_gj[kTabRows][3];
  __shared__ double s_base[2 + kMaxSamples + 1 + 4 * kMaxSplit];
  if (na > rows || ng > 3 * m) {   // more table rows than the launch sized its LDS for (a guard)
    if (threadIdx.x == 0) S->stop = STOP_INTERNAL;
    return;
  }
  for (int e = threadIdx.x; e < na * 16 * E; e += blockDim.x) st[e] = G(P.tab)[(e / E) * kTabEntry + e % E];
  for (int e = threadIdx.x; e < ng * 64; e += blockDim.x) sgm[e] = G(P.tabi)[kTiGm + e];
  for (int e = threadIdx.x; e < 2 * na; e += blockDim.x) s_aj[e >> 1][e & 1] = G(P.tabi)[kTiAj + e];
  for (int e = threadIdx.x; e < 3 * ng; e += blockDim.x) s_gj[e / 3][e % 3] = G(P.tabi)[kTiGj + e];
  for (int e = threadIdx.x; e < 3 + kMaxSamples + 4 * kMaxSplit; e += blockDim.x) s_base[e] = G(P.tab)[kTabBase + e];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cu = (uint32_t)c;
  auto dig = [&](int j) { return j >= 0 ? (int)((cu >> (2 * j)) & 3u) : 0; };
  bool formed = c < P.nch;
  for (int j = 0; j < m; ++j)
    if (!((mask >> j) & 1u) && dig(j) != 0) formed = false;
  double ub = __builtin_inf();
  if (formed) {
    I F{s_base[0], s_base[1]};
    double u[kMaxSamples];
#pragma unroll
    for (int q = 0; q < kMaxSamples; ++q) u[q] = s_base[2 + q];
    for (int a = 0; a < na; ++a) {
      const int cb = dig(s_aj[a][0]) | (dig(s_aj[a][1]) << 2);
      const double* e = st + (a * 16 + cb) * E;
      F = add(F, I{e[0], e[1]});
#pragma unroll
      for (int q = 0; q < kMaxSamples; ++q)
        if (q < ns) u[q] = u[q] + e[2 + q];
    }
#pragma unroll
    for (int q = 0; q < kMaxSamples; ++q)
      if (q < ns) ub = dmin(ub, u[q]);
    ub = hi_or_inf(ub);
    bool mo = false;
    for (int k = 0; k < ng; ++k) mo = mo || sgm[64 * k + (dig(s_gj[k][0]) | (dig(s_gj[k][1]) << 2) | (dig(s_gj[k][2]) << 4))];
    double wm = s_base[2 + kMaxSamples];
    for (int j = 0; j < m; ++j)
      if ((mask >> j) & 1u) wm = dmax(wm, s_base[3 + kMaxSamples + 4 * j + dig(j)]);
    G(P.ch_flo)[c] = lo_or_ninf(neg(F.n));
    G(P.ch_wmax)[c] = wm;
    G(P.ch_flag)[c] = mo ? 1 : 2;
  } else if (c < P.nch) {
    G(P.ch_flag)[c] = 0;   // takes a piece of a coordinate that cannot be cut
  }
  // GUB: the block's smallest sample bound
  __shared__ double s_u[256 / kWave];
  __shared__ int s_n[256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  double um = ub;
  int cnt = formed ? 1 : 0;
  for (int h = 32; h >= 1; h >>= 1) {
    um = dmin(um, __shfl_xor(um, h, kWave));
    cnt += __shfl_xor(cnt, h, kWave);
  }
  if (lane == 0) { s_u[wid] = um; s_n[wid] = cnt; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mn = s_u[0];
    int tot = s_n[0];
    for (int k = 1; k < 256 / kWave; ++k) { mn = dmin(mn, s_u[k]); tot += s_n[k]; }
    if (tot > 0) {
      const unsigned long long key = okey(mn);
      if (key < __hip_atomic_load(&S->gub_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)&S->gub_key, key);
      atomicAdd((unsigned long long*)&S->ub_evaluated, (unsigned long long)tot);
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_select4(const Params* __restrict__ PP, State* __restrict__ S, int nparts,
                                                int host_stop) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  select_body<NT, 4>(P, S, nparts, host_stop);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_select(const Params* __restrict__ PP, State* __restrict__ S, int nparts,
                                               int host_stop) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  select_body<NT>(P, S, nparts, host_stop);
}

// ---------------------------------------------------------------------------
// K > 1 boxes per sweep: Sec. 3.1 selects the region with the smallest lower
// bound; a sweep here may take the K smallest (lower bound, insertion number)
// at once (K a fixed option: it changes the iteration, so it is never tuned).
// One workgroup inserts the previous sweep's survivors (records of K parents,
// parent-major), counts the live list and tests the stopping criteria as for
// K = 1, then finds the K-th smallest lower bound by a radix selection over the
// ordered 64-bit keys of the live boxes (8 bits per pass from the top; a pass
// whose boundary bin is taken whole ends it), takes every box below that bound
// and, among boxes equal to it, the first ones in list order (list order is
// insertion order), ranks the at most K candidates by (lower bound, list
// index), and writes one row per selected box: box p of sweep t gets row
// 1 + t K + p, its cycling index, split points and split mask, and an entry in
// the selection table.
template <int NT>
struct KSelLds {
  int hist[256];
  int wtot[NT / kWave];
  int bin, below, ncand;
  double cf[kMaxSelectK];      // candidates, unordered
  int32_t ci[kMaxSelectK];
  int32_t si[kMaxSelectK];     // list index by rank
  int32_t sref[kMaxSelectK], sr[kMaxSelectK];   // parent row and child index by rank
};

template <int NT>
__device__ __forceinline__ int ksel_count_prefix(int v, KSelLds<NT>& L, int& total) {
  // exclusive prefix over the workgroup of one int per thread (thread order)
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  int incl = v;
  for (int h = 1; h < kWave; h <<= 1) {
    const int o = __shfl_up(incl, h, kWave);
    if (lane >= h) incl += o;
  }
  if (lane == kWave - 1) L.wtot[wid] = incl;
  __syncthreads();
  int before = 0;
  total = 0;
  for (int k = 0; k < NT / kWave; ++k) {
    const int t = L.wtot[k];
    before += k < wid ? t : 0;
    total += t;
  }
  __syncthreads();   // L.wtot is written again by the next call
  return before + incl - v;
}

// The end of a K > 1 selection, in one workgroup: rank the (at most K)
// candidates in L by (lower bound, list index) and write one row per selected box
// (rank p of sweep t: row 1 + t K + p), its table entry, and remove its key.
template <int NT>
__device__ void ksel_finish(const Params& P, State* S, KSelLds<NT>& L, int64_t t, double gub) {
  const int K = P.select_k;
  const int nc = min(L.ncand, K);
  // rank the candidates by (lower bound, list index)
  for (int q = threadIdx.x; q < nc; q += NT) {
    const double fq = L.cf[q];
    const int32_t iq = L.ci[q];
    int rank = 0;
    for (int j = 0; j < nc; ++j) {
      const double fj = L.cf[j];
      rank += (fj < fq || (fj == fq && L.ci[j] < iq)) ? 1 : 0;
    }
    L.si[rank] = iq;
  }
  __syncthreads();
  // per selected box (one wavefront each): remove its key, its cycling index,
  // split points and mask, its table entry
  const int n = P.n, lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
  for (int pr = wid; pr < nc; pr += NT / kWave) {
    const int32_t idx = L.si[pr];
    const int32_t ref = P.key_ref[idx];
    const int32_t r = P.key_r[idx];
    const int64_t seq = P.key_seq[idx];
    const int pcyc = P.hist_cyc[ref];
    const ChildRow src{P.hist_n + (int64_t)ref * n, P.hist_h + (int64_t)ref * n, P.hist_mid + (int64_t)ref * kMaxSplit,
                       n, P.m, pcyc, r >= 0 ? P.hist_mask[ref] : 0u, r >= 0 ? (uint32_t)r : 0u};
    const int cyc = r >= 0 ? add_mod(pcyc, P.m, n) : pcyc;
    const int64_t row = 1 + t * K + pr;
    bool ok = false;
    if (lane < P.m) {
      const I x = src.get(add_mod(cyc, lane, n));
      const double md = midpoint(x);
      ok = neg(x.n) < md && md < x.h;
      P.hist_mid[row * kMaxSplit + lane] = md;
    }
    const uint32_t mask = (uint32_t)__ballot(ok) & ((1u << P.m) - 1u);   // m <= 16
    if (lane == 0) {
      P.hist_mask[row] = mask;
      P.hist_cyc[row] = cyc;
      P.sel_tab[pr] = SelRec{seq, (int32_t)row, cyc, mask, 0u};
      P.key_flo[idx] = __builtin_inf();   // removed from the list
      L.sref[pr] = ref;
      L.sr[pr] = r;
      if (pr == 0) S->sel_seq = seq;
    }
  }
  __syncthreads();
  // the selected boxes' real endpoints, row by row
  for (int pr = 0; pr < nc; ++pr) {
    const int32_t ref = L.sref[pr], r = L.sr[pr];
    const ChildRow src{P.hist_n + (int64_t)ref * n, P.hist_h + (int64_t)ref * n, P.hist_mid + (int64_t)ref * kMaxSplit,
                       n, P.m, P.hist_cyc[ref], r >= 0 ? P.hist_mask[ref] : 0u, r >= 0 ? (uint32_t)r : 0u};
    const int64_t row = 1 + t * K + pr;
    (void)build_row<NT>(src, P.hist_n + row * n, P.hist_h + row * n, n, 0, 0);
  }
  if (threadIdx.x == 0) {
    S->sel_count = nc;
    S->gub_start = gub;
    S->pending = 1;
  }
}

template <int NT>
__device__ bool select_k_body(const Params& P, State* S, int host_stop, KSelLds<NT>& L) {
  const double gub = okey_inv(S->gub_key);
  SelAcc ins = sel_empty();
  if (S->pending) insert_children<NT>(P, S, gub, ins);   // ends with a barrier
  const int64_t nk = S->n_keys;
  const int K = P.select_k;
  const bool need_w = P.tol_x > 0.0;
  // live count, GLB and widest box over the whole list
  SelAcc a = sel_empty();
  for (int64_t i = threadIdx.x; i < nk; i += NT) {
    const double f = P.key_flo[i];
    if (!(f <= gub)) continue;
    a.cnt++;
    if (need_w) a.wm = dmax(a.wm, P.key_wmax[i]);
    if (f < a.best.f) a.best = Cand{f, i};
  }
  a = sel_block_reduce<NT>(a);
  __shared__ int32_t go;
  const int64_t t = S->sweeps;
  if (threadIdx.x == 0) {
    if (t > 0 && t - 1 < P.trace_cap) P.tr_nlive[t - 1] = a.cnt;
    S->n_live = a.cnt;
    S->glb = a.best.f;
    S->wmax = a.wm;
    int32_t stop = RUNNING;
    if (host_stop) stop = STOP_HOST;
    else if (a.cnt == 0) stop = STOP_EMPTY;
    else if (gub - a.best.f <= P.tol_f && (P.tol_x <= 0.0 || a.wm < P.tol_x)) stop = STOP_CONVERGED;
    else if (t >= P.max_sweeps) stop = STOP_SWEEPS;
    else if (P.max_live > 0 && a.cnt > P.max_live) stop = STOP_LIVE;
    else if ((t + 1) * K >= P.hist_cap || nk + (int64_t)K * P.nch > P.key_cap) stop = STOP_CAPACITY;
    if (stop) S->stop = stop;
    go = stop == RUNNING;
    L.ncand = 0;
  }
  __syncthreads();
  if (!go) return false;

  // radix selection of the K-th smallest ordered key among the live boxes
  uint64_t prefix = 0;
  int need = K, shift = 64;
  bool whole = a.cnt <= K;   // every live box is taken
  if (!whole) {
    for (shift = 56; shift >= 0; shift -= 8) {
      for (int b = threadIdx.x; b < 256; b += NT) L.hist[b] = 0;
      if (threadIdx.x == 0) { L.bin = 0; L.below = 0; }
      __syncthreads();
      const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
      for (int64_t i = threadIdx.x; i < nk; i += NT) {
        const double f = P.key_flo[i];
        if (!(f <= gub)) continue;
        const uint64_t u = skey(f);
        if ((u & hmask) == (prefix & hmask)) atomicAdd(&L.hist[(int)((u >> shift) & 255u)], 1);
      }
      __syncthreads();
      if (threadIdx.x < (unsigned)kWave) {   // the bin where the count below reaches `need`
        const int lane = threadIdx.x;
        const int h0 = L.hist[4 * lane], h1 = L.hist[4 * lane + 1], h2 = L.hist[4 * lane + 2], h3 = L.hist[4 * lane + 3];
        const int sum = h0 + h1 + h2 + h3;
        int incl = sum;
        for (int h = 1; h < kWave; h <<= 1) {
          const int o = __shfl_up(incl, h, kWave);
          if (lane >= h) incl += o;
        }
        const int excl = incl - sum;
        if (excl < need && need <= incl) {
          int below = excl, b = 4 * lane;
          const int hs[4] = {h0, h1, h2, h3};
          for (int q = 0; q < 4; ++q) {
            if (below + hs[q] >= need) { b = 4 * lane + q; break; }
            below += hs[q];
          }
          L.bin = b;
          L.below = below;
        }
      }
      __syncthreads();
      const int b = L.bin & 255, inbin = L.hist[b];
      prefix |= (uint64_t)b << shift;
      need -= L.below;
      __syncthreads();   // every thread has read the bin before the histogram is cleared
      if (inbin == need) { whole = true; break; }
    }
    if (!whole) shift = 0;   // all 64 bits fixed: prefix is the K-th smallest key itself
  }
  // take, in list order: every live key below the bound and, when the bound is a
  // single key value, the first `need` keys equal to it
  const uint64_t top = shift >= 64 ? 0ull : (prefix >> shift);
  int eqbase = 0;   // keys equal to the bound in earlier chunks (every thread keeps the same count)
  for (int64_t c0 = 0; c0 < nk; c0 += NT) {
    const int64_t i = c0 + threadIdx.x;
    bool take = false, eq = false;
    double f = 0.0;
    if (i < nk) {
      f = P.key_flo[i];
      if (f <= gub) {
        const uint64_t u = skey(f);
        if (whole) take = shift >= 64 || (u >> shift) <= top;
        else {
          take = u < prefix;
          eq = u == prefix;
        }
      }
    }
    if (!whole) {
      int tot = 0;
      const int rank = ksel_count_prefix<NT>(eq ? 1 : 0, L, tot);
      if (eq && eqbase + rank < need) take = true;
      eqbase += tot;
    }
    if (take) {
      const int slot = atomicAdd(&L.ncand, 1);
      if (slot < kMaxSelectK) {
        L.cf[slot] = f;
        L.ci[slot] = (int32_t)i;
      }
    }
  }
  __syncthreads();
  ksel_finish<NT>(P, S, L, t, gub);
  return true;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_select_k(const Params* __restrict__ PP, State* __restrict__ S, int host_stop) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  __shared__ KSelLds<NT> lds;
  select_k_body<NT>(P, S, host_stop, lds);
}

// K > 1 on long lists: the same selection in several launches, so that every
// pass over the list runs on many workgroups (one workgroup reads a list of
// millions of keys at a small fraction of HBM bandwidth):
//   k_select_part    partial live count / GLB / widest side of the list
//   k_ksel_begin     one workgroup: insert the previous records, the stop test,
//                    the first digit (the bits every live key shares are skipped)
//   k_ksel_hist x8   histogram of the current 8-bit digit of the keys that match
//                    the bits fixed so far; the last workgroup to finish picks the
//                    digit (the bin where the count below reaches the boxes still
//                    needed) and clears the histogram for the next launch
//   k_ksel_take      gather every live key below the bound (at most K)
//   k_ksel_rows      one workgroup: the keys equal to the bound in list order when
//                    the bound is one value with ties, then the ranking and rows
// The selected set is the one the one-workgroup kernel takes.
template <int NT>
__global__ __launch_bounds__(NT) void k_ksel_begin(const Params* __restrict__ PP, State* __restrict__ S, int nparts) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  const double gub = okey_inv(S->gub_key);
  const int32_t pending = S->pending;   // read by every thread before any barrier
  SelAcc a = sel_empty();
  for (int k = threadIdx.x; k < nparts; k += NT) {
    const SelAcc o{Cand{P.part_flo[k], P.part_idx[k]}, P.part_wmax[k], P.part_cnt[k]};
    a = sel_merge(a, o);
  }
  a = sel_block_reduce<NT>(a);
  if (pending) insert_children<NT>(P, S, gub, a);   // adds the inserted keys to a; ends with a barrier
  __shared__ int32_t go;
  const int64_t t = S->sweeps;
  const int64_t nk = S->n_keys;
  const int K = P.select_k;
  if (threadIdx.x == 0) {
    if (t > 0 && t - 1 < P.trace_cap) P.tr_nlive[t - 1] = a.cnt;
    S->n_live = a.cnt;
    S->glb = a.best.f;
    S->wmax = a.wm;
    int32_t stop = RUNNING;
    if (a.cnt == 0) stop = STOP_EMPTY;
    else if (gub - a.best.f <= P.tol_f && (P.tol_x <= 0.0 || a.wm < P.tol_x)) stop = STOP_CONVERGED;
    else if (t >= P.max_sweeps) stop = STOP_SWEEPS;
    else if (P.max_live > 0 && a.cnt > P.max_live) stop = STOP_LIVE;
    else if ((t + 1) * K >= P.hist_cap || nk + (int64_t)K * P.nch > P.key_cap) stop = STOP_CAPACITY;
    if (stop) S->stop = stop;
    go = stop == RUNNING;
    if (go) {
      S->ks_need = K;
      S->ks_whole = 0;
      S->ks_done = 0;
      if (a.cnt <= K) {   // every live box is taken
        S->ks_done = 1;
        S->ks_whole = 1;
        S->ks_shift = 64;
        S->ks_prefix = 0ull;
      } else {
        // every live key lies in [skey(GLB), skey(GUB)]: the bits above the first
        // one where those two differ are the same for all of them
        const uint64_t lo = skey(a.best.f), hi = skey(gub);
        const int lead = lo == hi ? 64 : __clzll((long long)(lo ^ hi));
        const int sh = lead >= 64 ? 0 : ((63 - lead) >> 3) << 3;
        S->ks_shift = sh;
        S->ks_prefix = sh >= 56 ? 0ull : (lo & (~0ull << (sh + 8)));
      }
      P.ksel->ticket = 0u;
      P.ksel->ncand = 0u;
    }
  }
  __syncthreads();
  if (go)
    for (int b = threadIdx.x; b < 256; b += NT) P.ksel->hist[b] = 0u;
}

__global__ __launch_bounds__(kSelThreads) void k_ksel_hist(const Params* __restrict__ PP, State* __restrict__ S) {
  // S->stop and S->ks_done change only between launches: the same for every workgroup
  if (S->stop || S->ks_done) return;
  const Params P = *PP;
  KselBuf* B = P.ksel;
  __shared__ uint32_t h[256];
  __shared__ int last;
  for (int b = threadIdx.x; b < 256; b += kSelThreads) h[b] = 0u;
  __syncthreads();
  const double gub = okey_inv(S->gub_key);
  const int shift = S->ks_shift;
  const uint64_t prefix = S->ks_prefix;
  const uint64_t hmask = shift >= 56 ? 0ull : (~0ull << (shift + 8));
  const int64_t nk = S->n_keys;
  const int64_t stride = (int64_t)gridDim.x * kSelThreads;
  for (int64_t i = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; i < nk; i += stride) {
    const double f = P.key_flo[i];
    if (!(f <= gub)) continue;
    const uint64_t u = skey(f);
    if ((u & hmask) == prefix) atomicAdd(&h[(int)((u >> shift) & 255u)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 256; b += kSelThreads)
    if (h[b]) atomicAdd(&B->hist[b], h[b]);
  __threadfence();   // this workgroup's counts are visible before its ticket
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&B->ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last || threadIdx.x >= kWave) return;
  __threadfence();
  // the last workgroup: the bin where the count below reaches the boxes still needed
  const int lane = threadIdx.x;
  int hs[4];
  for (int q = 0; q < 4; ++q) hs[q] = (int)__hip_atomic_load(&B->hist[4 * lane + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int need = S->ks_need;
  const int sum = hs[0] + hs[1] + hs[2] + hs[3];
  int incl = sum;
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  const int excl = incl - sum;
  if (excl < need && need <= incl) {   // one lane
    int below = excl, b = 4 * lane;
    for (int q = 0; q < 4; ++q) {
      if (below + hs[q] >= need) { b = 4 * lane + q; break; }
      below += hs[q];
    }
    const int inbin = hs[b - 4 * lane];
    const int left = need - below;
    S->ks_prefix = prefix | ((uint64_t)b << shift);
    S->ks_need = left;
    if (inbin == left) {           // the whole bin is taken: the bound is settled
      S->ks_done = 1;
      S->ks_whole = 1;
    } else if (shift == 0) {       // one key value with more keys than needed: ties
      S->ks_done = 1;
      S->ks_whole = 0;
    } else {
      S->ks_shift = shift - 8;
    }
  }
  for (int q = 0; q < 4; ++q) B->hist[4 * lane + q] = 0u;
  if (lane == 0) B->ticket = 0u;
}

__global__ __launch_bounds__(kSelThreads) void k_ksel_take(const Params* __restrict__ PP, State* __restrict__ S) {
  if (S->stop) return;
  const Params P = *PP;
  KselBuf* B = P.ksel;
  const double gub = okey_inv(S->gub_key);
  const int shift = S->ks_shift;
  const uint64_t prefix = S->ks_prefix;
  const bool whole = S->ks_whole != 0;
  const uint64_t top = shift >= 64 ? 0ull : (prefix >> shift);
  const int64_t nk = S->n_keys;
  const int64_t stride = (int64_t)gridDim.x * kSelThreads;
  for (int64_t i = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; i < nk; i += stride) {
    const double f = P.key_flo[i];
    if (!(f <= gub)) continue;
    const uint64_t u = skey(f);
    const bool take = whole ? (shift >= 64 || (u >> shift) <= top) : u < prefix;
    if (take) {
      const uint32_t slot = atomicAdd(&B->ncand, 1u);
      if (slot < (uint32_t)kMaxSelectK) {
        B->cf[slot] = f;
        B->ci[slot] = (int32_t)i;
      }
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_ksel_rows(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  const Params P = *PP;
  __shared__ KSelLds<NT> L;
  const double gub = okey_inv(S->gub_key);
  const int K = P.select_k;
  const KselBuf* B = P.ksel;
  if (threadIdx.x == 0) L.ncand = (int)min(B->ncand, (uint32_t)K);
  __syncthreads();
  const int nb = L.ncand;
  for (int q = threadIdx.x; q < nb; q += NT) {
    L.cf[q] = B->cf[q];
    L.ci[q] = B->ci[q];
  }
  if (!S->ks_whole) {
    // the bound is one key value: the first `need` keys equal to it, in list order
    const uint64_t prefix = S->ks_prefix;
    const int need = S->ks_need;
    const int64_t nk = S->n_keys;
    int eqbase = 0;   // keys equal to the bound in earlier chunks (every thread keeps the same count)
    for (int64_t c0 = 0; c0 < nk && eqbase < need; c0 += NT) {
      const int64_t i = c0 + threadIdx.x;
      bool eq = false;
      double f = 0.0;
      if (i < nk) {
        f = P.key_flo[i];
        eq = f <= gub && skey(f) == prefix;
      }
      int tot = 0;
      const int rank = ksel_count_prefix<NT>(eq ? 1 : 0, L, tot);
      if (eq && eqbase + rank < need) {
        const int slot = atomicAdd(&L.ncand, 1);
        if (slot < kMaxSelectK) {
          L.cf[slot] = f;
          L.ci[slot] = (int32_t)i;
        }
      }
      eqbase += tot;
    }
  }
  __syncthreads();
  ksel_finish<NT>(P, S, L, S->sweeps, gub);
}

// Bound the children of the selected box.
//
// W "box" wavefronts share one child: in round rd, wave w computes the terms of
// coordinate chunk rd*W + w (64 coordinates, one per lane) and parks them in
// LDS; wave 0 adds the W chunks to its slot sums in chunk order, so slot s
// still sums t_s, t_{s+64}, t_{s+128}, ... left to right and the bound is the
// same bit for bit whatever W is.
//
// CONC = 1 (latency mode, few children): W more wavefronts per child compute
// the midpoint upper bound at the same time, for every formed child.
// CONC = 0 (throughput mode): the same wavefronts compute the midpoint bound
// afterwards, and only when F.lo does not exceed the running GUB (a child whose
// lower bound exceeds GUB cannot lower it).  Both give the same GUB.
template <int FAM, int W, int CONC>
__device__ void bound_body(const Params& P, State* S, int cbase) {
  constexpr int WPC = CONC ? 2 * W : W;     // wavefronts per child
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int local = wid / WPC, role_w = wid % WPC;
  const bool mid_role = CONC && role_w >= W;
  const int w = role_w % W;
  const int first = local * WPC + (mid_role ? W : 0);   // wave slot of this role's wave 0
  // record g: child c of the selected box (K > 1: child c = g mod nch of the box
  // of rank g / nch, taken from the sweep's selection table)
  const int g = cbase + local;
  int row, cyc, c;
  uint32_t mask;
  bool in;   // a record of this sweep
  if (P.select_k > 1) {
    const int pr = g >> P.m;
    in = g < P.select_k * P.nch && pr < S->sel_count;
    const SelRec sr = P.sel_tab[in ? pr : 0];
    row = sr.row;
    cyc = sr.cyc;
    mask = sr.mask;
    c = g & (P.nch - 1);
  } else {
    in = g < P.nch;
    row = S->sel_row;
    cyc = S->sel_cyc;
    mask = S->sel_mask;
    c = g;
  }
  const bool formed = in && (((uint32_t)c & ~mask) == 0u);
  const ChildRow X{P.hist_n + (int64_t)row * P.n, P.hist_h + (int64_t)row * P.n, P.hist_mid + (int64_t)row * kMaxSplit,
                   P.n, P.m, cyc, mask, (uint32_t)(in ? c : 0)};
  const int n = P.n;
  const int rounds = ((n + kWave - 1) / kWave + W - 1) / W;
  __shared__ double ln[kBoundWaves][kWave], lh[kBoundWaves][kWave];
  __shared__ int s_flag[kBoundWaves];
  __shared__ double s_wm[kBoundWaves];
  // the children's midpoint bounds meet here: one GUB update per workgroup, and
  // only when its minimum is below GUB (atomics from every child on the one
  // address serialise in L2)
  __shared__ unsigned long long s_ukey[kBoundWaves];
  __shared__ int s_ucnt[kBoundWaves];
  if (lane == 0) {
    s_ukey[wid] = ~0ull;
    s_ucnt[wid] = 0;
  }

  // ---- pass 0 (FP32 filter, throughput mode only): a single-precision lower
  // bound over the FP32-enclosing box and the first-order test.  r32 = 2: the
  // bound exceeds the GUB at the start of the sweep (no FP64 work at all);
  // r32 = 1: the first-order test discards the child (FP64 midpoint bound only);
  // r32 = 0: bound the child in FP64 as usual.
  int r32 = 0;
  if (!CONC && P.prec32 && S->use32) {
    // same canonical order as the FP64 sum (slot = lane, rounds left to right,
    // then the wave fold), so the filter's decisions do not depend on W
    __shared__ float l32n[kBoundWaves][kWave], l32h[kBoundWaves][kWave];
    __shared__ int s_r32[kBoundWaves];
    J a32{0.0f, 0.0f};
    bool m32 = false;
    for (int rd = 0; rd < rounds; ++rd) {
      const int i = (rd * W + w) * kWave + lane;
      J t{0.0f, 0.0f};
      if (formed && i < n) filter32_coord<FAM>(P, X, i, t, m32);
      if (W == 1) {
        a32 = add32(a32, t);
      } else {
        l32n[wid][lane] = t.n;
        l32h[wid][lane] = t.h;
        __syncthreads();
        if (w == 0)
          for (int k = 0; k < W; ++k) a32 = add32(a32, J{l32n[first + k][lane], l32h[first + k][lane]});
        __syncthreads();
      }
    }
    const bool any32 = __any(m32);
    if (W == 1) {
      const J F32 = fold32(a32, lane);
      if (formed) r32 = ((double)neg32(F32.n) > S->gub_start) ? 2 : (any32 ? 1 : 0);
    } else {
      if (lane == 0) s_flag[wid] = any32;
      __syncthreads();
      if (w == 0) {
        const J F32 = fold32(a32, lane);
        bool any = false;
        for (int k = 0; k < W; ++k) any = any || s_flag[first + k];
        if (lane == 0) s_r32[local] = formed ? (((double)neg32(F32.n) > S->gub_start) ? 2 : (any ? 1 : 0)) : 0;
      }
      __syncthreads();
      r32 = s_r32[local];
    }
  }
  const bool run64 = formed && r32 == 0;

  I acc{0.0, 0.0};
  double hacc = 0.0;
  bool mo = false;
  double wm = 0.0;
  // ---- pass 1: F, first-order test, widest side (box waves); midpoint bound (mid waves) ----
  for (int rd = 0; rd < rounds; ++rd) {
    const int i = (rd * W + w) * kWave + lane;
    I t{0.0, 0.0};
    if ((mid_role ? formed : run64) && i < n) {
      if (mid_role) {
        if (FAM != FAM_CHAIN) t.h = sep_point_hi<FAM>(P.sep[i], midpoint(X.get(i)));
        else if (i + 1 < n) {
          I R, E;
          t.h = chain_term(P.chain[i], point(midpoint(X.get(i))), point(midpoint(X.get(i + 1))), R, E).h;
        }
      } else if (FAM != FAM_CHAIN) {
        const I x = X.get(i);
        I G;
        sep_box<FAM>(P.sep[i], x, t, G);
        mo |= (G.n < 0.0 && x.n != P.nl[i]) || (G.h < 0.0 && x.h != P.u[i]);
        wm = dmax(wm, x.n + x.h);
      } else {
        const I xi = X.get(i);
        const bool has_prev = i > 0, has_next = i + 1 < n;
        const I xp = has_prev ? X.get(i - 1) : xi;
        const I xn = has_next ? X.get(i + 1) : xi;
        if (has_next) {
          I R, E;
          t = chain_term(P.chain[i], xi, xn, R, E);
        }
        const I G = chain_grad(P.chain[has_prev ? i - 1 : i], P.chain[i], xp, xi, xn, has_prev, has_next);
        mo |= (G.n < 0.0 && xi.n != P.nl[i]) || (G.h < 0.0 && xi.h != P.u[i]);
        wm = dmax(wm, xi.n + xi.h);
      }
    }
    if (WPC == 1) {
      acc = add(acc, t);
    } else {
      ln[wid][lane] = t.n;
      lh[wid][lane] = t.h;
      __syncthreads();
      if (w == 0) {
        if (mid_role)
          for (int k = 0; k < W; ++k) hacc = hacc + lh[first + k][lane];
        else
          for (int k = 0; k < W; ++k) acc = add(acc, I{ln[first + k][lane], lh[first + k][lane]});
      }
      __syncthreads();
    }
  }
  const bool any_mo = __any(mo);
  const double wmx = wave_max(wm);
  if (W > 1) {
    if (lane == 0) { s_flag[wid] = any_mo; s_wm[wid] = wmx; }
    __syncthreads();
  }
  double flo = 0.0, cwm = wmx;
  bool cmo = any_mo;
  if (!mid_role && w == 0) {
    const I F = fold_slots(acc, lane);
    flo = lo_or_ninf(neg(F.n));
    for (int k = 1; k < W; ++k) { cmo = cmo || s_flag[first + k]; cwm = dmax(cwm, s_wm[first + k]); }
  }

  if (!CONC) {
    // ---- pass 2 (throughput mode): midpoint bound unless F.lo exceeds the running GUB ----
    bool do_ub;
    if (W > 1) {
      __syncthreads();
      if (w == 0 && lane == 0) {
        const double gcur = okey_inv(__hip_atomic_load(&S->gub_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        s_flag[local] = formed && (r32 == 1 || (r32 == 0 && !(flo > gcur)));
      }
      __syncthreads();
      do_ub = s_flag[local] != 0;
    } else {
      const double gcur = okey_inv(__hip_atomic_load(&S->gub_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      do_ub = formed && (r32 == 1 || (r32 == 0 && !(flo > gcur)));
    }
    for (int rd = 0; rd < rounds; ++rd) {
      const int i = (rd * W + w) * kWave + lane;
      double th = 0.0;
      if (do_ub && i < n) {
        if (FAM != FAM_CHAIN) {
          th = sep_point_hi<FAM>(P.sep[i], midpoint(X.get(i)));
        } else if (i + 1 < n) {
          I R, E;
          th = chain_term(P.chain[i], point(midpoint(X.get(i))), point(midpoint(X.get(i + 1))), R, E).h;
        }
      }
      if (W == 1) {
        hacc = hacc + th;
      } else {
        lh[wid][lane] = th;
        __syncthreads();
        if (w == 0)
          for (int k = 0; k < W; ++k) hacc = hacc + lh[local * W + k][lane];
        __syncthreads();
      }
    }
    if (w == 0) {
      const double u = fold_slots_hi(hacc, lane);
      if (lane == 0 && in) {
        if (formed) {
          if (do_ub) {
            s_ukey[wid] = okey(hi_or_inf(u));
            s_ucnt[wid] = 1;
          }
          if (r32) {
            P.ch_flag[g] = 3;
          } else {
            P.ch_flo[g] = flo;
            P.ch_flag[g] = cmo ? 1 : 2;
            P.ch_wmax[g] = cwm;
          }
        } else {
          P.ch_flag[g] = 0;   // takes the upper half of a coordinate that cannot be split
        }
      }
    }
  } else if (w == 0) {
    if (mid_role) {
      const double u = fold_slots_hi(hacc, lane);
      if (lane == 0 && formed) {
        s_ukey[wid] = okey(hi_or_inf(u));
        s_ucnt[wid] = 1;
      }
    } else if (lane == 0 && in) {
      if (formed) {
        P.ch_flo[g] = flo;
        P.ch_flag[g] = cmo ? 1 : 2;
        P.ch_wmax[g] = cwm;
      } else {
        P.ch_flag[g] = 0;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mn = s_ukey[0];
    int cnt = s_ucnt[0];
    for (int k = 1; k < kBoundWaves; ++k) {
      mn = s_ukey[k] < mn ? s_ukey[k] : mn;
      cnt += s_ucnt[k];
    }
    if (cnt > 0) {
      if (mn < __hip_atomic_load(&S->gub_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)&S->gub_key, mn);
      atomicAdd((unsigned long long*)&S->ub_evaluated, (unsigned long long)cnt);
    }
  }
}

template <int FAM, int W, int CONC>
__global__ __launch_bounds__(kWave* kBoundWaves) void k_bound(const Params* __restrict__ PP, State* __restrict__ S) {
  round_up_mode();
  if (S->stop) return;
  constexpr int CPB = kBoundWaves / (CONC ? 2 * W : W);   // children per workgroup
  const Params P = *PP;
  bound_body<FAM, W, CONC>(P, S, blockIdx.x * CPB);
}

// count live keys (lower bound <= GUB) and the smallest lower bound
__global__ __launch_bounds__(kSelThreads) void k_count_live(const Params* __restrict__ PP, State* __restrict__ S,
                                                            int64_t* __restrict__ flags) {
  const Params P = *PP;
  const double gub = okey_inv(S->gub_key);
  const int64_t nk = S->n_keys;
  for (int64_t i = (int64_t)blockIdx.x * kSelThreads + threadIdx.x; i < nk; i += (int64_t)gridDim.x * kSelThreads)
    flags[i] = P.key_flo[i] <= gub ? 1 : 0;
}

// stable compaction, pass 1: per-block counts
__global__ __launch_bounds__(256) void k_compact_count(const int64_t* __restrict__ flags, int64_t nk, int64_t per_block,
                                                       int64_t* __restrict__ block_cnt) {
  __shared__ int64_t s[256];
  const int64_t b0 = (int64_t)blockIdx.x * per_block, b1 = (b0 + per_block < nk) ? b0 + per_block : nk;
  int64_t c = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) c += flags[i];
  s[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (threadIdx.x < (unsigned)h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = s[0];
}

// pass 2: scatter kept keys in order (one block per segment, sequential within a segment)
__global__ __launch_bounds__(256) void k_compact_scatter(const Params* __restrict__ PP, const int64_t* __restrict__ flags,
                                                         int64_t nk, int64_t per_block,
                                                         const int64_t* __restrict__ block_cnt, int nblocks,
                                                         double* __restrict__ o_flo, int64_t* __restrict__ o_seq,
                                                         int32_t* __restrict__ o_ref, int32_t* __restrict__ o_r,
                                                         double* __restrict__ o_wmax) {
  const Params P = *PP;
  __shared__ int64_t base;
  __shared__ int64_t s[256];
  if (threadIdx.x == 0) {
    int64_t b = 0;
    for (int k = 0; k < (int)blockIdx.x; ++k) b += block_cnt[k];
    base = b;
  }
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * per_block, b1 = (b0 + per_block < nk) ? b0 + per_block : nk;
  for (int64_t chunk = b0; chunk < b1; chunk += 256) {
    const int64_t i = chunk + threadIdx.x;
    const int64_t f = i < b1 ? flags[i] : 0;
    s[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int64_t v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) {
      const int64_t o = base + s[threadIdx.x] - 1;
      o_flo[o] = P.key_flo[i];
      o_seq[o] = P.key_seq[i];
      o_ref[o] = P.key_ref[i];
      o_r[o] = P.key_r[i];
      o_wmax[o] = P.key_wmax[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) base += s[255];
    __syncthreads();
  }
}

// real endpoints of boxes given as (row, child index)
__global__ __launch_bounds__(256) void k_rows_out(const Params* __restrict__ PP, int64_t nb, const int32_t* __restrict__ ref,
                                                  const int32_t* __restrict__ rr, double* __restrict__ lo,
                                                  double* __restrict__ hi) {
  round_up_mode();
  const Params P = *PP;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int32_t row = ref[b], r = rr[b];
    const uint32_t mask = r >= 0 ? P.hist_mask[row] : 0u, rc = r >= 0 ? (uint32_t)r : 0u;
    if (P.pieces == 4) {
      const ChildRow4 X{P.hist_n + (int64_t)row * P.n, P.hist_h + (int64_t)row * P.n,
                        P.hist_cut + (int64_t)row * (3 * kMaxSplit), P.n, P.m, P.hist_cyc[row], mask, rc};
      for (int i = threadIdx.x; i < P.n; i += 256) {
        const I x = X.get(i);
        lo[b * P.n + i] = neg(x.n);
        hi[b * P.n + i] = x.h;
      }
    } else {
      const ChildRow X{P.hist_n + (int64_t)row * P.n, P.hist_h + (int64_t)row * P.n,
                       P.hist_mid + (int64_t)row * kMaxSplit, P.n, P.m, P.hist_cyc[row], mask, rc};
      for (int i = threadIdx.x; i < P.n; i += 256) {
        const I x = X.get(i);
        lo[b * P.n + i] = neg(x.n);
        hi[b * P.n + i] = x.h;
      }
    }
  }
}

// elementwise interval operations (tests)
__global__ void k_interval_op(int op, int64_t cnt, const double* __restrict__ a, const double* __restrict__ b,
                              double* __restrict__ out) {
  round_up_mode();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const I x{neg(a[2 * i]), a[2 * i + 1]};
  const I y = b ? I{neg(b[2 * i]), b[2 * i + 1]} : I{0.0, 0.0};
  I r;
  switch (op) {
    case 0: r = add(x, y); break;
    case 1: r = sub(x, y); break;
    case 2: r = mul(x, y); break;
    case 3: r = div(x, y); break;
    case 4: r = isqrt(x); break;
    case 5: r = sqr(x); break;
    case 6: r = iabs(x); break;
    case 7: r = recip(x); break;
    case 8: r = sincos2pi(x, true, false).c; break;
    case 9: r = sincos2pi(x, false, true).s; break;
    case 10: r = dabs(x); break;
    case 11: r = iexp(x); break;
    case 12: r = sincos2pi(mul(x, inv_two_pi()), true, false).c; break;
    default: r = sincos2pi(mul(x, inv_two_pi()), false, true).s; break;
  }
  if (__builtin_isnan(r.n) || __builtin_isnan(r.h)) r = entire();
  out[2 * i] = neg(r.n);
  out[2 * i + 1] = r.h;
}

__global__ void k_interval_op32(int op, int64_t cnt, const float* __restrict__ a, const float* __restrict__ b,
                                float* __restrict__ out) {
  round_up_mode();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const J x{neg32(a[2 * i]), a[2 * i + 1]};
  const J y = b ? J{neg32(b[2 * i]), b[2 * i + 1]} : J{0.0f, 0.0f};
  J r;
  switch (op) {
    case 0: r = add32(x, y); break;
    case 1: r = sub32(x, y); break;
    case 2: r = mul32(x, y); break;
    case 5: r = sqr32(x); break;
    case 6: r = abs32(x); break;
    case 8: r = sincos2pi32(x, true, false).c; break;
    case 9: r = sincos2pi32(x, false, true).s; break;
    default: r = dabs32(x); break;
  }
  out[2 * i] = neg32(r.n);
  out[2 * i + 1] = r.h;
}

__global__ void k_point_trig32(int fn, int64_t cnt, const float* __restrict__ y, float* __restrict__ out) {
  round_up_mode();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const TrigEnc32 e = sincos2pi_point32(y[i]);
  const J r = fn == 0 ? e.c : e.s;
  out[2 * i] = neg32(r.n);
  out[2 * i + 1] = r.h;
}

__global__ void k_point_trig(int fn, int64_t cnt, const double* __restrict__ y, double* __restrict__ out) {
  round_up_mode();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const TrigEnc e = sincos2pi_point(y[i]);
  const I r = fn == 0 ? e.c : e.s;
  out[2 * i] = neg(r.n);
  out[2 * i + 1] = r.h;
}

// ===========================================================================
// host side
// ===========================================================================

namespace {

thread_local std::string g_err;

// Held while a graph is being captured (batched solves) and while results are
// read back or freed: HIP refuses some operations in one thread while another
// thread captures.
std::mutex g_capture_mu;

ibb_status fail(ibb_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail(IBB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// device memory through the caller's allocator, or stream-ordered hipMallocAsync
// Device memory of one result or engine.  Small requests are carved from slabs
// (one allocator call per slab, 256-byte aligned pieces); a carved piece is
// given back with its slab when everything is released.
struct Mem {
  static constexpr size_t kSlabBytes = (size_t)1 << 20, kCarveMax = (size_t)1 << 18;
  ibb_allocator alloc{};
  bool have_alloc = false;
  hipStream_t stream = nullptr;
  struct Blk {
    void* p;
    size_t bytes;
    bool slab;
  };
  std::vector<Blk> blocks;
  char* slab = nullptr;
  size_t slab_used = 0;

  void* raw(size_t bytes, bool is_slab) {
    void* p = nullptr;
    if (have_alloc) {
      p = alloc.alloc(alloc.ctx, bytes, stream);
    } else if (hipMallocAsync(&p, bytes, stream) != hipSuccess) {
      p = nullptr;
    }
    if (p) blocks.push_back({p, bytes, is_slab});
    return p;
  }
  void* get(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
    if (bytes > kCarveMax) return raw(bytes, false);
    if (!slab || slab_used + bytes > kSlabBytes) {
      slab = static_cast<char*>(raw(kSlabBytes, true));
      slab_used = 0;
      if (!slab) return nullptr;
    }
    void* p = slab + slab_used;
    slab_used += bytes;
    return p;
  }
  void put(void* p) {   // pieces of a slab stay until release_all
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i].p == p && !blocks[i].slab) {
        if (have_alloc) alloc.free(alloc.ctx, p, blocks[i].bytes, stream);
        else (void)hipFreeAsync(p, stream);
        blocks.erase(blocks.begin() + i);
        return;
      }
  }
  void release_all() {
    for (auto& b : blocks) {
      if (have_alloc) alloc.free(alloc.ctx, b.p, b.bytes, stream);
      else (void)hipFreeAsync(b.p, stream);
    }
    blocks.clear();
    slab = nullptr;
    slab_used = 0;
  }
};

bool finite_bounded(double v) { return std::isfinite(v) && std::fabs(v) <= 1e15; }

// The tape of an IBB_TAPE problem, checked op by op (the encoding is in ibb.h);
// cols_at receives where the coefficient columns start in coef.
ibb_status parse_tape(const ibb_problem* p, TapeDev& T, int64_t& cols_at) {
  const double* c = p->coef;
  const int64_t len = p->coef_len, n = p->n;
  auto bad = [](const std::string& why) { return fail(IBB_E_INVALID, "tape: " + why); };
  auto as_int = [](double v, int64_t lo, int64_t hi, int64_t& out) {
    if (!(v >= (double)lo && v <= (double)hi) || v != std::floor(v)) return false;
    out = (int64_t)v;
    return true;
  };
  if (!c || len < 4 || c[0] != 1.0) return bad("unknown format (coef[0] must be 1)");
  int64_t K, Q, C;
  if (!as_int(c[1], 0, kTapeMaxRed, K) || !as_int(c[2], 1, kTapeMaxOps, Q) || !as_int(c[3], 0, 64, C))
    return bad("K, Q or C out of range");
  T = TapeDev{};
  T.K = (int32_t)K;
  T.Q = (int32_t)Q;
  T.C = (int32_t)C;
  int64_t at = 4;
  int nops_all = 0;
  auto read_op = [&](int q, bool elem, int lim, TapeOp& o) -> bool {
    int64_t code, a, b;
    if (!as_int(c[at], 0, 18, code)) return false;
    if (!as_int(c[at + 1], -1, kTapeMaxOps, a) || !as_int(c[at + 2], -1, kTapeMaxOps, b)) return false;
    o.code = (int32_t)code;
    o.a = (int32_t)a;
    o.b = (int32_t)b;
    o.lo = c[at + 3];
    o.hi = c[at + 4];
    at += 5;
    const bool elem_only = code == 1 || code == 2 || code == 3 || code == 18;
    if (elem_only && !elem) return false;
    if (code == 17 && elem) return false;
    if ((code == 3 || code == 17) && (a < 0 || a >= lim)) return false;
    if (code >= 4 && code <= 16 && (a < 0 || a >= q)) return false;
    if (code >= 4 && code <= 7 && (b < 0 || b >= q)) return false;
    if (code == 0 && !(finite_bounded(o.lo) && finite_bounded(o.hi) && o.lo <= o.hi)) return false;
    return true;
  };
  for (int k = 0; k < K; ++k) {
    if (at + 6 > len) return bad("truncated");
    int64_t kind, s_off, s_end, t_off, t_end, L;
    if (!as_int(c[at], 0, 1, kind) || !as_int(c[at + 1], -n, n, s_off) || !as_int(c[at + 2], 0, 1, s_end) ||
        !as_int(c[at + 3], -n, n, t_off) || !as_int(c[at + 4], 0, 1, t_end) || !as_int(c[at + 5], 1, kTapeMaxOps, L))
      return bad("reduction header " + std::to_string(k));
    at += 6;
    if (at + 5 * L > len) return bad("truncated");
    int64_t start = s_off + (s_end ? n : 0), stop = t_off + (t_end ? n : 0);
    start = std::max<int64_t>(start, 0);
    stop = std::min<int64_t>(stop, n);
    stop = std::max(stop, start);
    TapeRed& R = T.red[k];
    R.kind = (int32_t)kind;
    R.start = (int32_t)start;
    R.stop = (int32_t)stop;
    R.first = nops_all;
    R.nops = (int32_t)L;
    for (int q = 0; q < L; ++q) {
      TapeOp& o = T.op[nops_all + q];
      if (!read_op(q, true, (int)C, o)) return bad("op " + std::to_string(q) + " of reduction " + std::to_string(k));
      if (o.code == 2 && (kind != 0 || stop > n - 1)) return bad("x_{i+1} needs a sum ending by n - 1");
    }
    nops_all += (int)L;
    if (kind == 1) T.nprod++;
  }
  if (at + 5 * Q > len) return bad("truncated");
  T.sc_first = nops_all;
  for (int q = 0; q < Q; ++q)
    if (!read_op(q, false, (int)K, T.op[nops_all + q])) return bad("scalar op " + std::to_string(q));
  if (at + C * n != len) return bad("coef_len does not match the tape and its columns");
  for (int64_t i = at; i < len; ++i)
    if (!finite_bounded(c[i])) return bad("coefficient column value not finite or too large");
  cols_at = at;
  return IBB_OK;
}

ibb_status validate(const ibb_problem* p) {
  if (!p) return fail(IBB_E_INVALID, "problem is NULL");
  if (p->family != IBB_SEP_COS && p->family != IBB_CHAIN && p->family != IBB_SEP_ABS_SIN2 && p->family != IBB_TAPE)
    return fail(IBB_E_INVALID, "unknown family " + std::to_string(p->family));
  if (p->n < 1 || p->n > (1 << 24)) return fail(IBB_E_INVALID, "n out of range");
  if (p->family == IBB_TAPE) {
    if (!p->coef || !p->lower || !p->upper) return fail(IBB_E_INVALID, "NULL array");
    TapeDev T;
    int64_t at = 0;
    ibb_status st = parse_tape(p, T, at);
    if (st != IBB_OK) return st;
    for (int i = 0; i < p->n; ++i) {
      if (!finite_bounded(p->lower[i]) || !finite_bounded(p->upper[i])) return fail(IBB_E_INVALID, "bounds must be finite");
      if (!(p->lower[i] < p->upper[i])) return fail(IBB_E_INVALID, "need lower < upper");
    }
    if (!(p->tol_f > 0.0) || !std::isfinite(p->tol_f)) return fail(IBB_E_INVALID, "tol_f must be > 0");
    if (!(p->tol_x >= 0.0)) return fail(IBB_E_INVALID, "tol_x must be >= 0");
    return IBB_OK;
  }
  if (p->family == IBB_CHAIN && p->n < 2) return fail(IBB_E_INVALID, "CHAIN needs n >= 2");
  const int64_t need = p->family == IBB_CHAIN ? 2 * (int64_t)(p->n - 1) : 4 * (int64_t)p->n;
  if (p->coef_len != need) return fail(IBB_E_INVALID, "coef_len must be " + std::to_string(need));
  if (!p->coef || !p->lower || !p->upper) return fail(IBB_E_INVALID, "NULL array");
  for (int64_t i = 0; i < need; ++i)
    if (!finite_bounded(p->coef[i])) return fail(IBB_E_INVALID, "coefficient " + std::to_string(i) + " not finite or too large");
  if (p->family != IBB_CHAIN)
    for (int i = 0; i < p->n; ++i) {
      const double k = p->coef[2 * (int64_t)p->n + i];
      if (!(k >= 1.0) || k != std::floor(k) || k > 1e12) return fail(IBB_E_INVALID, "k must be a positive integer");
    }
  for (int i = 0; i < p->n; ++i) {
    if (!finite_bounded(p->lower[i]) || !finite_bounded(p->upper[i])) return fail(IBB_E_INVALID, "bounds must be finite");
    if (!(p->lower[i] < p->upper[i])) return fail(IBB_E_INVALID, "need lower < upper");
  }
  if (!(p->tol_f > 0.0) || !std::isfinite(p->tol_f)) return fail(IBB_E_INVALID, "tol_f must be > 0");
  if (!(p->tol_x >= 0.0)) return fail(IBB_E_INVALID, "tol_x must be >= 0");
  return IBB_OK;
}

template <typename T>
T* dalloc(Mem& M, int64_t count) {
  return static_cast<T*>(M.get((size_t)std::max<int64_t>(count, 1) * sizeof(T)));
}

// the per-sweep trace: four rows of `cap` 8-byte entries in one block
constexpr int64_t kTraceStart = 4096, kTraceMax = (int64_t)1 << 17;
void set_trace(Params& P, double* block, int64_t cap) {
  P.tr_gub = block;
  P.tr_nsurv = reinterpret_cast<int64_t*>(block + cap);
  P.tr_nlive = reinterpret_cast<int64_t*>(block + 2 * cap);
  P.tr_sel = reinterpret_cast<int64_t*>(block + 3 * cap);
  P.trace_cap = cap;
}

// Whether single-precision evaluation cannot overflow: every intermediate of the
// FP32 trees, bounded from the coefficient and domain magnitudes, stays below
// 2^120 (and k_i <= 2^24 is exact in float).  Otherwise the filter stays off.
bool fp32_safe(const ibb_problem* p) {
  const int n = p->n;
  double B = 0.0;
  for (int i = 0; i < n; ++i) B = std::max(B, std::max(std::fabs(p->lower[i]), std::fabs(p->upper[i])));
  const double lim = std::ldexp(1.0, 120) / (4.0 * n + 4.0);
  double worst = 0.0;
  if (p->family == IBB_CHAIN) {
    for (int i = 0; i < n - 1; ++i) {
      const double al = std::fabs(p->coef[i]), be = std::fabs(p->coef[(n - 1) + i]);
      const double R = B + B * B, E = B + 1.0;
      worst = std::max({worst, al * R * R + be * E * E, 4.0 * al * B * R + 2.0 * be * E + 2.0 * al * R, R * R});
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const double a = std::fabs(p->coef[i]), b = std::fabs(p->coef[n + i]), k = p->coef[2 * n + i];
      const double D = B + std::fabs(p->coef[3 * n + i]);
      if (k > 16777216.0) return false;
      worst = std::max({worst, a * D * D + a * D + 2.0 * b, 2.0 * a * D + 7.0 * k * b, k * D, D * D});
    }
  }
  return worst < lim;
}

// coefficient tables and bounds on the device; the float tables only with want32
ibb_status upload_problem(Mem& M, const ibb_problem* p, Params& P, bool want32 = false) {
  const int n = p->n;
  P.family = p->family;
  P.n = n;
  std::vector<double> nl(n);
  for (int i = 0; i < n; ++i) nl[i] = -p->lower[i];
  double* d_nl = dalloc<double>(M, n);
  double* d_u = dalloc<double>(M, n);
  double* d_coef = dalloc<double>(M, p->coef_len);
  if (!d_nl || !d_u || !d_coef) return fail(IBB_E_NOMEM, "device allocation failed");
  HIPCHK(hipMemcpyAsync(d_nl, nl.data(), n * sizeof(double), hipMemcpyHostToDevice, M.stream));
  HIPCHK(hipMemcpyAsync(d_u, p->upper, n * sizeof(double), hipMemcpyHostToDevice, M.stream));
  HIPCHK(hipMemcpyAsync(d_coef, p->coef, p->coef_len * sizeof(double), hipMemcpyHostToDevice, M.stream));
  P.nl = d_nl;
  P.u = d_u;
  P.sep = nullptr;
  P.chain = nullptr;
  P.sep32 = nullptr;
  P.chain32 = nullptr;
  P.prec32 = want32 ? 1 : 0;
  P.incremental = 0;
  P.tape = nullptr;
  P.tcols = nullptr;
  P.tws = nullptr;
  const int blocks = (n + 255) / 256;
  if (p->family == IBB_TAPE) {   // the tape (checked by validate) and its columns, which stay in d_coef
    TapeDev T;
    int64_t at = 0;
    ibb_status st = parse_tape(p, T, at);
    if (st != IBB_OK) return st;
    TapeDev* dT = dalloc<TapeDev>(M, 1);
    if (!dT) return fail(IBB_E_NOMEM, "device allocation failed");
    HIPCHK(hipMemcpyAsync(dT, &T, sizeof(TapeDev), hipMemcpyHostToDevice, M.stream));
    HIPCHK(hipStreamSynchronize(M.stream));   // T and nl (host) must outlive their copies
    P.tape = dT;
    P.tcols = d_coef + at;
    return IBB_OK;
  }
  if (p->family == IBB_CHAIN) {
    CoefChain* c = dalloc<CoefChain>(M, n);
    CoefChain32* c32 = want32 ? dalloc<CoefChain32>(M, n) : nullptr;
    if (!c || (want32 && !c32)) return fail(IBB_E_NOMEM, "device allocation failed");
    hipLaunchKernelGGL(k_setup_chain, dim3(blocks), dim3(256), 0, M.stream, n, d_coef, c, c32);
    P.chain = c;
    P.chain32 = c32;
  } else {
    CoefSep* c = dalloc<CoefSep>(M, n);
    CoefSep32* c32 = want32 ? dalloc<CoefSep32>(M, n) : nullptr;
    if (!c || (want32 && !c32)) return fail(IBB_E_NOMEM, "device allocation failed");
    hipLaunchKernelGGL(k_setup_sep, dim3(blocks), dim3(256), 0, M.stream, n, p->family, d_coef, c, c32);
    P.sep = c;
    P.sep32 = c32;
  }
  HIPCHK(hipGetLastError());
  // nl (host) must outlive its copy; d_coef is not needed after the setup kernel
  HIPCHK(hipStreamSynchronize(M.stream));
  M.put(d_coef);
  return IBB_OK;
}

template <typename F>
void dispatch_family(int family, F&& f) {
  if (family == IBB_SEP_COS) f(std::integral_constant<int, FAM_SEP_COS>{});
  else if (family == IBB_CHAIN) f(std::integral_constant<int, FAM_CHAIN>{});
  else f(std::integral_constant<int, FAM_SEP_ABS_SIN2>{});
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Device memory of ibb_eval_boxes_noalloc: one fixed array per GPU (each device
// holds its own copy of a __device__ variable, for the life of the process).
// A call carves it, 256-byte aligned, as: Params, -lower[n], upper[n], the
// coefficients as given, the FP64 coefficient records, the FP32 ones.  Every
// field is written by the call before its kernels read it; nothing has to start
// at zero.  In host code `scratch` names a host-side stand-in, not device
// memory: the address each device uses comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;        // the per-device address table
std::mutex g_scratch_call_mu;   // calls that use the array, one at a time
void* g_scratch_addr[kScratchDevices] = {};

struct ScratchLayout {
  size_t nl, u, coef, tab, tab32, total;
};

ScratchLayout scratch_layout(const ibb_problem* p, bool want32) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t n = (size_t)p->n;
  const bool chain = p->family == IBB_CHAIN;
  ScratchLayout L{};
  L.nl = up(sizeof(Params));
  L.u = L.nl + up(n * sizeof(double));
  L.coef = L.u + up(n * sizeof(double));
  L.tab = L.coef + up((size_t)p->coef_len * sizeof(double));
  L.tab32 = L.tab + up(n * (chain ? sizeof(CoefChain) : sizeof(CoefSep)));
  L.total = L.tab32 + (want32 ? up(n * (chain ? sizeof(CoefChain32) : sizeof(CoefSep32))) : 0);
  return L;
}

// the current device's address of `scratch`, looked up on the first call on
// that device (with it current) and kept
ibb_status scratch_for_current_device(unsigned char** out) {
  int dev = -1;
  const hipError_t ed = hipGetDevice(&dev);
  if (ed != hipSuccess) return fail(IBB_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(ed));
  if (dev < 0 || dev >= kScratchDevices) return fail(IBB_E_DEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(IBB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = ptr;
  }
  *out = (unsigned char*)g_scratch_addr[dev];
  return IBB_OK;
}

}  // namespace

// result object -------------------------------------------------------------
struct ibb_result {
  ibb_info info{};
  Mem mem;
  Params P{};
  Params* dP = nullptr;
  State* dS = nullptr;                  // device state, kept so that ibb_sweep can continue the run
  ibb_options opts{};
  int64_t n_boxes = 0;
  // compacted live keys
  double* flo = nullptr;
  int64_t* seq = nullptr;
  int32_t* ref = nullptr;
  int32_t* r = nullptr;
  double* wmax = nullptr;
  std::vector<double> tr_gub;
  std::vector<int64_t> tr_nsurv, tr_nlive, tr_sel;
  // set when an ibb_sweep call failed after it had started to change the run:
  // the device state and the boxes are then no longer a consistent result
  bool broken = false;
};

namespace {

ibb_status push_params(Mem& M, const Params& P, Params* dP) {
  HIPCHK(hipMemcpyAsync(dP, &P, sizeof(Params), hipMemcpyHostToDevice, M.stream));
  return IBB_OK;
}

// one workgroup up to 4 Ki keys (no partials kernel), else ~8 keys per thread
int sel_blocks_for(int64_t keys) {
  if (keys <= 4096) return 1;
  int64_t b = (keys + kSelThreads * 8 - 1) / (kSelThreads * 8);
  return (int)std::min<int64_t>(std::max<int64_t>(b, 2), kMaxSelBlocks);
}

// stable compaction of keys with lower bound <= GUB into fresh arrays
ibb_status compact_keys(Mem& M, Params& P, Params* dP, State* dS, int64_t nk, int64_t cap_out, double*& o_flo,
                        int64_t*& o_seq, int32_t*& o_ref, int32_t*& o_r, double*& o_wmax, int64_t& kept) {
  int64_t* flags = dalloc<int64_t>(M, nk);
  const int64_t per_block = 4096;
  const int nblocks = (int)std::max<int64_t>(1, (nk + per_block - 1) / per_block);
  int64_t* bcnt = dalloc<int64_t>(M, nblocks);
  o_flo = dalloc<double>(M, cap_out);
  o_seq = dalloc<int64_t>(M, cap_out);
  o_ref = dalloc<int32_t>(M, cap_out);
  o_r = dalloc<int32_t>(M, cap_out);
  o_wmax = dalloc<double>(M, cap_out);
  if (!flags || !bcnt || !o_flo || !o_seq || !o_ref || !o_r || !o_wmax) return fail(IBB_E_NOMEM, "device allocation failed");
  hipLaunchKernelGGL(k_count_live, dim3(sel_blocks_for(nk)), dim3(kSelThreads), 0, M.stream, dP, dS, flags);
  hipLaunchKernelGGL(k_compact_count, dim3(nblocks), dim3(256), 0, M.stream, flags, nk, per_block, bcnt);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nblocks), dim3(256), 0, M.stream, dP, flags, nk, per_block, bcnt, nblocks,
                     o_flo, o_seq, o_ref, o_r, o_wmax);
  HIPCHK(hipGetLastError());
  std::vector<int64_t> h(nblocks);
  HIPCHK(hipMemcpyAsync(h.data(), bcnt, nblocks * sizeof(int64_t), hipMemcpyDeviceToHost, M.stream));
  HIPCHK(hipStreamSynchronize(M.stream));
  kept = 0;
  for (auto v : h) kept += v;
  M.put(flags);
  M.put(bcnt);
  return IBB_OK;
}

}  // namespace

namespace {

// One problem in flight: its result object (which owns the device memory), where
// its Params and State live on the device, and the host's view of its progress.
struct Run {
  ibb_result* R = nullptr;
  Params* dP = nullptr;
  State* dS = nullptr;
  ibb_options opts{};
  int64_t n_keys = 1, sweeps = 0;
  bool pending = false;
  State hs{};
  std::chrono::steady_clock::time_point t0;
  bool term_cache = false;   // ibb_solve's runs: keep the rows' shared terms (large n)
  bool mem_stop = false;     // the server ends this run at its next selection (memory budget)
};

// Allocate the problem's arrays, upload it and enqueue its root box (Sec. 3.1,
// Initialization).  dP/dS must already point to device storage.
ibb_status run_setup(Run& U, const ibb_problem* prob) {
  ibb_result* R = U.R;
  Mem& M = R->mem;
  Params& P = R->P;
  const int n = prob->n;
  ibb_status st = upload_problem(M, prob, P, U.opts.precision == IBB_FP32_BULK && fp32_safe(prob));
  if (st != IBB_OK) return st;
  P.incremental = U.opts.incremental && !P.tape ? 1 : 0;   // the generic family is bounded in full
  P.m = std::min(n, U.opts.split_dims);
  P.pieces = U.opts.pieces == 4 ? 4 : 2;
  P.nch = P.pieces == 4 ? 1 << (2 * P.m) : 1 << P.m;
  P.nsamp = U.opts.diag_samples;
  for (int q = 0; q < kMaxSamples; ++q)   // the double nearest (q + 1) / (S + 1)
    P.cs[q] = q < P.nsamp ? (double)(q + 1) / (double)(P.nsamp + 1) : 0.0;
  P.tol_f = prob->tol_f;
  P.tol_x = prob->tol_x;
  P.max_sweeps = U.opts.max_sweeps;
  P.max_live = U.opts.max_live_boxes;
  P.trace_cap = std::min<int64_t>(std::min<int64_t>(U.opts.max_sweeps + 1, kTraceMax), kTraceStart);
  P.select_k = U.opts.select_k;
  const int64_t nrec = (int64_t)P.select_k * P.nch;   // child records per sweep
  P.key_cap = std::max<int64_t>(4096, 4 * nrec);
  P.hist_cap = std::max<int64_t>(64, 2 * (int64_t)P.select_k + 2);
  P.key_flo = dalloc<double>(M, P.key_cap);
  P.key_seq = dalloc<int64_t>(M, P.key_cap);
  P.key_ref = dalloc<int32_t>(M, P.key_cap);
  P.key_r = dalloc<int32_t>(M, P.key_cap);
  P.key_wmax = dalloc<double>(M, P.key_cap);
  P.hist_n = dalloc<double>(M, P.hist_cap * n);
  P.hist_h = dalloc<double>(M, P.hist_cap * n);
  P.hist_cyc = dalloc<int32_t>(M, P.hist_cap);
  P.hist_mask = dalloc<uint32_t>(M, P.hist_cap);
  P.hist_mid = dalloc<double>(M, P.hist_cap * kMaxSplit);
  const bool four = P.pieces == 4;
  P.hist_cut = four ? dalloc<double>(M, P.hist_cap * 3 * kMaxSplit) : nullptr;
  P.tab = four ? dalloc<double>(M, kTabDoubles) : nullptr;
  P.tabi = four ? dalloc<int32_t>(M, kTabInts) : nullptr;
  P.ins_cnt = four ? dalloc<int32_t>(M, 2 * kMaxSelBlocks) : nullptr;
  P.ch_flo = dalloc<double>(M, nrec);
  P.ch_flag = dalloc<uint8_t>(M, nrec);
  P.ch_wmax = dalloc<double>(M, nrec);
  P.sel_tab = dalloc<SelRec>(M, P.select_k);
  P.ksel = P.select_k > 1 ? dalloc<KselBuf>(M, 1) : nullptr;
  const bool tc = U.term_cache && P.incremental && P.select_k == 1 && P.pieces == 2 && n >= kTermCacheMinN;
  P.tcache = tc ? dalloc<double>(M, P.hist_cap * 3 * n) : nullptr;
  P.hist_par = tc ? dalloc<int32_t>(M, P.hist_cap) : nullptr;
  P.ibsum = tc ? dalloc<double>(M, kIbWOff + (n + kIbRowBlock - 1) / kIbRowBlock) : nullptr;
  if (P.tape) {   // right products of the product reductions: n intervals each per child record
    TapeDev T;
    int64_t at = 0;
    if ((st = parse_tape(prob, T, at)) != IBB_OK) return st;
    if (T.nprod > 0) {
      const int64_t cnt = std::max<int64_t>(nrec, 1) * T.nprod * n;
      if (cnt * (int64_t)sizeof(I) > ((int64_t)8 << 30))
        return fail(IBB_E_CAPACITY, "the tape's product reductions need more than 8 GiB of workspace at this size");
      P.tws = dalloc<I>(M, cnt);
      if (!P.tws) return fail(IBB_E_NOMEM, "device allocation failed");
    }
  }
  P.part_flo = dalloc<double>(M, kMaxSelBlocks);
  P.part_idx = dalloc<int64_t>(M, kMaxSelBlocks);
  P.part_wmax = dalloc<double>(M, kMaxSelBlocks);
  P.part_cnt = dalloc<int64_t>(M, kMaxSelBlocks);
  set_trace(P, dalloc<double>(M, 4 * P.trace_cap), P.trace_cap);
  if (!P.key_flo || !P.key_seq || !P.key_ref || !P.key_r || !P.key_wmax || !P.hist_n || !P.hist_h || !P.hist_cyc ||
      !P.hist_mask || !P.hist_mid || !P.ch_flo || !P.ch_flag || !P.ch_wmax || !P.sel_tab ||
      (four && (!P.hist_cut || !P.tab || !P.tabi || !P.ins_cnt)) || (P.select_k > 1 && !P.ksel) ||
      (tc && (!P.tcache || !P.hist_par || !P.ibsum)) || !P.part_flo ||
      !P.part_idx || !P.part_wmax || !P.part_cnt || !P.tr_gub || !P.tr_nsurv || !P.tr_nlive || !P.tr_sel)
    return fail(IBB_E_NOMEM, "device allocation failed");
  // root row: (-l, u)
  std::vector<double> nl(n);
  for (int i = 0; i < n; ++i) nl[i] = -prob->lower[i];
  HIPCHK(hipMemcpyAsync(P.hist_n, nl.data(), n * sizeof(double), hipMemcpyHostToDevice, M.stream));
  HIPCHK(hipMemcpyAsync(P.hist_h, prob->upper, n * sizeof(double), hipMemcpyHostToDevice, M.stream));
  HIPCHK(hipMemsetAsync(U.dS, 0, sizeof(State), M.stream));
  // child records start as "not formed": nothing reads a record no bound kernel wrote
  HIPCHK(hipMemsetAsync(P.ch_flag, 0, nrec, M.stream));
  st = push_params(M, P, U.dP);
  if (st != IBB_OK) return st;
  HIPCHK(hipStreamSynchronize(M.stream));   // nl must outlive its copy
  if (P.tape)
    hipLaunchKernelGGL(k_tape_root, dim3(1), dim3(kWave), 0, M.stream, U.dP, U.dS);
  else
    dispatch_family(P.family, [&](auto fam) {
      hipLaunchKernelGGL(k_root<decltype(fam)::value>, dim3(1), dim3(kWave), 0, M.stream, U.dP, U.dS);
    });
  HIPCHK(hipGetLastError());
  U.n_keys = 1;
  U.sweeps = 0;
  U.pending = false;
  return IBB_OK;
}

// room for `chunk` more sweeps: one row and at most nch keys per sweep.
// Every array that has to grow is allocated before anything is copied or given
// back: if the allocator refuses a request, the blocks taken so far are returned
// and the arrays, the capacities and the device copy of the parameters stay as
// they were (the run can go on with what it has, or be released).  Only when
// every request succeeded are the contents copied, the old blocks returned, the
// new layout taken and the parameters pushed.
struct GrowPlan {
  bool rows = false, keys = false, tr = false;
  int64_t hist_cap = 0, key_cap = 0, tr_cap = 0;
  size_t bytes = 0;   // device memory the grown arrays take
};

GrowPlan plan_growth(const Run& U, int chunk) {
  const Params& P = U.R->P;
  const int64_t n = P.n;
  const int64_t K = P.select_k;
  // rows 0 .. (sweeps + 1) K are in use (the last K may belong to a pending selection)
  const int64_t need_rows = (U.sweeps + chunk + 1) * K + 1;
  const int64_t need_keys = U.n_keys + (int64_t)(chunk + 1) * K * P.nch;   // +1: children pending from the last chunk
  const int64_t need_tr = std::min<int64_t>(U.sweeps + chunk + 1, kTraceMax);
  GrowPlan g;
  g.rows = need_rows > P.hist_cap;
  g.keys = need_keys > P.key_cap;
  g.tr = need_tr > P.trace_cap;
  g.hist_cap = g.rows ? std::max<int64_t>(2 * P.hist_cap, need_rows) : P.hist_cap;
  g.key_cap = g.keys ? std::max<int64_t>(2 * P.key_cap, need_keys) : P.key_cap;
  g.tr_cap = g.tr ? std::min<int64_t>(std::max<int64_t>(2 * P.trace_cap, need_tr), kTraceMax) : P.trace_cap;
  if (g.rows) {
    int64_t per_row = 2 * n * 8 + 4 + 4 + kMaxSplit * 8;
    if (P.pieces == 4) per_row += 3 * kMaxSplit * 8;
    if (P.tcache) per_row += 3 * n * 8 + 4;
    g.bytes += (size_t)(g.hist_cap * per_row);
  }
  if (g.keys) g.bytes += (size_t)(g.key_cap * (8 + 8 + 4 + 4 + 8));
  if (g.tr) g.bytes += (size_t)(4 * g.tr_cap * 8);
  return g;
}

ibb_status run_capacity(Run& U, int chunk) {
  Mem& M = U.R->mem;
  Params& P = U.R->P;
  const int n = P.n;
  const GrowPlan gp = plan_growth(U, chunk);
  const bool g_rows = gp.rows, g_keys = gp.keys, g_tr = gp.tr;
  if (!g_rows && !g_keys && !g_tr) return IBB_OK;
  const int64_t K = P.select_k;
  Params Q = P;   // the grown layout
  std::vector<void*> fresh;
  bool ok = true;
  auto take = [&](auto*& dst, int64_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(dst)>>;
    dst = ok ? dalloc<std::remove_const_t<T>>(M, count) : nullptr;
    if (dst) fresh.push_back((void*)dst);
    else ok = false;
  };
  if (g_rows) {
    Q.hist_cap = gp.hist_cap;
    take(Q.hist_n, Q.hist_cap * n);
    take(Q.hist_h, Q.hist_cap * n);
    take(Q.hist_cyc, Q.hist_cap);
    take(Q.hist_mask, Q.hist_cap);
    take(Q.hist_mid, Q.hist_cap * kMaxSplit);
    if (P.pieces == 4) take(Q.hist_cut, Q.hist_cap * 3 * kMaxSplit);
    if (P.tcache) {
      take(Q.tcache, Q.hist_cap * 3 * n);
      take(Q.hist_par, Q.hist_cap);
    }
  }
  if (g_keys) {
    Q.key_cap = gp.key_cap;
    take(Q.key_flo, Q.key_cap);
    take(Q.key_seq, Q.key_cap);
    take(Q.key_ref, Q.key_cap);
    take(Q.key_r, Q.key_cap);
    take(Q.key_wmax, Q.key_cap);
  }
  double* tr = nullptr;
  int64_t tr_cap = P.trace_cap;
  if (g_tr) {
    tr_cap = gp.tr_cap;
    take(tr, 4 * tr_cap);
  }
  if (!ok) {
    for (void* q : fresh) M.put(q);
    return fail(IBB_E_NOMEM, "device allocation failed while growing the box list");
  }
  auto copy = [&](void* dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, M.stream) == hipSuccess;
  };
  bool copied = true;
  if (g_rows) {
    const int64_t keep = (U.sweeps + 1) * K + 1;
    copied = copied && copy(Q.hist_n, P.hist_n, keep * n * sizeof(double)) &&
             copy(Q.hist_h, P.hist_h, keep * n * sizeof(double)) && copy(Q.hist_cyc, P.hist_cyc, keep * sizeof(int32_t)) &&
             copy(Q.hist_mask, P.hist_mask, keep * sizeof(uint32_t)) &&
             copy(Q.hist_mid, P.hist_mid, keep * kMaxSplit * sizeof(double)) &&
             (P.pieces != 4 || copy(Q.hist_cut, P.hist_cut, keep * 3 * kMaxSplit * sizeof(double))) &&
             (!P.tcache || (copy(Q.tcache, P.tcache, keep * 3 * n * sizeof(double)) &&
                            copy(Q.hist_par, P.hist_par, keep * sizeof(int32_t))));
  }
  if (g_keys) {
    const int64_t keep = U.n_keys;
    copied = copied && copy(Q.key_flo, P.key_flo, keep * sizeof(double)) && copy(Q.key_seq, P.key_seq, keep * sizeof(int64_t)) &&
             copy(Q.key_ref, P.key_ref, keep * sizeof(int32_t)) && copy(Q.key_r, P.key_r, keep * sizeof(int32_t)) &&
             copy(Q.key_wmax, P.key_wmax, keep * sizeof(double));
  }
  if (g_tr) {
    const int64_t keep = std::min<int64_t>(U.sweeps, P.trace_cap);
    if (keep > 0)   // the four rows of the old block into the new one
      copied = copied && hipMemcpy2DAsync(tr, tr_cap * 8, P.tr_gub, P.trace_cap * 8, keep * 8, 4,
                                          hipMemcpyDeviceToDevice, M.stream) == hipSuccess;
    set_trace(Q, tr, tr_cap);
  }
  if (!copied) {   // the old arrays are untouched; the new blocks go back with the rest at release
    return fail(IBB_E_DEVICE, "copy failed while growing the box list");
  }
  if (g_rows) {
    M.put(P.hist_n); M.put(P.hist_h); M.put(P.hist_cyc); M.put(P.hist_mask); M.put(P.hist_mid);
    if (P.pieces == 4) M.put(P.hist_cut);
    if (P.tcache) { M.put(P.tcache); M.put(P.hist_par); }
  }
  if (g_keys) { M.put(P.key_flo); M.put(P.key_seq); M.put(P.key_ref); M.put(P.key_r); M.put(P.key_wmax); }
  if (g_tr) M.put(P.tr_gub);
  P = Q;
  return push_params(M, P, U.dP);
}

// End the run at its next selection with no more room: that selection inserts the
// children still pending (run_capacity left room for one sweep's children beyond
// the last chunk) and then stops at the sweep budget, so the list it leaves
// covers every box not yet discarded and [GLB, GUB] stays rigorous.
ibb_status run_stop_next(Run& U) {
  Params& P = U.R->P;
  P.max_sweeps = std::min<int64_t>(P.max_sweeps, U.sweeps);
  U.mem_stop = true;
  return push_params(U.R->mem, P, U.dP);
}

// after a chunk: take the device counters, drop removed keys when they dominate
ibb_status run_after_chunk(Run& U) {
  U.n_keys = U.hs.n_keys;
  U.sweeps = U.hs.sweeps;
  U.pending = U.hs.pending != 0;
  Params& P = U.R->P;
  if (!U.hs.stop && U.n_keys > 4 * (U.hs.n_live + P.nch) && U.n_keys > (int64_t)1 << 14) {
    Mem& M = U.R->mem;
    double* f; int64_t* sq; int32_t* rf; int32_t* rr; double* wx; int64_t kept = 0;
    ibb_status st = compact_keys(M, P, U.dP, U.dS, U.n_keys, P.key_cap, f, sq, rf, rr, wx, kept);
    if (st != IBB_OK) return st;
    M.put(P.key_flo); M.put(P.key_seq); M.put(P.key_ref); M.put(P.key_r); M.put(P.key_wmax);
    P.key_flo = f; P.key_seq = sq; P.key_ref = rf; P.key_r = rr; P.key_wmax = wx;
    st = push_params(M, P, U.dP);
    if (st != IBB_OK) return st;
    HIPCHK(hipMemcpyAsync(&U.dS->n_keys, &kept, sizeof(int64_t), hipMemcpyHostToDevice, M.stream));
    HIPCHK(hipStreamSynchronize(M.stream));
    U.n_keys = kept;
  }
  return IBB_OK;
}

// final list (keys with lower bound <= GUB, in insertion order), trace, info
ibb_status run_finish(Run& U) {
  ibb_result* R = U.R;
  Mem& M = R->mem;
  Params& P = R->P;
  const State& hs = U.hs;
  int64_t kept = 0;
  ibb_status st = compact_keys(M, P, U.dP, U.dS, U.n_keys, std::max<int64_t>(U.n_keys, 1), R->flo, R->seq, R->ref, R->r,
                               R->wmax, kept);
  if (st != IBB_OK) return st;
  R->n_boxes = kept;
  std::vector<double> hflo(kept);
  if (kept) HIPCHK(hipMemcpy(hflo.data(), R->flo, kept * sizeof(double), hipMemcpyDeviceToHost));
  double glb = INFINITY;
  for (double v : hflo) glb = std::min(glb, v);
  const int64_t tn = std::min<int64_t>(hs.sweeps, P.trace_cap);
  R->tr_gub.resize(tn); R->tr_nsurv.resize(tn); R->tr_nlive.resize(tn); R->tr_sel.resize(tn);
  if (tn > 0) {   // the four trace rows in one copy
    std::vector<uint64_t> h(4 * tn);
    HIPCHK(hipMemcpy2DAsync(h.data(), tn * 8, P.tr_gub, P.trace_cap * 8, tn * 8, 4, hipMemcpyDeviceToHost, M.stream));
    HIPCHK(hipStreamSynchronize(M.stream));
    std::memcpy(R->tr_gub.data(), h.data(), tn * 8);
    std::memcpy(R->tr_nsurv.data(), h.data() + tn, tn * 8);
    std::memcpy(R->tr_nlive.data(), h.data() + 2 * tn, tn * 8);
    std::memcpy(R->tr_sel.data(), h.data() + 3 * tn, tn * 8);
    if (hs.sweeps <= P.trace_cap) R->tr_nlive[tn - 1] = kept;
  }
  R->info.f_lo = glb;
  R->info.f_hi = okey_inv(hs.gub_key);
  R->info.n_boxes = kept;
  R->info.sweeps = hs.sweeps;
  R->info.boxes_evaluated = hs.evaluated;
  R->info.fp32_pruned = hs.fp32_pruned;
  R->info.fp64_confirmed = hs.evaluated - hs.fp32_pruned;
  R->info.fp32_sweeps = (int32_t)std::min<int64_t>(hs.fp32_sweeps, INT32_MAX);
  R->info.ub_evaluated = hs.ub_evaluated;
  R->info.status = hs.stop == STOP_CONVERGED ? IBB_OK
                   : (hs.stop == STOP_EMPTY || hs.stop == STOP_CAPACITY || hs.stop == STOP_INTERNAL) ? IBB_E_INTERNAL
                                                                                                 : IBB_NOT_CONVERGED;
  R->info.stop_reason = U.mem_stop && hs.stop == STOP_SWEEPS ? STOP_MEMORY : hs.stop;
  R->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - U.t0).count();
  if (hs.stop == STOP_CAPACITY) return fail(IBB_E_INTERNAL, "a sweep would pass the sized row or key capacity");
  if (hs.stop == STOP_INTERNAL) return fail(IBB_E_INTERNAL, "the selection counted live boxes but found none");
  if (R->info.status == IBB_E_INTERNAL) return fail(IBB_E_INTERNAL, "the live list became empty");
  return IBB_OK;
}

ibb_status check_options(const ibb_options& o) {
  if (o.split_dims < 1 || o.split_dims > kMaxSplit) return fail(IBB_E_INVALID, "split_dims must be in 1..16");
  if (o.select_k < 1 || o.select_k > kMaxSelectK) return fail(IBB_E_INVALID, "select_k must be in 1..1024");
  if (((int64_t)o.select_k << o.split_dims) > ((int64_t)1 << 24))
    return fail(IBB_E_INVALID, "select_k * 2^split_dims must not exceed 2^24 children per sweep");
  if (o.precision != IBB_FP64 && o.precision != IBB_FP32_BULK) return fail(IBB_E_INVALID, "unknown precision");
  if (o.incremental != 0 && o.incremental != 1) return fail(IBB_E_INVALID, "incremental must be 0 or 1");
  if (o.incremental && o.precision == IBB_FP32_BULK)
    return fail(IBB_E_INVALID, "the FP32 filter works on full bounds: set incremental = 0 with IBB_FP32_BULK");
  if (o.incremental && o.bound_shape != 0)
    return fail(IBB_E_INVALID, "bound_shape applies to full bounds (incremental = 0)");
  if (o.max_sweeps < 0) return fail(IBB_E_INVALID, "max_sweeps must be >= 0");
  const int pc = o.pieces == 0 ? 2 : o.pieces;   // 0: the default, bisection
  if (!((pc == 2 && o.diag_samples == 0) || (pc == 4 && o.diag_samples >= 1 && o.diag_samples <= kMaxSamples)))
    return fail(IBB_E_INVALID, "pieces and diag_samples: 2 and 0 (bisection, midpoint), or 4 and 1..16 (the paper's schedule)");
  if (pc == 4) {
    if (!o.incremental || o.select_k != 1 || o.precision != IBB_FP64 || o.bound_shape != 0)
      return fail(IBB_E_INVALID, "the four-piece schedule runs with incremental bounds, select_k = 1 and FP64");
    if (o.split_dims > 12) return fail(IBB_E_INVALID, "the four-piece schedule splits at most 12 coordinates (4^12 children)");
  }
  return IBB_OK;
}

// ---------------------------------------------------------------------------
// bound kernel shapes and the autotuner
//
// A shape is W wavefronts per child over the coordinate tiles (W = 1, 2, 4), in
// latency mode (CONC = 1: W more wavefronts per child compute the midpoint bound
// at the same time) or throughput mode (CONC = 0: F first, then the midpoint
// bound unless F.lo already exceeds the GUB; the FP32 filter runs only here).
// A workgroup holds 4 wavefronts, so 4 / (W (1 + CONC)) children.
struct BoundShape {
  int w, conc;
};
constexpr int kNumBoundShapes = 5;
constexpr BoundShape kBoundShapes[kNumBoundShapes] = {{1, 1}, {2, 1}, {1, 0}, {2, 0}, {4, 0}};

template <int FAM>
void launch_bound(int shape, int nch, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, Params* dP, State* dS) {
  const BoundShape bs = kBoundShapes[shape];
  const int cpb = kBoundWaves / (bs.w * (1 + bs.conc));
  const dim3 g((nch + cpb - 1) / cpb), b(kWave * kBoundWaves);
  switch (shape) {
    case 0: hipExtLaunchKernelGGL((k_bound<FAM, 1, 1>), g, b, 0, stream, e0, e1, 0, dP, dS); break;
    case 1: hipExtLaunchKernelGGL((k_bound<FAM, 2, 1>), g, b, 0, stream, e0, e1, 0, dP, dS); break;
    case 2: hipExtLaunchKernelGGL((k_bound<FAM, 1, 0>), g, b, 0, stream, e0, e1, 0, dP, dS); break;
    case 3: hipExtLaunchKernelGGL((k_bound<FAM, 2, 0>), g, b, 0, stream, e0, e1, 0, dP, dS); break;
    default: hipExtLaunchKernelGGL((k_bound<FAM, 4, 0>), g, b, 0, stream, e0, e1, 0, dP, dS); break;
  }
}

std::mutex g_tune_mu;
std::unordered_map<uint64_t, int> g_tuned;

int tuned_shape(uint64_t key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  return it == g_tuned.end() ? -1 : it->second;
}
void store_tuned_shape(uint64_t key, int shape) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = shape;
}

// Time every admissible shape on the first sweep of this problem and return the
// fastest.  The first sweep's selection runs as usual; its bound kernel then runs
// once per shape to warm up and 3 times per shape under HIP events.  Repeating it
// is harmless: every run writes the same child records, and the GUB is a minimum
// of the same upper bounds; the counters are restored from the state after the
// first run.  The solve then continues with the next sweep's selection.
ibb_status autotune_bound(Run& U, int n_tiles, int& best) {
  ibb_result* R = U.R;
  Mem& M = R->mem;
  Params& P = R->P;
  best = P.prec32 ? (n_tiles <= 1 ? 2 : (n_tiles <= 4 ? 3 : 4)) : (n_tiles <= 1 ? 0 : (n_tiles <= 4 ? 1 : 4));
  if (P.select_k > 1)
    hipLaunchKernelGGL(k_select_k<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP, U.dS, 0);
  else
    hipLaunchKernelGGL(k_select<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP, U.dS, 0, 0);
  HIPCHK(hipMemcpyAsync(&U.hs, U.dS, sizeof(State), hipMemcpyDeviceToHost, M.stream));
  HIPCHK(hipStreamSynchronize(M.stream));
  U.sweeps = U.hs.sweeps;
  U.pending = U.hs.pending != 0;
  if (U.hs.stop || !U.hs.pending) return IBB_OK;   // nothing to bound: keep the default shape
  hipEvent_t ev[2];
  HIPCHK(hipEventCreate(&ev[0]));
  if (hipEventCreate(&ev[1]) != hipSuccess) { (void)hipEventDestroy(ev[0]); return fail(IBB_E_DEVICE, "hipEventCreate failed"); }
  State after{};
  float best_ms = 0.0f;
  ibb_status st = IBB_OK;
  dispatch_family(P.family, [&](auto fam) {
    constexpr int FAM = decltype(fam)::value;
    bool first = true;
    for (int v = 0; v < kNumBoundShapes && st == IBB_OK; ++v) {
      if (P.prec32 && kBoundShapes[v].conc) continue;
      if (kBoundShapes[v].w > 1 && kBoundShapes[v].w > n_tiles) continue;   // idle waves
      launch_bound<FAM>(v, P.select_k * P.nch, M.stream, nullptr, nullptr, U.dP, U.dS);
      if (first) {
        if (hipMemcpyAsync(&after, U.dS, sizeof(State), hipMemcpyDeviceToHost, M.stream) != hipSuccess ||
            hipStreamSynchronize(M.stream) != hipSuccess) { st = fail(IBB_E_DEVICE, "autotune copy failed"); break; }
        first = false;
      }
      float tot = 0.0f;
      for (int r = 0; r < 3; ++r) {
        float ms = 0.0f;
        launch_bound<FAM>(v, P.select_k * P.nch, M.stream, ev[0], ev[1], U.dP, U.dS);
        if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
          st = fail(IBB_E_DEVICE, "autotune timing failed");
          break;
        }
        tot += ms;
      }
      if (st == IBB_OK && (best_ms == 0.0f || tot < best_ms)) { best_ms = tot; best = v; }
    }
  });
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st != IBB_OK) return st;
  if (hipGetLastError() != hipSuccess) return fail(IBB_E_DEVICE, "autotune launch failed");
  HIPCHK(hipMemcpyAsync(U.dS, &after, sizeof(State), hipMemcpyHostToDevice, M.stream));
  HIPCHK(hipStreamSynchronize(M.stream));
  U.hs = after;
  return IBB_OK;
}

// Run sweeps in chunks (4, 8, ..., 256 sweeps enqueued between two reads of the
// device state) until the stop test or the time limit ends the iteration.
ibb_status run_sweeps(Run& U, int bound_shape) {
  ibb_result* R = U.R;
  Mem& M = R->mem;
  Params& P = R->P;
  ibb_status st = IBB_OK;
  struct Events {
    std::vector<hipEvent_t> v;
    ~Events() { for (auto e : v) (void)hipEventDestroy(e); }
  } evs;
  auto& ev = evs.v;
  int grow_chunk = 4;   // sweeps per host round trip on the per-sweep path (and under a time limit): 4, 8, ..., 256
  // Shape of the per-sweep incremental kernel (one box per sweep, long lists):
  // 512 or 1024 threads, i.e. 8 or 16 wavefronts and 4 or 2 base terms per thread
  // between barriers; both give the same bits.  Tuned per (family, n, m): the
  // first run that needs it times one chunk with each and keeps the faster.
  const bool ib_sweep = P.incremental && P.select_k == 1 && P.pieces == 2 && P.tape == nullptr && !P.tcache;
  // one box per sweep at large n: every sweep on several workgroups (k_ib_pick ... k_ib_finish)
  const bool ib_pipe = P.incremental && P.select_k == 1 && P.pieces == 2 && P.tape == nullptr && P.tcache &&
                       P.n >= kIbPipeMinN;
  const uint64_t ib_key = (1ull << 63) | ((uint64_t)P.family << 56) | ((uint64_t)std::min(P.n, 1 << 24) << 8) |
                          (uint64_t)P.m;
  int ib_shape = ib_sweep ? tuned_shape(ib_key) : 0;   // 0: 512 threads, 1: 1024; -1: not known yet
  float ib_us[2] = {-1.0f, -1.0f};
  struct TuneEvents {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~TuneEvents() { for (auto x : e) if (x) (void)hipEventDestroy(x); }
  } tev;
  for (;;) {
    // incremental bounds on a list one workgroup scans quickly: a whole chunk of
    // sweeps in one launch, as many as keep the list's growth within a bound
    const bool multi = P.select_k > 1;   // K boxes per sweep: a selection kernel and a bound kernel per sweep
    const bool four = P.pieces == 4;     // the paper's schedule: selection, tables, children kernels per sweep
    const bool tape = P.tape != nullptr; // the generic family: selection and a children kernel per sweep
    const bool persist = !multi && !four && !ib_pipe && P.incremental && U.n_keys <= kPersistentMaxKeys;
    int chunk = persist ? (int)std::min<int64_t>(std::max<int64_t>(kPersistentGrowth / P.nch, 16), 256) : grow_chunk;
    if (!persist)   // the key arrays are sized for every child of the chunk surviving: keep that within 2^23 keys
      chunk = (int)std::max<int64_t>(1, std::min<int64_t>(chunk, ((int64_t)1 << 23) / ((int64_t)P.select_k * P.nch)));
    if (U.opts.time_limit_s > 0.0) chunk = std::min(chunk, grow_chunk);   // the limit is checked between launches
    if ((st = run_capacity(U, chunk)) != IBB_OK) return st;
    const int sb = sel_blocks_for(U.n_keys + (int64_t)(chunk + 1) * P.nch);
    // the paper's schedule with many records per sweep: their insertion on many
    // workgroups (about 1024 records each) before the selection, not in it
    const int ins_blocks = four && !multi && !P.prec32 && P.nch >= (1 << 16)
                               ? (int)std::min<int64_t>(kMaxSelBlocks, ((int64_t)P.nch + 1023) / 1024)
                               : 0;
    const bool prof = U.opts.profile != 0;
    // a chunk on the per-sweep incremental path while the shape is not known times one shape
    const bool tuning = ib_shape < 0 && !persist && !multi && !four && !tape;
    const int ib_try = tuning ? (ib_us[0] < 0.0f ? 0 : 1) : std::max(ib_shape, 0);
    if (tuning) {
      for (auto& x : tev.e)
        if (!x && hipEventCreate(&x) != hipSuccess) return fail(IBB_E_DEVICE, "hipEventCreate failed");
      HIPCHK(hipEventRecord(tev.e[0], M.stream));
    }
    const int nev = persist ? 4 : 4 * chunk;
    if (prof && (int)ev.size() < nev) {
      const size_t old_n = ev.size();
      ev.resize(nev);
      for (size_t e = old_n; e < ev.size(); ++e)
        if (hipEventCreate(&ev[e]) != hipSuccess) return (fail(IBB_E_DEVICE, "hipEventCreate failed"));
    }
    // LDS of the children kernel of the four-piece schedule: table rows for at most
    // m affected terms (2 m + 2 for the chained family), 3 m test rows
    const int rows4 = P.family == IBB_CHAIN ? 2 * P.m + 2 : P.m;
    const size_t lds4 = (size_t)rows4 * 16 * (2 + P.nsamp) * sizeof(double) + (size_t)3 * P.m * 64 * sizeof(int);
    dispatch_family(P.family, [&](auto fam) {
      constexpr int FAM = decltype(fam)::value;
      if (persist) {
        hipExtLaunchKernelGGL((k_sweeps_ib<kSweepThreads, FAM>), dim3(1), dim3(kSweepThreads), 0, M.stream,
                              prof ? ev[0] : nullptr, prof ? ev[3] : nullptr, 0, U.dP, U.dS, chunk);
        return;
      }
      for (int s = 0; s < chunk && tape; ++s) {   // the generic family: selection, then every child in full
        if (ins_blocks > 0) {
          hipLaunchKernelGGL(k_ins_count, dim3(ins_blocks), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ins_scatter, dim3(ins_blocks), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ins_finish, dim3(1), dim3(kWave), 0, M.stream, U.dP, U.dS, ins_blocks);
        }
        if (sb > 1)
          hipExtLaunchKernelGGL(k_select_part, dim3(sb), dim3(kSelThreads), 0, M.stream, prof ? ev[4 * s + 0] : nullptr,
                                nullptr, 0, U.dP, U.dS);
        if (four)
          hipExtLaunchKernelGGL(k_select4<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                                (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                                U.dS, sb > 1 ? sb : 0, 0);
        else
          hipExtLaunchKernelGGL(k_select<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                                (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                                U.dS, sb > 1 ? sb : 0, 0);
        const dim3 gch((unsigned)((P.nch + 255) / 256));
        if (four) {
          hipExtLaunchKernelGGL(k_tape_children<4>, gch, dim3(256), 0, M.stream, prof ? ev[4 * s + 1] : nullptr,
                                nullptr, 0, U.dP, U.dS);
          hipExtLaunchKernelGGL(k_tape_samples<4>, gch, dim3(256), 0, M.stream, nullptr,
                                prof ? ev[4 * s + 2] : nullptr, 0, U.dP, U.dS);
        } else {
          hipExtLaunchKernelGGL(k_tape_children<2>, gch, dim3(256), 0, M.stream, prof ? ev[4 * s + 1] : nullptr,
                                nullptr, 0, U.dP, U.dS);
          hipExtLaunchKernelGGL(k_tape_samples<2>, gch, dim3(256), 0, M.stream, nullptr,
                                prof ? ev[4 * s + 2] : nullptr, 0, U.dP, U.dS);
        }
      }
      for (int s = 0; s < chunk && four && !tape; ++s) {
        if (ins_blocks > 0) {
          hipLaunchKernelGGL(k_ins_count, dim3(ins_blocks), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ins_scatter, dim3(ins_blocks), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ins_finish, dim3(1), dim3(kWave), 0, M.stream, U.dP, U.dS, ins_blocks);
        }
        if (sb > 1)
          hipExtLaunchKernelGGL(k_select_part, dim3(sb), dim3(kSelThreads), 0, M.stream, prof ? ev[4 * s + 0] : nullptr,
                                nullptr, 0, U.dP, U.dS);
        hipExtLaunchKernelGGL(k_select4<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                              (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                              U.dS, sb > 1 ? sb : 0, 0);
        hipExtLaunchKernelGGL((k_prep4<kSweepThreads, FAM>), dim3(1), dim3(kSweepThreads), 0, M.stream,
                              prof ? ev[4 * s + 1] : nullptr, nullptr, 0, U.dP, U.dS);
        hipExtLaunchKernelGGL(k_children4<FAM>, dim3((unsigned)((P.nch + 255) / 256)), dim3(256), lds4, M.stream,
                              nullptr, prof ? ev[4 * s + 2] : nullptr, 0, U.dP, U.dS, rows4);
      }
      for (int s = 0; s < chunk && multi; ++s) {
        if (sb > 1) {   // a long list: the selection's passes over it on sb workgroups
          hipExtLaunchKernelGGL(k_select_part, dim3(sb), dim3(kSelThreads), 0, M.stream,
                                prof ? ev[4 * s + 0] : nullptr, nullptr, 0, U.dP, U.dS);
          hipLaunchKernelGGL(k_ksel_begin<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP,
                             U.dS, sb);
          for (int q = 0; q < 8; ++q)
            hipLaunchKernelGGL(k_ksel_hist, dim3(sb), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ksel_take, dim3(sb), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
          hipExtLaunchKernelGGL(k_ksel_rows<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                                nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP, U.dS);
        } else {
          hipExtLaunchKernelGGL(k_select_k<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                                prof ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP, U.dS, 0);
        }
        if (P.incremental)
          hipExtLaunchKernelGGL((k_ib_parents<kSweepThreads, FAM>), dim3(P.select_k), dim3(kSweepThreads), 0, M.stream,
                                prof ? ev[4 * s + 1] : nullptr, prof ? ev[4 * s + 2] : nullptr, 0, U.dP, U.dS);
        else
          launch_bound<FAM>(bound_shape, P.select_k * P.nch, M.stream, prof ? ev[4 * s + 1] : nullptr,
                            prof ? ev[4 * s + 2] : nullptr, U.dP, U.dS);
      }
      for (int s = 0; s < chunk && !multi && !four && !tape; ++s) {
        if (sb > 1)
          hipExtLaunchKernelGGL(k_select_part, dim3(sb), dim3(kSelThreads), 0, M.stream, prof ? ev[4 * s + 0] : nullptr,
                                nullptr, 0, U.dP, U.dS);
        if (ib_pipe) {   // the sweep on several workgroups
          const int nblk = (P.n + kIbRowBlock - 1) / kIbRowBlock;
          hipExtLaunchKernelGGL(k_ib_pick<kSelIbThreads>, dim3(1), dim3(kSelIbThreads), 0, M.stream,
                                (prof && sb == 1) ? ev[4 * s + 0] : nullptr, nullptr, 0, U.dP, U.dS, sb > 1 ? sb : 0,
                                0);
          // the separable families: one more workgroup for the tables of the split halves
          hipLaunchKernelGGL(k_ib_rowterms<FAM>, dim3(nblk + (FAM != FAM_CHAIN ? 1 : 0)), dim3(kIbRowBlock), 0,
                             M.stream, U.dP, U.dS);
          hipLaunchKernelGGL(k_ib_slots, dim3(3), dim3(kIbSlotsThreads), 0, M.stream, U.dP, U.dS);
          hipExtLaunchKernelGGL((k_ib_finish<kSelIbThreads, FAM>), dim3(1), dim3(kSelIbThreads), 0, M.stream, nullptr,
                                prof ? ev[4 * s + 3] : nullptr, 0, U.dP, U.dS, nblk);
          continue;
        }
        if (P.incremental) {   // selection and the children's bounds in one workgroup
          if (ib_try == 1)
            hipExtLaunchKernelGGL((k_select_ib<1024, FAM>), dim3(1), dim3(1024), 0, M.stream,
                                  (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                                  U.dS, sb > 1 ? sb : 0, 0);
          else
            hipExtLaunchKernelGGL((k_select_ib<kSelIbThreads, FAM>), dim3(1), dim3(kSelIbThreads), 0, M.stream,
                                  (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                                  U.dS, sb > 1 ? sb : 0, 0);
          continue;
        }
        hipExtLaunchKernelGGL(k_select<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream,
                              (prof && sb == 1) ? ev[4 * s + 0] : nullptr, prof ? ev[4 * s + 3] : nullptr, 0, U.dP,
                              U.dS, sb > 1 ? sb : 0, 0);
        launch_bound<FAM>(bound_shape, P.nch, M.stream, prof ? ev[4 * s + 1] : nullptr, prof ? ev[4 * s + 2] : nullptr,
                          U.dP, U.dS);
      }
    });
    if (hipGetLastError() != hipSuccess) return (fail(IBB_E_DEVICE, "sweep launch failed"));
    if (tuning) HIPCHK(hipEventRecord(tev.e[1], M.stream));
    if (hipMemcpyAsync(&U.hs, U.dS, sizeof(State), hipMemcpyDeviceToHost, M.stream) != hipSuccess ||
        hipStreamSynchronize(M.stream) != hipSuccess)
      return (fail(IBB_E_DEVICE, "sweep failed"));
    if (tuning) {
      // time per sweep of this chunk; a chunk that ran fewer than 4 sweeps is not counted
      const int64_t ran = U.hs.sweeps - U.sweeps;
      float ms = 0.0f;
      if (ran >= 4 && hipEventElapsedTime(&ms, tev.e[0], tev.e[1]) == hipSuccess) {
        ib_us[ib_try] = 1e3f * ms / (float)ran;
        if (ib_us[0] >= 0.0f && ib_us[1] >= 0.0f) {
          ib_shape = ib_us[1] < ib_us[0] ? 1 : 0;
          store_tuned_shape(ib_key, ib_shape);
        }
      }
    }
    if (prof && persist) {
      // one launch for the chunk: its time over the selections it made
      const int64_t ran = (U.hs.sweeps + (U.hs.pending ? 1 : 0)) - (U.sweeps + (U.pending ? 1 : 0));
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[0], ev[3]) == hipSuccess) R->info.t_select_ms += ms;
      R->info.n_select_launches += ran + (U.hs.stop ? 1 : 0);
      R->info.n_persistent_launches++;
      R->info.t_persistent_ms += ms;
      R->info.n_persistent_sweeps += ran + (U.hs.stop ? 1 : 0);
    } else if (prof) {
      // bound launches that did work in this chunk; the select of the stopping sweep ran too
      const int64_t ran = (U.hs.sweeps + (U.hs.pending ? 1 : 0)) - (U.sweeps + (U.pending ? 1 : 0));
      for (int s = 0; s < chunk; ++s) {
        float ms = 0.f;
        if (s < ran || (s == ran && U.hs.stop)) {
          if (hipEventElapsedTime(&ms, ev[4 * s + 0], ev[4 * s + 3]) == hipSuccess) R->info.t_select_ms += ms;
          R->info.n_select_launches++;
        }
        if (s < ran && (!P.incremental || multi || four)) {
          if (hipEventElapsedTime(&ms, ev[4 * s + 1], ev[4 * s + 2]) == hipSuccess) R->info.t_bound_ms += ms;
          R->info.n_bound_launches++;
        }
      }
    }
    if (U.hs.stop) { if ((st = run_after_chunk(U)) != IBB_OK) return st; break; }
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - U.t0).count();
    if (U.opts.time_limit_s > 0.0 && el > U.opts.time_limit_s) {
      // insert the last sweep's children, then stop
      if (multi) {
        hipLaunchKernelGGL(k_select_k<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP, U.dS, 1);
      } else if (four) {
        const int sbf = sel_blocks_for(U.hs.n_keys);
        if (sbf > 1) hipLaunchKernelGGL(k_select_part, dim3(sbf), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
        hipLaunchKernelGGL(k_select4<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP, U.dS,
                           sbf > 1 ? sbf : 0, 1);
      } else {
        const int sbf = sel_blocks_for(U.hs.n_keys);
        if (sbf > 1) hipLaunchKernelGGL(k_select_part, dim3(sbf), dim3(kSelThreads), 0, M.stream, U.dP, U.dS);
        hipLaunchKernelGGL(k_select<kSelSingleThreads>, dim3(1), dim3(kSelSingleThreads), 0, M.stream, U.dP, U.dS,
                           sbf > 1 ? sbf : 0, 1);
      }
      if (hipMemcpyAsync(&U.hs, U.dS, sizeof(State), hipMemcpyDeviceToHost, M.stream) != hipSuccess ||
          hipStreamSynchronize(M.stream) != hipSuccess)
        return (fail(IBB_E_DEVICE, "final insert failed"));
      U.n_keys = U.hs.n_keys;
      U.sweeps = U.hs.sweeps;
      break;
    }
    if ((st = run_after_chunk(U)) != IBB_OK) return st;
    grow_chunk = std::min(grow_chunk * 2, 256);
  }
  return IBB_OK;
}

}  // namespace

extern "C" {

ibb_status ibb_options_default(ibb_options* o) {
  if (!o) return fail(IBB_E_INVALID, "options is NULL");
  o->precision = IBB_FP64;
  o->split_dims = 10;
  o->select_k = 1;
  o->deterministic = 1;
  o->max_sweeps = 1000000;
  o->max_live_boxes = (int64_t)1 << 26;
  o->time_limit_s = 0.0;
  o->profile = 0;
  o->bound_shape = 0;
  o->incremental = 1;
  o->pieces = 2;
  o->diag_samples = 0;
  o->reserved = 0;
  return IBB_OK;
}

const char* ibb_status_string(ibb_status s) {
  switch (s) {
    case IBB_OK: return "ok";
    case IBB_NOT_CONVERGED: return "not converged (budget reached; enclosure still rigorous)";
    case IBB_PENDING: return "pending";
    case IBB_E_INVALID: return "invalid argument";
    case IBB_E_NOMEM: return "out of memory";
    case IBB_E_DEVICE: return "device error";
    case IBB_E_CAPACITY: return "capacity exceeded";
    case IBB_E_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ibb_last_error(void) { return g_err.c_str(); }

static ibb_status solve_impl(const ibb_problem* prob, const ibb_options* opts_in, const ibb_allocator* alloc,
                             void* hip_stream, ibb_result** out) {
  if (!out) return fail(IBB_E_INVALID, "out is NULL");
  *out = nullptr;
  ibb_status st = validate(prob);
  if (st != IBB_OK) return st;
  Run U;
  U.t0 = std::chrono::steady_clock::now();
  if (opts_in) U.opts = *opts_in; else ibb_options_default(&U.opts);
  if (prob->family == IBB_TAPE) {
    // the generic family is bounded in full, one box per sweep, in FP64
    if (U.opts.select_k != 1 || U.opts.precision != IBB_FP64 || U.opts.bound_shape != 0)
      return fail(IBB_E_INVALID, "the generic family (IBB_TAPE) runs with select_k = 1, FP64 and bound_shape 0");
    U.opts.incremental = 1;   // passes the option checks; the tape kernels bound every child in full
  }
  if ((st = check_options(U.opts)) != IBB_OK) return st;

  ibb_result* R = new ibb_result();
  U.R = R;
  Mem& M = R->mem;
  M.stream = (hipStream_t)hip_stream;
  if (alloc && alloc->alloc && alloc->free) { M.alloc = *alloc; M.have_alloc = true; }
  auto bail = [&](ibb_status s) { (void)hipStreamSynchronize(M.stream); M.release_all(); delete R; return s; };
  U.dP = dalloc<Params>(M, 1);
  U.dS = dalloc<State>(M, 1);
  if (!U.dP || !U.dS) return bail(fail(IBB_E_NOMEM, "device allocation failed"));
  R->dP = U.dP;
  R->dS = U.dS;
  R->opts = U.opts;
  U.term_cache = true;
  if ((st = run_setup(U, prob)) != IBB_OK) return bail(st);
  Params& P = R->P;
  const int n = P.n;

  // bound kernel shape (children per workgroup x waves per child), picked by the
  // autotuner below unless the caller forces one; every shape gives the same bits
  int bound_variant = -1;
  if (U.opts.bound_shape > 0) {
    bound_variant = U.opts.bound_shape - 1;
    if (bound_variant >= kNumBoundShapes || (P.prec32 && kBoundShapes[bound_variant].conc) ||
        (kBoundShapes[bound_variant].w > 1 && kBoundShapes[bound_variant].w > (n + kWave - 1) / kWave))
      return bail(fail(IBB_E_INVALID, "forced bound shape not available for this precision"));
  }
  const int n_tiles = (n + kWave - 1) / kWave;
  const uint64_t tune_key = ((uint64_t)P.family << 52) | ((uint64_t)std::min(P.select_k, 1 << 11) << 40) |
                            ((uint64_t)std::min(n_tiles, 1 << 20) << 8) | ((uint64_t)P.m << 1) | (uint64_t)(P.prec32 != 0);
  if (P.incremental || P.tape) bound_variant = -1;   // the tape kernels have one shape
  else if (bound_variant < 0) bound_variant = tuned_shape(tune_key);
  if (!P.incremental && !P.tape && bound_variant < 0) {
    st = autotune_bound(U, n_tiles, bound_variant);
    if (st != IBB_OK) return bail(st);
    store_tuned_shape(tune_key, bound_variant);
  }
  R->info.bound_shape = bound_variant;
  if ((st = run_sweeps(U, bound_variant)) != IBB_OK) return bail(st);
  if ((st = run_finish(U)) != IBB_OK) return bail(st);
  *out = R;
  return (ibb_status)R->info.status;
}

ibb_status ibb_solve(const ibb_problem* prob, const ibb_options* opts, const ibb_allocator* alloc, void* hip_stream,
                     ibb_result** out) {
  try {
    return solve_impl(prob, opts, alloc, hip_stream, out);
  } catch (...) {
    return fail(IBB_E_INTERNAL, "exception in ibb_solve");
  }
}

ibb_status ibb_sweep(ibb_result* R, int64_t n_sweeps, void* hip_stream) {
  try {
    if (!R) return fail(IBB_E_INVALID, "result is NULL");
    if (n_sweeps < 0) return fail(IBB_E_INVALID, "n_sweeps < 0");
    if (!R->dS || !R->dP) return fail(IBB_E_INVALID, "result holds no device state");
    if (R->broken) return fail(IBB_E_INVALID, "an earlier ibb_sweep on this result failed; free it");
    Run U;
    U.R = R;
    U.dP = R->dP;
    U.dS = R->dS;
    U.opts = R->opts;
    Mem& M = R->mem;
    M.stream = (hipStream_t)hip_stream;
    Params& P = R->P;
    HIPCHK(hipMemcpyAsync(&U.hs, U.dS, sizeof(State), hipMemcpyDeviceToHost, M.stream));
    HIPCHK(hipStreamSynchronize(M.stream));
    if (n_sweeps == 0 || U.hs.stop == STOP_CONVERGED || U.hs.stop == STOP_EMPTY || U.hs.stop == STOP_CAPACITY ||
        U.hs.stop == STOP_INTERNAL)
      return (ibb_status)R->info.status;
    const double before = R->info.seconds;
    U.t0 = std::chrono::steady_clock::now();
    U.n_keys = U.hs.n_keys;
    U.sweeps = U.hs.sweeps;
    U.pending = U.hs.pending != 0;
    P.max_sweeps = U.hs.sweeps + n_sweeps;
    ibb_status st = push_params(M, P, U.dP);
    if (st != IBB_OK) return st;
    const int32_t running = RUNNING;
    HIPCHK(hipMemcpyAsync(&U.dS->stop, &running, sizeof(int32_t), hipMemcpyHostToDevice, M.stream));
    HIPCHK(hipStreamSynchronize(M.stream));
    // from here on a failure leaves the run half-way: the result is marked unusable
    // (its info is kept, its boxes are dropped) and only ibb_result_info and
    // ibb_result_free accept it afterwards
    auto broken = [&](ibb_status e) {
      R->broken = true;
      R->n_boxes = 0;
      R->info.n_boxes = 0;
      R->info.status = e;
      return e;
    };
    if ((st = run_sweeps(U, R->info.bound_shape)) != IBB_OK) return broken(st);
    M.put(R->flo); M.put(R->seq); M.put(R->ref); M.put(R->r); M.put(R->wmax);
    R->flo = nullptr; R->seq = nullptr; R->ref = nullptr; R->r = nullptr; R->wmax = nullptr;
    if ((st = run_finish(U)) != IBB_OK) return broken(st);
    R->info.seconds += before;
    return (ibb_status)R->info.status;
  } catch (...) {
    return fail(IBB_E_INTERNAL, "exception in ibb_sweep");
  }
}

ibb_status ibb_result_info(const ibb_result* res, ibb_info* info) {
  if (!res || !info) return fail(IBB_E_INVALID, "NULL argument");
  *info = res->info;
  return IBB_OK;
}

ibb_status ibb_result_boxes(const ibb_result* res, double* lo, double* hi, double* f_lo_per_box, int64_t* seq,
                            int64_t capacity, int64_t* written) {
  if (!res || capacity < 0) return fail(IBB_E_INVALID, "bad argument");
  if (res->broken) return fail(IBB_E_INVALID, "an ibb_sweep on this result failed; its boxes are gone");
  ibb_result* R = const_cast<ibb_result*>(res);
  const int64_t k = std::min(capacity, R->n_boxes);
  if (written) *written = k;
  if (k == 0) return IBB_OK;
  Mem& M = R->mem;
  const int n = R->P.n;
  // copies on the result's own stream (never a legacy-stream copy: another
  // thread of the process may be capturing a graph), serialised with captures
  std::lock_guard<std::mutex> lk(g_capture_mu);
  if (f_lo_per_box) HIPCHK(hipMemcpyAsync(f_lo_per_box, R->flo, k * sizeof(double), hipMemcpyDeviceToHost, M.stream));
  if (seq) HIPCHK(hipMemcpyAsync(seq, R->seq, k * sizeof(int64_t), hipMemcpyDeviceToHost, M.stream));
  if (lo || hi) {
    double* dlo = dalloc<double>(M, k * n);
    double* dhi = dalloc<double>(M, k * n);
    if (!dlo || !dhi) return fail(IBB_E_NOMEM, "device allocation failed");
    hipLaunchKernelGGL(k_rows_out, dim3((unsigned)std::min<int64_t>(k, 65535)), dim3(256), 0, M.stream, R->dP, k, R->ref,
                       R->r, dlo, dhi);
    HIPCHK(hipGetLastError());
    if (lo) HIPCHK(hipMemcpyAsync(lo, dlo, k * n * sizeof(double), hipMemcpyDeviceToHost, M.stream));
    if (hi) HIPCHK(hipMemcpyAsync(hi, dhi, k * n * sizeof(double), hipMemcpyDeviceToHost, M.stream));
    M.put(dlo);
    M.put(dhi);
  }
  HIPCHK(hipStreamSynchronize(M.stream));
  return IBB_OK;
}

ibb_status ibb_result_trace(const ibb_result* res, double* gub, int64_t* n_inserted, int64_t* n_live,
                            int64_t* selected_seq, int64_t capacity, int64_t* written) {
  if (!res || capacity < 0) return fail(IBB_E_INVALID, "bad argument");
  const int64_t k = std::min<int64_t>(capacity, (int64_t)res->tr_gub.size());
  for (int64_t i = 0; i < k; ++i) {
    if (gub) gub[i] = res->tr_gub[i];
    if (n_inserted) n_inserted[i] = res->tr_nsurv[i];
    if (n_live) n_live[i] = res->tr_nlive[i];
    if (selected_seq) selected_seq[i] = res->tr_sel[i];
  }
  if (written) *written = k;
  return IBB_OK;
}

void ibb_result_free(ibb_result* res) {
  if (!res) return;
  std::lock_guard<std::mutex> lk(g_capture_mu);
  (void)hipStreamSynchronize(res->mem.stream);
  res->mem.release_all();
  (void)hipStreamSynchronize(res->mem.stream);
  delete res;
}

ibb_status ibb_eval_boxes(const ibb_problem* prob, int32_t precision, int64_t nb, const double* d_lo, const double* d_hi,
                          double* d_F, double* d_ub_mid, uint8_t* d_mono_prune, double* d_G, void* hip_stream) {
  ibb_status st = validate(prob);
  if (st != IBB_OK) return st;
  if (precision != IBB_FP64 && precision != IBB_FP32_BULK) return fail(IBB_E_INVALID, "unknown precision");
  const bool p32 = precision == IBB_FP32_BULK;
  if (p32 && !fp32_safe(prob))
    return fail(IBB_E_INVALID, "coefficient or domain magnitudes too large for single-precision bounds");
  if (nb < 0) return fail(IBB_E_INVALID, "nb < 0");
  if (p32 && prob->family == IBB_TAPE) return fail(IBB_E_INVALID, "the generic family (IBB_TAPE) is FP64 only");
  if (nb == 0) return IBB_OK;
  if (!d_lo || !d_hi || !d_F || !d_ub_mid || !d_mono_prune) return fail(IBB_E_INVALID, "NULL device array");
  Mem M;
  M.stream = (hipStream_t)hip_stream;
  Params P{};
  st = upload_problem(M, prob, P, p32);
  if (st != IBB_OK) { M.release_all(); return st; }
  if (P.tape) {   // one thread per box; right products of the product reductions in a workspace
    TapeDev T;
    int64_t at = 0;
    if ((st = parse_tape(prob, T, at)) != IBB_OK) { M.release_all(); return st; }
    I* ws = nullptr;
    if (T.nprod > 0) {
      const int64_t cnt = nb * T.nprod * (int64_t)prob->n;
      if (cnt * (int64_t)sizeof(I) > ((int64_t)8 << 30)) { M.release_all(); return fail(IBB_E_CAPACITY, "too many boxes for the workspace"); }
      ws = dalloc<I>(M, cnt);
      if (!ws) { M.release_all(); return fail(IBB_E_NOMEM, "device allocation failed"); }
    }
    Params* dP = dalloc<Params>(M, 1);
    if (!dP) { M.release_all(); return fail(IBB_E_NOMEM, "device allocation failed"); }
    if (hipMemcpyAsync(dP, &P, sizeof(Params), hipMemcpyHostToDevice, M.stream) != hipSuccess) {
      M.release_all();
      return fail(IBB_E_DEVICE, "copy failed");
    }
    const int64_t tb = (nb + 255) / 256;
    if (tb > 0x7fffffff) { M.release_all(); return fail(IBB_E_CAPACITY, "too many boxes"); }
    hipLaunchKernelGGL(k_eval_tape, dim3((unsigned)tb), dim3(256), 0, M.stream, dP, nb, d_lo, d_hi, d_F, d_ub_mid,
                       d_mono_prune, d_G, ws);
    const hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(M.stream);
    M.release_all();
    if (e != hipSuccess) return fail(IBB_E_DEVICE, std::string("eval launch: ") + hipGetErrorString(e));
    return IBB_OK;
  }
  Params* dP = dalloc<Params>(M, 1);
  if (!dP) { M.release_all(); return fail(IBB_E_NOMEM, "device allocation failed"); }
  if (hipMemcpyAsync(dP, &P, sizeof(Params), hipMemcpyHostToDevice, M.stream) != hipSuccess) {
    M.release_all();
    return fail(IBB_E_DEVICE, "copy failed");
  }
  const int64_t blocks = (nb + kBoundWaves - 1) / kBoundWaves;
  if (blocks > 0x7fffffff) { M.release_all(); return fail(IBB_E_CAPACITY, "too many boxes"); }
  dispatch_family(P.family, [&](auto fam) {
    if (p32)
      hipLaunchKernelGGL(k_eval_boxes32<decltype(fam)::value>, dim3((unsigned)blocks), dim3(kWave * kBoundWaves), 0,
                         M.stream, dP, nb, d_lo, d_hi, d_F, d_ub_mid, d_mono_prune, d_G);
    else
      hipLaunchKernelGGL(k_eval_boxes<decltype(fam)::value>, dim3((unsigned)blocks), dim3(kWave * kBoundWaves), 0,
                         M.stream, dP, nb, d_lo, d_hi, d_F, d_ub_mid, d_mono_prune, d_G);
  });
  hipError_t e = hipGetLastError();
  // the host copy of P is gone after return; the device copy was enqueued before the kernel
  (void)hipStreamSynchronize(M.stream);
  M.release_all();
  if (e != hipSuccess) return fail(IBB_E_DEVICE, std::string("eval launch: ") + hipGetErrorString(e));
  return IBB_OK;
}

ibb_status ibb_eval_boxes_noalloc(const ibb_problem* prob, int32_t precision, int64_t nb, const double* d_lo,
                                  const double* d_hi, double* d_F, double* d_ub_mid, uint8_t* d_mono_prune,
                                  double* d_G, void* hip_stream) {
  ibb_status st = validate(prob);
  if (st != IBB_OK) return st;
  if (precision != IBB_FP64 && precision != IBB_FP32_BULK) return fail(IBB_E_INVALID, "unknown precision");
  const bool p32 = precision == IBB_FP32_BULK;
  if (p32 && !fp32_safe(prob))
    return fail(IBB_E_INVALID, "coefficient or domain magnitudes too large for single-precision bounds");
  if (nb < 0) return fail(IBB_E_INVALID, "nb < 0");
  if (prob->family == IBB_TAPE)
    return fail(IBB_E_INVALID, "ibb_eval_boxes_noalloc takes the fixed families (the generic one needs a workspace)");
  const ScratchLayout lay = scratch_layout(prob, p32);
  if (lay.total > kScratchBytes)
    return fail(IBB_E_CAPACITY, "problem needs " + std::to_string(lay.total) + " bytes of the fixed device array (" +
                                    std::to_string(kScratchBytes) + " bytes): n too large for ibb_eval_boxes_noalloc");
  if (nb == 0) return IBB_OK;
  if (!d_lo || !d_hi || !d_F || !d_ub_mid || !d_mono_prune) return fail(IBB_E_INVALID, "NULL device array");
  const int64_t blocks = (nb + kBoundWaves - 1) / kBoundWaves;
  if (blocks > 0x7fffffff) return fail(IBB_E_CAPACITY, "too many boxes");
  std::lock_guard<std::mutex> serial(g_scratch_call_mu);   // one call at a time uses the array
  unsigned char* base = nullptr;
  if ((st = scratch_for_current_device(&base)) != IBB_OK) return st;
  const hipStream_t stream = (hipStream_t)hip_stream;
  const int n = prob->n;
  const bool chain = prob->family == IBB_CHAIN;
  Params P{};
  P.family = prob->family;
  P.n = n;
  P.nl = (double*)(base + lay.nl);
  P.u = (double*)(base + lay.u);
  P.prec32 = p32 ? 1 : 0;
  P.incremental = 0;
  double* coef = (double*)(base + lay.coef);
  HIPCHK(hipMemcpyAsync(base + lay.nl, prob->lower, n * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(base + lay.u, prob->upper, n * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(coef, prob->coef, prob->coef_len * sizeof(double), hipMemcpyHostToDevice, stream));
  const int cblocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_negate, dim3(cblocks), dim3(256), 0, stream, n, (double*)(base + lay.nl));
  if (chain) {
    CoefChain* c = (CoefChain*)(base + lay.tab);
    CoefChain32* c32 = p32 ? (CoefChain32*)(base + lay.tab32) : nullptr;
    hipLaunchKernelGGL(k_setup_chain, dim3(cblocks), dim3(256), 0, stream, n, coef, c, c32);
    P.chain = c;
    P.chain32 = c32;
  } else {
    CoefSep* c = (CoefSep*)(base + lay.tab);
    CoefSep32* c32 = p32 ? (CoefSep32*)(base + lay.tab32) : nullptr;
    hipLaunchKernelGGL(k_setup_sep, dim3(cblocks), dim3(256), 0, stream, n, prob->family, coef, c, c32);
    P.sep = c;
    P.sep32 = c32;
  }
  Params* dP = (Params*)base;
  HIPCHK(hipMemcpyAsync(dP, &P, sizeof(Params), hipMemcpyHostToDevice, stream));
  dispatch_family(P.family, [&](auto fam) {
    if (p32)
      hipLaunchKernelGGL(k_eval_boxes32<decltype(fam)::value>, dim3((unsigned)blocks), dim3(kWave * kBoundWaves), 0,
                         stream, dP, nb, d_lo, d_hi, d_F, d_ub_mid, d_mono_prune, d_G);
    else
      hipLaunchKernelGGL(k_eval_boxes<decltype(fam)::value>, dim3((unsigned)blocks), dim3(kWave * kBoundWaves), 0,
                         stream, dP, nb, d_lo, d_hi, d_F, d_ub_mid, d_mono_prune, d_G);
  });
  const hipError_t e = hipGetLastError();
  // P (host) and the caller's host arrays are read by the copies above, and the
  // next call rewrites the array: wait for the work before returning
  const hipError_t es = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(IBB_E_DEVICE, std::string("eval launch: ") + hipGetErrorString(e));
  if (es != hipSuccess) return fail(IBB_E_DEVICE, std::string("eval: ") + hipGetErrorString(es));
  return IBB_OK;
}

ibb_status ibb_interval_op(int32_t op, int64_t count, const double* d_a, const double* d_b, double* d_out,
                           void* hip_stream) {
  if (op < 0 || op > 13) return fail(IBB_E_INVALID, "unknown op");
  if (count < 0) return fail(IBB_E_INVALID, "count < 0");
  if (count == 0) return IBB_OK;
  const bool binary = op <= 3;
  if (!d_a || !d_out || (binary && !d_b)) return fail(IBB_E_INVALID, "NULL device array");
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7fffffff) return fail(IBB_E_CAPACITY, "count too large");
  hipLaunchKernelGGL(k_interval_op, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, op, count, d_a,
                     binary ? d_b : nullptr, d_out);
  HIPCHK(hipGetLastError());
  return IBB_OK;
}

ibb_status ibb_point_trig(int32_t fn, int64_t count, const double* d_y, double* d_out, void* hip_stream) {
  if (fn != 0 && fn != 1) return fail(IBB_E_INVALID, "fn must be 0 (cos) or 1 (sin)");
  if (count < 0) return fail(IBB_E_INVALID, "count < 0");
  if (count == 0) return IBB_OK;
  if (!d_y || !d_out) return fail(IBB_E_INVALID, "NULL device array");
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7fffffff) return fail(IBB_E_CAPACITY, "count too large");
  hipLaunchKernelGGL(k_point_trig, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, fn, count, d_y, d_out);
  HIPCHK(hipGetLastError());
  return IBB_OK;
}

ibb_status ibb_interval_op32(int32_t op, int64_t count, const float* d_a, const float* d_b, float* d_out,
                             void* hip_stream) {
  if (!(op == 0 || op == 1 || op == 2 || op == 5 || op == 6 || op == 8 || op == 9 || op == 10))
    return fail(IBB_E_INVALID, "op not available in single precision");
  if (count < 0) return fail(IBB_E_INVALID, "count < 0");
  if (count == 0) return IBB_OK;
  const bool binary = op <= 2;
  if (!d_a || !d_out || (binary && !d_b)) return fail(IBB_E_INVALID, "NULL device array");
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7fffffff) return fail(IBB_E_CAPACITY, "count too large");
  hipLaunchKernelGGL(k_interval_op32, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, op, count, d_a,
                     binary ? d_b : nullptr, d_out);
  HIPCHK(hipGetLastError());
  return IBB_OK;
}

ibb_status ibb_point_trig32(int32_t fn, int64_t count, const float* d_y, float* d_out, void* hip_stream) {
  if (fn != 0 && fn != 1) return fail(IBB_E_INVALID, "fn must be 0 (cos) or 1 (sin)");
  if (count < 0) return fail(IBB_E_INVALID, "count < 0");
  if (count == 0) return IBB_OK;
  if (!d_y || !d_out) return fail(IBB_E_INVALID, "NULL device array");
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7fffffff) return fail(IBB_E_CAPACITY, "count too large");
  hipLaunchKernelGGL(k_point_trig32, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, fn, count, d_y,
                     d_out);
  HIPCHK(hipGetLastError());
  return IBB_OK;
}

}  // extern "C"

#include "serve.inc"
