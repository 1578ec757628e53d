/*
 * ibb.h -- C ABI of libibb: rigorous interval branch-and-bound minimisation of a
 * closed-form f over a box, on AMD MI355X (gfx950).
 *
 * Method: Zhang, Shan & Cagan, "Global optimization tailored for GPUs: complete
 * and rigorous search for large-scale nonlinear minimization" (arXiv 2507.01770).
 * The problem is Eqs. (1)-(2) (minimise f subject to l <= x <= u); the iteration
 * is Sec. 3.1 (select the region with the smallest lower bound, sample it to
 * update GUB, remove regions whose lower bound exceeds GUB, partition the
 * selected region and rule out subregions by the cutoff and first-order tests,
 * insert the rest, stop, output [GLB, GUB] and the regions); partitioning uses
 * the variable cycling of Sec. 3.2; bounds are natural interval extensions with
 * outward rounding (Sec. 2.1, Eqs. (3)-(6)).
 *
 * Conventions (every entry point):
 *   - nothing throws across the ABI; every call returns an ibb_status and, on an
 *     error, leaves a message for ibb_last_error() (per calling thread);
 *   - problem arrays are host memory and are copied; the caller keeps ownership;
 *   - "d_" pointers are device memory owned by the caller;
 *   - work is enqueued on the given HIP stream (NULL = the null stream);
 *     ibb_solve synchronises that stream before it returns, the kernel-level
 *     entry points do not;
 *   - device memory the library needs is taken from the ibb_allocator when one is
 *     given (for example PyTorch's caching allocator), else from hipMalloc.
 */
#ifndef IBB_H
#define IBB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IBB_OK = 0,
  IBB_NOT_CONVERGED = 1, /* a budget ended the run; [f_lo, f_hi] and the boxes are still rigorous */
  IBB_PENDING = 2,
  IBB_E_INVALID = -1,    /* bad argument (see ibb_last_error) */
  IBB_E_NOMEM = -2,      /* device or host allocation failed */
  IBB_E_DEVICE = -3,     /* a HIP call failed */
  IBB_E_CAPACITY = -4,   /* a size exceeds what the library supports */
  IBB_E_INTERNAL = -5    /* the live list became empty, a sweep would have passed the row or key
                            capacity sized for it (a guard: the library grows both before every chunk),
                            or the selection counted live boxes but found none to take (a guard) */
} ibb_status;

/* Objective families (closed forms with per-coordinate coefficients).
 *   IBB_SEP_COS      f = sum_i a_i (x_i - c_i)^2 + b_i (1 - cos(2 pi k_i (x_i - c_i)))
 *                    coef = a[n], b[n], k[n], c[n]        (k_i positive integers)
 *   IBB_CHAIN        f = sum_{i<n-1} alpha_i (x_{i+1} - x_i^2)^2 + beta_i (x_i - 1)^2
 *                    coef = alpha[n-1], beta[n-1]         (n >= 2)
 *   IBB_SEP_ABS_SIN2 f = sum_i s_i |x_i - c_i| + b_i sin^2(pi k_i (x_i - c_i))
 *                    coef = s[n], b[n], k[n], c[n]        (k_i positive integers)
 * The interval extension of each family follows a fixed expression tree and a
 * fixed summation order (term i in slot i mod 64, slots summed left to right,
 * then folded with strides 32..1), which makes the bounds reproducible bit for
 * bit.  cos and sin are evaluated as cos(2 pi y), sin(2 pi y) of y = k (x - c)
 * (or k/2 (x - c)), so the argument reduction is exact. */
/* IBB_TAPE: a generic closed-form f given as an expression tape in coef (the
 * benchmark functions of the paper's SI Appendix A, Eqs. S1-S21, and Appendix D,
 * Eq. S22, are all of this form):  f = g(R_1, ..., R_K), each R_k a sum (kind 0)
 * or a product (kind 1) over i in a range of an element program in x_i,
 * x_{i+1} (sums only, ranges ending by n - 1), i + 1 and coefficient columns;
 * g a scalar program of the R_k and constants.  coef (doubles):
 *   [1, K, Q, C]                              K <= 8 reductions, 1 <= Q <= 32
 *   per reduction: [kind, s_off, s_end, t_off, t_end, L] then L ops (1..32):
 *       i runs from s_off + (s_end ? n : 0) to t_off + (t_end ? n : 0), exclusive
 *   Q scalar ops, the last one's value being f
 *   C coefficient columns of n values (coef_len must match exactly)
 * An op is 5 doubles [code, a, b, c_lo, c_hi]; a, b index earlier ops of the
 * same program.  Codes: 0 constant [c_lo, c_hi]; 1 x_i; 2 x_{i+1}; 3 column a
 * at i; 4 a + b; 5 a - b; 6 a * b; 7 a / b (= a * (1/b), Eq. (6)); 8 -a; 9 a^2;
 * 10 sqrt a; 11 exp a; 12 cos a; 13 sin a; 14 cos(2 pi a); 15 sin(2 pi a);
 * 16 |a|; 17 reduction a (scalar program only); 18 i + 1 (element programs
 * only; 1, 2, 3 likewise).  Every operation rounds outward (Sec. 2.1); the
 * gradient for the first-order test (Sec. 3.1) comes from forward tangents in
 * the element programs and adjoints of the scalar program (the order of
 * every sum and product is fixed by the library and the same in the checks).
 * A malformed tape is refused with IBB_E_INVALID.  The generic family is
 * bounded in full (no incremental bounds), one box per sweep, FP64. */
typedef enum { IBB_SEP_COS = 1, IBB_CHAIN = 2, IBB_SEP_ABS_SIN2 = 3, IBB_TAPE = 4 } ibb_family;

/* IBB_FP64: every box is bounded in double precision, as in the paper's
 * experiments (Sec. 4).
 * IBB_FP32_BULK (an addition to the paper's method): a single-precision filter
 * runs first on each child while it pays: the child's box is enclosed in
 * floats, F and the first-order test are evaluated in single precision with
 * outward rounding, and a child whose float lower bound exceeds the GUB at the
 * start of the sweep, or that fails the float first-order test, is discarded
 * without its double-precision bound.  Other children are bounded in FP64 as
 * usual, and midpoint upper bounds are always FP64.  The filter runs in a sweep
 * only while it discards at least half of the children (after a sweep where it
 * discarded less it is off for 2, 4, ..., 64 sweeps, and it is turned on when
 * half of an FP64 sweep's children were discarded); it stays off for problems
 * whose magnitudes could overflow single precision.  Results remain rigorous
 * and deterministic but are not the FP64 run's bit for bit. */
typedef enum { IBB_FP64 = 0, IBB_FP32_BULK = 1 } ibb_precision;

typedef struct {
  int32_t family;        /* ibb_family */
  int32_t n;             /* dimension, 1 <= n <= 1<<24 (CHAIN: n >= 2) */
  const double* coef;    /* host, coef_len values, layout above */
  int64_t coef_len;      /* 4n (SEP_COS, SEP_ABS_SIN2), 2(n-1) (CHAIN), the tape's length (TAPE) */
  const double* lower;   /* host [n]: l, finite */
  const double* upper;   /* host [n]: u, finite, l_i < u_i */
  double tol_f;          /* stop once GUB - GLB (rounded up) <= tol_f; > 0 */
  double tol_x;          /* optional: also require every box width < tol_x (0 = off) */
} ibb_problem;

typedef struct {
  int32_t precision;     /* ibb_precision; default IBB_FP64 */
  int32_t split_dims;    /* M: coordinates bisected per selected box, 1..16; default 10 */
  int32_t select_k;      /* K: boxes selected per sweep, 1..1024; default 1 (the paper's choice: Sec. 3.1
                            selects the region with the smallest lower bound).  K > 1 takes the K
                            smallest (lower bound, insertion number) at once, bounds the children of
                            all K before GUB is updated and inserts them in (rank, child index)
                            order; K * 2^split_dims <= 2^24.  ibb_solve and ibb_sweep only
                            (ibb_solve_batch and the server return IBB_E_INVALID for K > 1) */
  int32_t deterministic; /* results independent of scheduling; default 1 (always honoured) */
  int64_t max_sweeps;    /* budget; default 1,000,000 */
  int64_t max_live_boxes;/* budget on the live list; default 1<<26 */
  double time_limit_s;   /* budget; <= 0 means none; default 0 */
  int32_t profile;       /* 1: time every sweep kernel with HIP events (ibb_info t_* fields); default 0 */
  int32_t bound_shape;   /* 0 (default): the autotuner picks the bound kernel's shape; k = 1..5 forces
                            shape k-1 (W waves per child, concurrent midpoint waves or not):
                            0 {1, yes}, 1 {2, yes}, 2 {1, no}, 3 {2, no}, 4 {4, no}.  Every shape gives
                            the same results; IBB_E_INVALID for a shape with concurrent midpoint
                            waves under IBB_FP32_BULK or with W above ceil(n / 64).
                            Applies to full bounds only (incremental = 0) */
  int32_t incremental;   /* 1 (default): incremental child bounds.  A child differs from the selected
                            box only on the split coordinates, so every term of f that involves none
                            of them is shared: the selection workgroup sums those once per sweep (in
                            the canonical slot order, the others left out) and bounds each child as
                            that sum plus its affected terms in increasing index; the midpoint upper
                            bound likewise.  The same enclosures up to the order of the additions,
                            O(n + 2^m m) work per sweep instead of O(2^m n).  0: every child is
                            bounded over all n terms (the FP32 filter and bound_shape apply only here;
                            IBB_E_INVALID for incremental = 1 with IBB_FP32_BULK or a bound_shape) */
  int32_t pieces;        /* subintervals per split coordinate: 2 (default; 0 means 2): bisection at the
                            midpoint; 4: the schedule of the paper's experiments (Sec. 4), each of the
                            split_dims cycled coordinates cut into four equal pieces (Sec. 3.2,
                            Eqs. (8)-(11): digit j of the child index in base 4 picks the piece of the
                            j-th coordinate), 4^split_dims children per sweep.  4 needs diag_samples
                            in 1..16, incremental = 1, select_k = 1, IBB_FP64, split_dims <= 12 */
  int32_t diag_samples;  /* 0 with pieces = 2 (the child midpoint is the one sample); with pieces = 4,
                            S sample points per child on its diagonal, cutting it into S + 1 equal
                            pieces (the paper uses 10); GUB starts at +inf and takes the smallest
                            sample upper bound.  The paper stops on region width: set tol_x = 1e-4
                            and a tol_f that never binds (e.g. 1e300) */
  int32_t reserved;      /* 0 */
} ibb_options;

typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* hip_stream);
  void (*free)(void* ctx, void* p, size_t bytes, void* hip_stream);
} ibb_allocator;

typedef struct {
  double f_lo, f_hi;          /* rigorous enclosure [GLB, GUB] of min f */
  int64_t n_boxes;            /* live boxes at the end (lower bound <= GUB) */
  int64_t sweeps;             /* iterations run */
  int64_t boxes_evaluated;    /* children bounded, plus the root */
  int64_t fp32_pruned;        /* children discarded by the FP32 filter (no FP64 bound formed) */
  int64_t fp64_confirmed;     /* boxes bounded in FP64 (boxes_evaluated - fp32_pruned) */
  double seconds;             /* wall time of ibb_solve */
  int32_t status;             /* IBB_OK or IBB_NOT_CONVERGED */
  int32_t fp32_sweeps;        /* sweeps in which the FP32 filter ran */
  int64_t ub_evaluated;       /* children whose midpoint upper bound was computed */
  /* filled when options.profile = 1: summed kernel times (ms) and launch counts of
     the sweeps that ran (launches after the stop are not counted) */
  double t_bound_ms, t_select_ms;
  int64_t n_bound_launches, n_select_launches;
  int32_t bound_shape;        /* shape of the bound kernel used (0..4, see ibb_options; -1: incremental) */
  int32_t stop_reason;        /* why the run ended: 1 converged, 2 max_sweeps, 3 max_live_boxes, 5 the time
                                 limit, 8 the server's memory budget (see ibb_server_create) */
  int64_t n_persistent_launches; /* with profile = 1: launches of the persistent sweep kernel (each runs a
                                    chunk of sweeps; their time is part of t_select_ms) */
  double t_persistent_ms;        /* with profile = 1: the persistent launches' summed time */
  int64_t n_persistent_sweeps;   /* with profile = 1: the sweeps those launches ran */
} ibb_info;

typedef struct ibb_result ibb_result;

/* Fill *opts with the defaults listed above. */
ibb_status ibb_options_default(ibb_options* opts);

/* Run the whole iteration (Sec. 3.1) on the device.  On IBB_OK or
 * IBB_NOT_CONVERGED, *out owns the result until ibb_result_free.  alloc may be
 * NULL.  Validation failures (IBB_E_INVALID): family unknown, n out of range,
 * coef_len mismatch, non-finite or |value| > 1e15 coefficients or bounds,
 * l_i >= u_i, tol_f <= 0, k_i not a positive integer, split_dims or select_k out
 * of range. */
ibb_status ibb_solve(const ibb_problem* prob, const ibb_options* opts, const ibb_allocator* alloc,
                     void* hip_stream, ibb_result** out);

/* Continue a run: up to n_sweeps more sweeps (Sec. 3.1) on the state that res
 * keeps on the device, for instance after ibb_solve stopped at max_sweeps or the
 * time limit.  The list, GUB, rows and trace continue exactly where they were,
 * so ibb_solve with budget a then ibb_sweep(b) gives the same run as ibb_solve
 * with budget a + b.  Updates res (info, boxes, trace) and returns its status:
 * IBB_OK once converged (a converged result is left as it is), else
 * IBB_NOT_CONVERGED.  Runs on hip_stream and synchronises it.
 * Failure: an error returned after the sweeps started (a refused allocation, a
 * device error, an internal stop) leaves the run half-way: the result is then
 * marked unusable, its info keeps the error as status and no boxes; further
 * ibb_sweep and ibb_result_boxes calls on it return IBB_E_INVALID, and
 * ibb_result_info and ibb_result_free still work.  When the list or row arrays
 * have to grow, every new block is allocated before anything is copied or
 * freed, so a refused allocation leaves the arrays as they were. */
ibb_status ibb_sweep(ibb_result* res, int64_t n_sweeps, void* hip_stream);

/* The output of the iteration (Sec. 3.1, output: the enclosure [GLB, GUB] of the
 * global minimum and the regions left in the list) and the run's counters. */
ibb_status ibb_result_info(const ibb_result* res, ibb_info* info);

/* The regions of the output (Sec. 3.1): copy up to `capacity` live boxes
 * (ordered by insertion number) to host arrays lo, hi ([box][n], row-major),
 * their lower bounds of f and insertion numbers (seq: an addition to the
 * paper's output, the order in which the boxes entered the list, which the
 * selection uses to break ties); any output pointer may be NULL.  *written
 * receives the count.  IBB_E_INVALID on a result marked unusable by a failed
 * ibb_sweep. */
ibb_status ibb_result_boxes(const ibb_result* res, double* lo, double* hi, double* f_lo_per_box,
                            int64_t* seq, int64_t capacity, int64_t* written);

/* Per-sweep record (for comparisons with a reference implementation): GUB after
 * the sweep, children inserted, live boxes after the cutoff, insertion number
 * of the first selected parent.  Host arrays; *written receives the count. */
ibb_status ibb_result_trace(const ibb_result* res, double* gub, int64_t* n_inserted, int64_t* n_live,
                            int64_t* selected_seq, int64_t capacity, int64_t* written);

/* Release a result and every block of device memory it holds (through the
 * allocator it was created with). */
void ibb_result_free(ibb_result* res);

/* Bound nb boxes given in device memory (d_lo, d_hi: [nb][n] row-major):
 * d_F[nb][2] receives the enclosure of f over each box, d_ub_mid[nb] the upper
 * bound of f at the box midpoint (0.5 lo + 0.5 hi rounded up), d_mono_prune[nb]
 * 1 when the first-order test of Sec. 3.1 discards the box (some DLB_j > 0 with
 * x_j^lo != l_j, or some DUB_j < 0 with x_j^hi != u_j), and d_G (may be NULL)
 * [nb][n][2] the enclosures of the partial derivatives.  With precision
 * IBB_FP32_BULK, F, the test and G are the single-precision filter's (over the
 * box enclosed in floats, converted exactly to double) and d_ub_mid stays FP64;
 * IBB_E_INVALID if the magnitudes could overflow single precision. */
ibb_status ibb_eval_boxes(const ibb_problem* prob, int32_t precision, int64_t nb, const double* d_lo,
                          const double* d_hi, double* d_F, double* d_ub_mid, uint8_t* d_mono_prune,
                          double* d_G, void* hip_stream);

/* ibb_eval_boxes for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, kernels and results, bit for bit, but the problem's coefficient
 * records, its bounds and the kernel parameters go into one fixed device array
 * of 16 MiB that the library holds on each GPU it runs on until the process
 * ends.  The call makes no device allocation and frees nothing.  The inputs
 * d_lo, d_hi and the outputs are the caller's, as for ibb_eval_boxes.
 * Limit: the problem must fit the array (144 bytes per coordinate for the
 * separable families with IBB_FP32_BULK, about 116,000 coordinates; 96 bytes,
 * about 174,000, in FP64; less for the chained family); a larger one gives
 * IBB_E_CAPACITY before any device work.  The array belongs to the current
 * device (hipGetDevice); calls are serialised inside the library, each one
 * rewrites the array completely and returns when its bounds are written (it
 * synchronises hip_stream), so the array's earlier contents never matter. */
ibb_status ibb_eval_boxes_noalloc(const ibb_problem* prob, int32_t precision, int64_t nb, const double* d_lo,
                                  const double* d_hi, double* d_F, double* d_ub_mid, uint8_t* d_mono_prune,
                                  double* d_G, void* hip_stream);

/* Elementwise interval operations with outward rounding (Sec. 2.1, Eqs. (3)-(6)),
 * for testing the arithmetic.  d_a, d_b, d_out: device [count][2] (lo, hi).
 * op: 0 add, 1 sub, 2 mul, 3 div (= a * (1/b), Eq. (6)), 4 sqrt, 5 sqr, 6 abs,
 * 7 reciprocal, 8 cos(2 pi a), 9 sin(2 pi a), 10 derivative of |.|, 11 exp,
 * 12 cos(a), 13 sin(a) (a in radians: cos / sin(2 pi y) of y = a [1 / (2 pi)]).
 * Unary ops ignore d_b (may be NULL).  A divisor that contains 0 gives
 * [-inf, +inf]. */
ibb_status ibb_interval_op(int32_t op, int64_t count, const double* d_a, const double* d_b, double* d_out,
                           void* hip_stream);

/* Point enclosures: d_out[count][2] receives [lo, hi] around cos(2 pi y)
 * (fn = 0) or sin(2 pi y) (fn = 1) for each double d_y[i]. */
ibb_status ibb_point_trig(int32_t fn, int64_t count, const double* d_y, double* d_out, void* hip_stream);

/* Single-precision counterparts, for testing the FP32 filter's arithmetic
 * (round-up mode on the negated lower endpoint, so +, -, x and sqr give the
 * tightest float enclosure).  d_a, d_b, d_out: device float [count][2] (lo, hi).
 * op as in ibb_interval_op, restricted to 0 add, 1 sub, 2 mul, 5 sqr, 6 abs,
 * 8 cos(2 pi a), 9 sin(2 pi a), 10 derivative of |.| (others: IBB_E_INVALID). */
ibb_status ibb_interval_op32(int32_t op, int64_t count, const float* d_a, const float* d_b, float* d_out,
                             void* hip_stream);
/* d_out[count][2] (float) receives [lo, hi] around cos(2 pi y) (fn = 0) or
 * sin(2 pi y) (fn = 1) for each float d_y[i]. */
ibb_status ibb_point_trig32(int32_t fn, int64_t count, const float* d_y, float* d_out, void* hip_stream);

/* ---- many problems at once ------------------------------------------------
 * Problems solved together share kernel launches: with incremental bounds (the
 * default) one persistent workgroup per problem runs a whole chunk of its
 * sweeps in one launch; with full bounds each sweep is two launches (selection,
 * one workgroup per problem; bounds, one wavefront per child of every problem,
 * any mix of families and sizes).  ibb_solve_batch captures a chunk as a HIP
 * graph and replays it while the set of problems is unchanged.  Each problem
 * keeps its own list, rows and GUB and follows exactly the iteration ibb_solve
 * runs for it, so its result is the same bit for bit alone or in any mix. */

/* Solve count problems together.  outs[i] receives problem i's result (NULL if
 * it failed; free each with ibb_result_free) and statuses[i] its status
 * (IBB_OK, IBB_NOT_CONVERGED or an error).  The call returns IBB_OK unless the
 * batch itself could not run; after such an error outs[i] still holds the
 * results of the problems that finished before it, which the caller frees.  The work runs on a stream of its own, ordered
 * after the work enqueued on hip_stream; the call returns when it is done and the
 * results are bound to hip_stream. */
ibb_status ibb_solve_batch(const ibb_problem* probs, int32_t count, const ibb_options* opts,
                           const ibb_allocator* alloc, void* hip_stream, ibb_result** outs, int32_t* statuses);

/* Continuous-batching server.  A host thread owned by the server runs batched
 * sweeps over the admitted problems in chunks of 8 sweeps (launched directly,
 * not captured: the caller's threads use the device meanwhile).  Between
 * chunks it retires finished problems and admits queued ones while a slot is
 * free (at most max_slots at once) and the device memory in use plus the new
 * problem's starting footprint stays within mem_budget_bytes.  A running problem
 * whose box list or rows must grow past the budget, or whose growth the
 * allocator refuses, is ended at its next sweep with IBB_NOT_CONVERGED and
 * stop_reason 8: its enclosure and boxes are rigorous, as after any budget.  A
 * problem whose result the server cannot form (an allocation at the end fails)
 * gets that error as its poll status; the other problems go on.  The server's
 * device work runs on a stream of its own, ordered after the work enqueued on
 * hip_stream when the server is created; results are handed over bound to
 * hip_stream (the caller keeps it alive until the last result from this server
 * is freed). */
typedef struct ibb_server ibb_server;
ibb_status ibb_server_create(size_t mem_budget_bytes, int32_t max_slots, const ibb_allocator* alloc,
                             void* hip_stream, ibb_server** out);
/* Copy a problem into the queue; *ticket identifies it.  Per-problem time limits
 * are not applied by the server (sweep and list budgets are).  IBB_E_CAPACITY if
 * the problem alone exceeds the memory budget. */
ibb_status ibb_server_submit(ibb_server* srv, const ibb_problem* prob, const ibb_options* opts, uint64_t* ticket);
/* IBB_PENDING while the problem is queued or running; once it has finished, the
 * call hands over the result (*out, owned by the caller) and returns its status;
 * a ticket is handed over once. */
ibb_status ibb_server_poll(ibb_server* srv, uint64_t ticket, ibb_result** out);
/* Counters: problems admitted, completed, the largest number run at once, queued now. */
ibb_status ibb_server_stats(ibb_server* srv, int64_t* admitted, int64_t* completed, int64_t* max_active,
                            int64_t* queued);
/* Stop the thread, drop problems still queued or running, free unclaimed results. */
ibb_status ibb_server_destroy(ibb_server* srv);

const char* ibb_status_string(ibb_status s);
const char* ibb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IBB_H */
