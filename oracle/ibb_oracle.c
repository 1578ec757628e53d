/*
 * ibb_oracle.c -- plain, slow, CPU reference ("oracle") for the interval
 * branch-and-bound sweep of Zhang, Shan & Cagan, "Global optimization tailored
 * for GPUs: complete and rigorous search for large-scale nonlinear
 * minimization" (arXiv 2507.01770).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links, imports or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no source with the GPU library.
 *
 * Every endpoint operation switches the x86 rounding mode with fesetround()
 * right before it and reads its operands through volatile copies, so the
 * compiler can neither fold nor move the arithmetic across the mode switch.
 * This is deliberately the most literal way to get IEEE directed rounding.
 *
 * What each part follows (paper section / equation):
 *   - interval +, -, x, / : Sec. 2.1, Eqs. (3)-(6); division is multiplication
 *     by the reciprocal interval, exactly as Eq. (6) writes it.
 *   - outward rounding (lower endpoint rounded down, upper rounded up): Sec. 2.1.
 *   - natural interval extension of f and of its first derivatives: Sec. 2.1
 *     and Sec. 3.1 ("Partition the selected region ..." and the first-order test).
 *   - the iteration (select smallest lower bound, sample, cut off regions whose
 *     lower bound exceeds GUB, partition with variable cycling, first-order
 *     test, insert, stop, output [GLB, GUB]): Sec. 3.1 and Sec. 3.2.
 * Readings of points the paper leaves open are listed in the design notes of
 * the repository; the ones that change numbers are restated where they apply.
 */
#include <fenv.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FENV_ACCESS ON

/* ------------------------------------------------------------------------- */
/* directed scalar operations                                                */
/* ------------------------------------------------------------------------- */

static double dn_add(double a, double b) { volatile double x = a, y = b; fesetround(FE_DOWNWARD); volatile double r = x + y; fesetround(FE_TONEAREST); return r; }
static double up_add(double a, double b) { volatile double x = a, y = b; fesetround(FE_UPWARD);   volatile double r = x + y; fesetround(FE_TONEAREST); return r; }
static double dn_sub(double a, double b) { volatile double x = a, y = b; fesetround(FE_DOWNWARD); volatile double r = x - y; fesetround(FE_TONEAREST); return r; }
static double up_sub(double a, double b) { volatile double x = a, y = b; fesetround(FE_UPWARD);   volatile double r = x - y; fesetround(FE_TONEAREST); return r; }
static double dn_mul(double a, double b) { volatile double x = a, y = b; fesetround(FE_DOWNWARD); volatile double r = x * y; fesetround(FE_TONEAREST); return r; }
static double up_mul(double a, double b) { volatile double x = a, y = b; fesetround(FE_UPWARD);   volatile double r = x * y; fesetround(FE_TONEAREST); return r; }
static double dn_div(double a, double b) { volatile double x = a, y = b; fesetround(FE_DOWNWARD); volatile double r = x / y; fesetround(FE_TONEAREST); return r; }
static double up_div(double a, double b) { volatile double x = a, y = b; fesetround(FE_UPWARD);   volatile double r = x / y; fesetround(FE_TONEAREST); return r; }
static double dn_sqrt(double a) { volatile double x = a; fesetround(FE_DOWNWARD); volatile double r = sqrt(x); fesetround(FE_TONEAREST); return r; }
static double up_sqrt(double a) { volatile double x = a; fesetround(FE_UPWARD);   volatile double r = sqrt(x); fesetround(FE_TONEAREST); return r; }

static double dmin(double a, double b) { return b < a ? b : a; }
static double dmax(double a, double b) { return b > a ? b : a; }

/* ------------------------------------------------------------------------- */
/* intervals                                                                 */
/* ------------------------------------------------------------------------- */

typedef struct { double lo, hi; } iv;

static iv mk(double lo, double hi) { iv r; r.lo = lo; r.hi = hi; return r; }
static iv entire(void) { return mk(-INFINITY, INFINITY); }
static int bad(iv a) { return isnan(a.lo) || isnan(a.hi); }
static iv fix(iv r) { return bad(r) ? entire() : r; }

/* Eq. (3) */
static iv iv_add(iv a, iv b) { return fix(mk(dn_add(a.lo, b.lo), up_add(a.hi, b.hi))); }
/* Eq. (4) */
static iv iv_sub(iv a, iv b) { return fix(mk(dn_sub(a.lo, b.hi), up_sub(a.hi, b.lo))); }
/* Eq. (5): min / max over the four endpoint products, each rounded outward */
static iv iv_mul(iv a, iv b) {
  double p[4] = { a.lo, a.lo, a.hi, a.hi }, q[4] = { b.lo, b.hi, b.lo, b.hi };
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < 4; ++i) {
    double l = dn_mul(p[i], q[i]), h = up_mul(p[i], q[i]);
    if (isnan(l) || isnan(h)) return entire();
    lo = dmin(lo, l);
    hi = dmax(hi, h);
  }
  return mk(lo, hi);
}
/* reciprocal of an interval not containing zero; otherwise the whole line */
static iv iv_recip(iv b) {
  if (!(b.lo > 0.0 || b.hi < 0.0)) return entire();
  return fix(mk(dn_div(1.0, b.hi), up_div(1.0, b.lo)));
}
/* Eq. (6): a / b = a * (1 / b) */
static iv iv_div(iv a, iv b) { return iv_mul(a, iv_recip(b)); }
/* square root on the non-negative part */
static iv iv_sqrt(iv a) {
  if (bad(a) || a.hi < 0.0) return entire();
  return mk(a.lo > 0.0 ? dn_sqrt(a.lo) : 0.0, up_sqrt(a.hi));
}
/* x^2 as a single operation (tighter than a*a when 0 lies inside) */
static iv iv_sqr(iv a) {
  if (a.lo >= 0.0) return fix(mk(dn_mul(a.lo, a.lo), up_mul(a.hi, a.hi)));
  if (a.hi <= 0.0) return fix(mk(dn_mul(a.hi, a.hi), up_mul(a.lo, a.lo)));
  double m = dmax(-a.lo, a.hi);
  return fix(mk(0.0, up_mul(m, m)));
}
static iv iv_abs(iv a) {
  if (a.lo >= 0.0) return a;
  if (a.hi <= 0.0) return mk(-a.hi, -a.lo);
  return mk(0.0, dmax(-a.lo, a.hi));
}
/* enclosure of the generalized derivative of |x| over a */
static iv iv_dabs(iv a) {
  if (a.lo > 0.0) return mk(1.0, 1.0);
  if (a.hi < 0.0) return mk(-1.0, -1.0);
  return mk(-1.0, 1.0);
}
static iv iv_scale(double s, iv a) { return iv_mul(mk(s, s), a); }
static iv iv_sub_s(iv a, double s) { return iv_sub(a, mk(s, s)); }

/* ------------------------------------------------------------------------- */
/* cos(2 pi y) and sin(2 pi y)                                              */
/*                                                                           */
/* The families use the elementary functions cos(2*pi*y) and sin(2*pi*y) of  */
/* an argument y that carries no pi.  The point enclosure at a double y:     */
/*   f = y - nearest_integer(y)      (exact, |f| <= 1/2)                      */
/*   then exact octant identities bring the argument to g with |g| <= 1/8:   */
/*     cos(2 pi a) = sin(2 pi (1/4 - a)),   cos(2 pi a) = -cos(2 pi (1/2 - a)) */
/*     sin(2 pi a) = cos(2 pi (a - 1/4)),   sin(2 pi a) =  sin(2 pi (1/2 - a)) */
/*   v = cosl/sinl(2 pi * g) in x87 extended precision, round to nearest,    */
/*   and the enclosure is [v - |v| 2^-58, v + |v| 2^-58] rounded outward to   */
/*   double, then clamped to [-1, 1].                                         */
/* The extended-precision error (argument rounding plus the library) is a    */
/* few units of 2^-63 relative, far inside the 2^-58 margin.                 */
/* ------------------------------------------------------------------------- */

static const long double TWO_PI_L = 6.283185307179586476925286766559005768L;

static void ld_enclose(long double v, double* lo, double* hi) {
  long double m = fabsl(v) * 0x1p-58L;
  volatile long double vv = v, mm = m;
  fesetround(FE_DOWNWARD);
  volatile long double l = vv - mm;
  volatile double ld = (double)l;
  fesetround(FE_UPWARD);
  volatile long double h = vv + mm;
  volatile double hd = (double)h;
  fesetround(FE_TONEAREST);
  *lo = ld < -1.0 ? -1.0 : ld;
  *hi = hd > 1.0 ? 1.0 : hd;
}

/* which = 0: cos(2 pi y); which = 1: sin(2 pi y) */
static void pt_trig2pi(int which, double y, double* lo, double* hi) {
  if (isnan(y) || isinf(y)) { *lo = -1.0; *hi = 1.0; return; }
  double f = y - nearbyint(y);          /* exact */
  double a = fabs(f);
  double s = f < 0.0 ? -1.0 : 1.0;
  long double v;
  double g;                             /* reduced argument, |g| <= 1/8 */
  if (which == 0) {                     /* cos is even in f */
    if (a <= 0.125)       { g = a;         v = cosl(TWO_PI_L * (long double)g); }
    else if (a <= 0.375)  { g = 0.25 - a;  v = sinl(TWO_PI_L * (long double)g); }   /* 0.25 - a exact */
    else                  { g = 0.5 - a;   v = -cosl(TWO_PI_L * (long double)g); }  /* 0.5 - a exact  */
  } else {                              /* sin is odd in f */
    if (a <= 0.125)       { g = a;         v = sinl(TWO_PI_L * (long double)g); }
    else if (a <= 0.375)  { g = a - 0.25;  v = cosl(TWO_PI_L * (long double)g); }
    else                  { g = 0.5 - a;   v = sinl(TWO_PI_L * (long double)g); }
    v = (long double)s * v;
  }
  if (g == 0.0) {                       /* sin 0 = 0 and cos 0 = 1 exactly */
    *lo = *hi = (double)v;
    return;
  }
  ld_enclose(v, lo, hi);
}

/* does [p, q] contain an integer? (exact) */
static int has_int(double p, double q) { return ceil(p) <= floor(q); }

/* interval cos(2 pi Y): hull of the endpoint enclosures, +1 added when Y holds
 * an integer, -1 added when Y holds a half-integer, whole [-1,1] when the
 * width (rounded up) reaches one period. */
static iv iv_cos2pi(iv y) {
  if (bad(y) || isinf(y.lo) || isinf(y.hi)) return mk(-1.0, 1.0);
  if (up_sub(y.hi, y.lo) >= 1.0) return mk(-1.0, 1.0);
  double al, ah, bl, bh;
  pt_trig2pi(0, y.lo, &al, &ah);
  pt_trig2pi(0, y.hi, &bl, &bh);
  double lo = dmin(al, bl), hi = dmax(ah, bh);
  if (has_int(y.lo, y.hi)) hi = 1.0;                                   /* max at y in Z        */
  if (has_int(dn_sub(y.lo, 0.5), up_sub(y.hi, 0.5))) lo = -1.0;        /* min at y in Z + 1/2  */
  return mk(lo, hi);
}
/* interval sin(2 pi Y): max at y in Z + 1/4, min at y in Z - 1/4 */
static iv iv_sin2pi(iv y) {
  if (bad(y) || isinf(y.lo) || isinf(y.hi)) return mk(-1.0, 1.0);
  if (up_sub(y.hi, y.lo) >= 1.0) return mk(-1.0, 1.0);
  double al, ah, bl, bh;
  pt_trig2pi(1, y.lo, &al, &ah);
  pt_trig2pi(1, y.hi, &bl, &bh);
  double lo = dmin(al, bl), hi = dmax(ah, bh);
  if (has_int(dn_sub(y.lo, 0.25), up_sub(y.hi, 0.25))) hi = 1.0;
  if (has_int(dn_add(y.lo, 0.25), up_add(y.hi, 0.25))) lo = -1.0;
  return mk(lo, hi);
}

/* ------------------------------------------------------------------------- */
/* pi enclosures used by the derivative scale factors                        */
/* ------------------------------------------------------------------------- */

static double hexd(uint64_t u) { double d; memcpy(&d, &u, 8); return d; }
#define PI_LO_BITS 0x400921FB54442D18ull   /* largest double below pi  */
#define PI_HI_BITS 0x400921FB54442D19ull   /* smallest double above pi */

/* [c * pi * k * b] for a scale c in {1, 2} (exact power of two), k > 0 */
static iv pi_k_b(double c, double k, double b) {
  double pl = hexd(PI_LO_BITS) * c, ph = hexd(PI_HI_BITS) * c;   /* exact scaling */
  iv pk = mk(dn_mul(pl, k), up_mul(ph, k));
  return iv_mul(pk, mk(b, b));
}

/* ------------------------------------------------------------------------- */
/* families                                                                  */
/* ------------------------------------------------------------------------- */

enum { FAM_SEP_COS = 1, FAM_CHAIN = 2, FAM_SEP_ABS_SIN2 = 3 };

typedef struct {
  int32_t family, n;
  const double* coef; int64_t coef_len;
  const double* lower; const double* upper;
  double tol_f, tol_x;
} orc_problem;

static int64_t n_terms(const orc_problem* P) { return P->family == FAM_CHAIN ? (P->n >= 1 ? P->n - 1 : 0) : P->n; }

/*
 * Term t_i of f on the box x (intervals).  Expression trees:
 *   SEP_COS      f = sum a_i (x_i - c_i)^2 + b_i (1 - cos(2 pi k_i (x_i - c_i)))
 *                D = X_i - c_i,  Y = k_i D,  t = a_i D^2 + b_i (1 - cos2pi(Y))
 *   CHAIN        f = sum_{i<n-1} alpha_i (x_{i+1} - x_i^2)^2 + beta_i (x_i - 1)^2
 *                R = X_{i+1} - X_i^2,  E = X_i - 1,  t = alpha_i R^2 + beta_i E^2
 *   SEP_ABS_SIN2 f = sum s_i |x_i - c_i| + b_i sin^2(pi k_i (x_i - c_i))
 *                D = X_i - c_i,  H = (k_i/2) D,  t = s_i |D| + b_i sin2pi(H)^2
 * (cos2pi(y) = cos(2 pi y), sin2pi(y) = sin(2 pi y).)
 */
static iv term(const orc_problem* P, const iv* X, int64_t i) {
  const int64_t n = P->n;
  const double* cf = P->coef;
  switch (P->family) {
  case FAM_SEP_COS: {
    double a = cf[i], b = cf[n + i], k = cf[2 * n + i], c = cf[3 * n + i];
    iv D = iv_sub_s(X[i], c);
    iv Y = iv_scale(k, D);
    iv S = iv_sqr(D);
    iv C = iv_cos2pi(Y);
    return iv_add(iv_scale(a, S), iv_scale(b, iv_sub(mk(1.0, 1.0), C)));
  }
  case FAM_CHAIN: {
    double al = cf[i], be = cf[(n - 1) + i];
    iv R = iv_sub(X[i + 1], iv_sqr(X[i]));
    iv E = iv_sub_s(X[i], 1.0);
    return iv_add(iv_scale(al, iv_sqr(R)), iv_scale(be, iv_sqr(E)));
  }
  case FAM_SEP_ABS_SIN2: {
    double s = cf[i], b = cf[n + i], k = cf[2 * n + i], c = cf[3 * n + i];
    iv D = iv_sub_s(X[i], c);
    iv H = iv_scale(0.5 * k, D);
    iv Sn = iv_sin2pi(H);
    return iv_add(iv_scale(s, iv_abs(D)), iv_scale(b, iv_sqr(Sn)));
  }
  }
  return entire();
}

/*
 * Interval partial derivative G_j on the box x.
 *   SEP_COS      G_j = (2 a_j) D + [2 pi k_j b_j] sin2pi(k_j D)
 *   CHAIN        G_j = [j <= n-2] ( ((-4 alpha_j) X_j) R_j + (2 beta_j) E_j )
 *                      + [j >= 1] (2 alpha_{j-1}) R_{j-1}
 *                (parts that do not exist are left out, not added as zero)
 *   SEP_ABS_SIN2 G_j = s_j dabs(D) + [pi k_j b_j] sin2pi(k_j D)
 *                (d/dx b sin^2(pi k u) = pi k b sin(2 pi k u); dabs encloses
 *                 the generalized derivative of |.|)
 */
static iv grad(const orc_problem* P, const iv* X, int64_t j) {
  const int64_t n = P->n;
  const double* cf = P->coef;
  switch (P->family) {
  case FAM_SEP_COS: {
    double a = cf[j], b = cf[n + j], k = cf[2 * n + j], c = cf[3 * n + j];
    iv D = iv_sub_s(X[j], c);
    iv Y = iv_scale(k, D);
    return iv_add(iv_scale(2.0 * a, D), iv_mul(pi_k_b(2.0, k, b), iv_sin2pi(Y)));
  }
  case FAM_CHAIN: {
    int have = 0;
    iv g = mk(0.0, 0.0);
    if (j <= n - 2) {
      double al = cf[j], be = cf[(n - 1) + j];
      iv R = iv_sub(X[j + 1], iv_sqr(X[j]));
      iv E = iv_sub_s(X[j], 1.0);
      g = iv_add(iv_mul(iv_scale(-4.0 * al, X[j]), R), iv_scale(2.0 * be, E));
      have = 1;
    }
    if (j >= 1) {
      double al = cf[j - 1];
      iv R = iv_sub(X[j], iv_sqr(X[j - 1]));
      iv B = iv_scale(2.0 * al, R);
      g = have ? iv_add(g, B) : B;
      have = 1;
    }
    return g;
  }
  case FAM_SEP_ABS_SIN2: {
    double s = cf[j], b = cf[n + j], k = cf[2 * n + j], c = cf[3 * n + j];
    iv D = iv_sub_s(X[j], c);
    iv Y = iv_scale(k, D);
    return iv_add(iv_scale(s, iv_dabs(D)), iv_mul(pi_k_b(1.0, k, b), iv_sin2pi(Y)));
  }
  }
  return entire();
}

/*
 * Canonical sum: term t_i goes to slot i mod 64, each slot sums its terms left
 * to right, then the slots are folded pairwise with strides 32, 16, 8, 4, 2, 1
 * (slot s absorbs slot s + h); absent slots are skipped.  This order is part
 * of the definition of the enclosure F (the paper does not fix one).
 */
static iv canonical_sum_except(const orc_problem* P, const iv* X, const unsigned char* leave_out) {
  iv slot[64];
  int present[64];
  int64_t T = n_terms(P);
  for (int s = 0; s < 64; ++s) present[s] = 0;
  for (int64_t i = 0; i < T; ++i) {
    if (leave_out && leave_out[i]) continue;
    int s = (int)(i % 64);
    iv t = term(P, X, i);
    slot[s] = present[s] ? iv_add(slot[s], t) : t;
    present[s] = 1;
  }
  for (int h = 32; h >= 1; h /= 2)
    for (int s = 0; s < h; ++s)
      if (present[s + h]) {
        slot[s] = present[s] ? iv_add(slot[s], slot[s + h]) : slot[s + h];
        present[s] = 1;
      }
  return present[0] ? slot[0] : mk(0.0, 0.0);
}

static iv canonical_sum(const orc_problem* P, const iv* X) { return canonical_sum_except(P, X, NULL); }

/* ------------------------------------------------------------------------- */
/* generic closed-form f: an expression tape                                 */
/*                                                                           */
/* f = g(R_1, ..., R_K): each R_k is a sum or a product over i in a range of */
/* an element expression e_k(x_i, x_{i+1}, i), and g is a scalar expression  */
/* of the R_k and constants.  This covers the benchmark functions of the     */
/* paper's SI Appendix A (Eqs. S1-S21) and Appendix D (Eq. S22), which are    */
/* sums and products over the coordinates with an outer nonlinearity.        */
/*                                                                           */
/* The tape is carried in the problem's coefficient array (doubles):         */
/*   [1, K, Q, C]                                                            */
/*   K reductions: [kind (0 sum, 1 product), s_off, s_end, t_off, t_end, L]   */
/*                 then L ops of 5 doubles [code, a, b, c_lo, c_hi]          */
/*                 (range: i from s_off + (s_end ? n : 0) to t_off +           */
/*                  (t_end ? n : 0), exclusive)                               */
/*   Q scalar ops of 5 doubles; the last one's value is f                    */
/*   C coefficient columns of n doubles                                      */
/* Operands a, b index earlier ops of the same program.                      */
/*                                                                           */
/* Values are intervals (Sec. 2.1, Eqs. (3)-(6), outward rounding).          */
/* Derivatives: the element programs carry forward tangents with respect to   */
/* x_i and x_{i+1}; the scalar program is differentiated in reverse (adjoint  */
/* intervals); then G_j = sum over k of adj(R_k) dR_k/dx_j, k increasing,     */
/* where for a sum dR/dx_j = D0 e(j) + D1 e(j-1) and for a product            */
/* dR/dx_j = D0 e(j) * (prod_{i<j} e(i)) * (prod_{i>j} e(i)), the left        */
/* product taken left to right and the right one nested from the right.     */
/* Orders: sums and products run left to right over i; adjoint contributions */
/* are added in reverse op order.  These orders define the bounds.           */
/* ------------------------------------------------------------------------- */

enum { FAM_TAPE = 4 };
enum { T_CONST = 0, T_X = 1, T_XNEXT = 2, T_COEF = 3, T_ADD = 4, T_SUB = 5, T_MUL = 6, T_DIV = 7, T_NEG = 8,
       T_SQR = 9, T_SQRT = 10, T_EXP = 11, T_COS = 12, T_SIN = 13, T_COS2PI = 14, T_SIN2PI = 15, T_ABS = 16,
       T_RED = 17, T_INDEX = 18 };
#define TAPE_MAX_OPS 64
#define TAPE_MAX_RED 8

typedef struct { int code, a, b; double clo, chi; } tape_op;
typedef struct { int kind, start, stop, nops; tape_op op[TAPE_MAX_OPS]; } tape_red;
typedef struct { int K, Q, C; tape_red red[TAPE_MAX_RED]; tape_op sc[TAPE_MAX_OPS]; const double* col; } tape;

/* an op that the stage does not allow, or whose operands are not earlier ops */
static int tape_op_bad(const tape_op* o, int q, int elem, int lim) {
  const int c = o->code;
  if (c < 0 || c > T_INDEX) return 1;
  if (elem && c == T_RED) return 1;
  if (!elem && (c == T_X || c == T_XNEXT || c == T_COEF || c == T_INDEX)) return 1;
  if ((c == T_COEF || c == T_RED) && (o->a < 0 || o->a >= lim)) return 1;
  if (c >= T_ADD && c <= T_ABS && (o->a < 0 || o->a >= q)) return 1;
  if (c >= T_ADD && c <= T_DIV && (o->b < 0 || o->b >= q)) return 1;
  if (c == T_CONST && !(o->clo <= o->chi)) return 1;
  return 0;
}

static int tape_parse(const orc_problem* P, tape* T) {
  const double* c = P->coef;
  const int64_t n = P->n, len = P->coef_len;
  if (len < 4 || c[0] != 1.0) return -1;
  T->K = (int)c[1]; T->Q = (int)c[2]; T->C = (int)c[3];
  if (T->K < 0 || T->K > TAPE_MAX_RED || T->Q < 1 || T->Q > TAPE_MAX_OPS || T->C < 0) return -1;
  int64_t at = 4;
  for (int k = 0; k < T->K; ++k) {
    if (at + 6 > len) return -1;
    tape_red* R = &T->red[k];
    R->kind = (int)c[at];
    int64_t s = (int64_t)c[at + 1] + (c[at + 2] != 0.0 ? n : 0), t = (int64_t)c[at + 3] + (c[at + 4] != 0.0 ? n : 0);
    R->nops = (int)c[at + 5];
    at += 6;
    if (R->nops < 1 || R->nops > TAPE_MAX_OPS || at + 5 * R->nops > len) return -1;
    if (s < 0) s = 0;
    if (t > n) t = n;
    R->start = (int)s; R->stop = (int)(t > s ? t : s);
    for (int q = 0; q < R->nops; ++q, at += 5) {
      R->op[q].code = (int)c[at]; R->op[q].a = (int)c[at + 1]; R->op[q].b = (int)c[at + 2];
      R->op[q].clo = c[at + 3]; R->op[q].chi = c[at + 4];
      if (tape_op_bad(&R->op[q], q, 1, T->C)) return -1;
      if (R->op[q].code == T_XNEXT && (R->kind != 0 || R->stop > n - 1)) return -1;
    }
  }
  if (at + 5 * T->Q > len) return -1;
  for (int q = 0; q < T->Q; ++q, at += 5) {
    T->sc[q].code = (int)c[at]; T->sc[q].a = (int)c[at + 1]; T->sc[q].b = (int)c[at + 2];
    T->sc[q].clo = c[at + 3]; T->sc[q].chi = c[at + 4];
    if (tape_op_bad(&T->sc[q], q, 0, T->K)) return -1;
  }
  if (at + (int64_t)T->C * n != len) return -1;
  T->col = c + at;
  return 0;
}

/* exp enclosure of a double: expl in extended precision +- |v| 2^-58 */
static void pt_exp(double x, double* lo, double* hi) {
  if (x == 0.0) { *lo = *hi = 1.0; return; }
  if (isinf(x)) { *lo = *hi = x > 0 ? INFINITY : 0.0; return; }
  long double v = expl((long double)x);
  long double m = v * 0x1p-58L;
  volatile long double vv = v, mm = m;
  fesetround(FE_DOWNWARD);
  volatile long double l = vv - mm;
  volatile double ld = (double)l;
  fesetround(FE_UPWARD);
  volatile long double h = vv + mm;
  volatile double hd = (double)h;
  fesetround(FE_TONEAREST);
  *lo = ld < 0.0 ? 0.0 : ld;
  *hi = hd;
}
static iv iv_exp(iv a) {
  if (bad(a)) return mk(0.0, INFINITY);
  double l, h, t;
  pt_exp(a.lo, &l, &t);
  pt_exp(a.hi, &t, &h);
  return mk(l, h);
}
/* [1 / (2 pi)]: the two adjacent doubles around it (1 / (2 pi) =
 * 0.15915494309189533576888..., between 0x3FC45F306DC9C882 = 0.159154943091895317...
 * and 0x3FC45F306DC9C883 = 0.159154943091895345...) */
static iv inv_two_pi(void) { return mk(hexd(0x3FC45F306DC9C882ull), hexd(0x3FC45F306DC9C883ull)); }
/* [2 pi] from the doubles around pi (exact doubling) */
static iv two_pi(void) { return mk(2.0 * hexd(PI_LO_BITS), 2.0 * hexd(PI_HI_BITS)); }
static iv iv_cos(iv a) { return iv_cos2pi(iv_mul(a, inv_two_pi())); }
static iv iv_sin(iv a) { return iv_sin2pi(iv_mul(a, inv_two_pi())); }
static iv iv_neg(iv a) { return mk(-a.hi, -a.lo); }

/* value with optional tangents (d0: d/dx_i, d1: d/dx_{i+1}); has0/has1 = 0: exactly zero */
typedef struct { iv v, d0, d1; int has0, has1; } tv;

static iv acc_add(iv s, int* has, iv t) { if (*has) return iv_add(s, t); *has = 1; return t; }

/* the value of one op from its operands' values (shared by both stages) */
static iv op_value(const tape_op* o, const iv* V, iv x0, iv x1, int64_t i, const tape* T, int64_t n,
                   const iv* red) {
  switch (o->code) {
  case T_CONST: return mk(o->clo, o->chi);
  case T_X: return x0;
  case T_XNEXT: return x1;
  case T_COEF: { double v = T->col[(int64_t)o->a * n + i]; return mk(v, v); }
  case T_INDEX: return mk((double)(i + 1), (double)(i + 1));
  case T_RED: return red[o->a];
  case T_ADD: return iv_add(V[o->a], V[o->b]);
  case T_SUB: return iv_sub(V[o->a], V[o->b]);
  case T_MUL: return iv_mul(V[o->a], V[o->b]);
  case T_DIV: return iv_div(V[o->a], V[o->b]);
  case T_NEG: return iv_neg(V[o->a]);
  case T_SQR: return iv_sqr(V[o->a]);
  case T_SQRT: return iv_sqrt(V[o->a]);
  case T_EXP: return iv_exp(V[o->a]);
  case T_COS: return iv_cos(V[o->a]);
  case T_SIN: return iv_sin(V[o->a]);
  case T_COS2PI: return iv_cos2pi(V[o->a]);
  case T_SIN2PI: return iv_sin2pi(V[o->a]);
  case T_ABS: return iv_abs(V[o->a]);
  }
  return entire();
}

/* the derivative factor of a unary op u = h(a): dh/da over the operand's value a
 * and the op's own value v */
static iv unary_factor(int code, iv a, iv v) {
  switch (code) {
  case T_NEG: return mk(-1.0, -1.0);
  case T_SQR: return iv_scale(2.0, a);
  case T_SQRT: return iv_recip(iv_scale(2.0, v));
  case T_EXP: return v;
  case T_COS: return iv_neg(iv_sin(a));
  case T_SIN: return iv_cos(a);
  case T_COS2PI: return iv_neg(iv_mul(two_pi(), iv_sin2pi(a)));
  case T_SIN2PI: return iv_mul(two_pi(), iv_cos2pi(a));
  case T_ABS: return iv_dabs(a);
  }
  return entire();
}

/* forward pass of one element program at index i; returns the last op's value
 * and tangents in *out */
static void elem_eval(const tape* T, const tape_red* R, int64_t n, int64_t i, iv x0, iv x1, int want_d, tv* out) {
  iv V[TAPE_MAX_OPS];
  tv W[TAPE_MAX_OPS];
  for (int q = 0; q < R->nops; ++q) {
    const tape_op* o = &R->op[q];
    V[q] = op_value(o, V, x0, x1, i, T, n, NULL);
    tv w;
    w.v = V[q]; w.has0 = w.has1 = 0; w.d0 = w.d1 = mk(0.0, 0.0);
    if (want_d) {
      const tv* A = o->a >= 0 && o->a < q ? &W[o->a] : NULL;
      const tv* B = o->b >= 0 && o->b < q ? &W[o->b] : NULL;
      switch (o->code) {
      case T_X: w.d0 = mk(1.0, 1.0); w.has0 = 1; break;
      case T_XNEXT: w.d1 = mk(1.0, 1.0); w.has1 = 1; break;
      case T_ADD: case T_SUB: {
        if (A->has0) w.d0 = acc_add(w.d0, &w.has0, A->d0);
        if (A->has1) w.d1 = acc_add(w.d1, &w.has1, A->d1);
        if (B->has0) w.d0 = acc_add(w.d0, &w.has0, o->code == T_SUB ? iv_neg(B->d0) : B->d0);
        if (B->has1) w.d1 = acc_add(w.d1, &w.has1, o->code == T_SUB ? iv_neg(B->d1) : B->d1);
        break;
      }
      case T_MUL: {   /* d(ab) = da b + a db */
        if (A->has0) w.d0 = acc_add(w.d0, &w.has0, iv_mul(A->d0, B->v));
        if (A->has1) w.d1 = acc_add(w.d1, &w.has1, iv_mul(A->d1, B->v));
        if (B->has0) w.d0 = acc_add(w.d0, &w.has0, iv_mul(A->v, B->d0));
        if (B->has1) w.d1 = acc_add(w.d1, &w.has1, iv_mul(A->v, B->d1));
        break;
      }
      case T_DIV: {   /* d(a/b) = (da - (a/b) db) (1/b) */
        const iv rb = iv_recip(B->v);
        for (int s = 0; s < 2; ++s) {
          const int ha = s ? A->has1 : A->has0, hb = s ? B->has1 : B->has0;
          if (!ha && !hb) continue;
          iv num;
          if (ha && hb) num = iv_sub(s ? A->d1 : A->d0, iv_mul(V[q], s ? B->d1 : B->d0));
          else if (ha) num = s ? A->d1 : A->d0;
          else num = iv_neg(iv_mul(V[q], s ? B->d1 : B->d0));
          if (s) { w.d1 = iv_mul(num, rb); w.has1 = 1; } else { w.d0 = iv_mul(num, rb); w.has0 = 1; }
        }
        break;
      }
      case T_NEG: case T_SQR: case T_SQRT: case T_EXP: case T_COS: case T_SIN: case T_COS2PI: case T_SIN2PI:
      case T_ABS: {
        if (!A->has0 && !A->has1) break;
        const iv f = unary_factor(o->code, A->v, V[q]);
        if (A->has0) { w.d0 = iv_mul(f, A->d0); w.has0 = 1; }
        if (A->has1) { w.d1 = iv_mul(f, A->d1); w.has1 = 1; }
        break;
      }
      default: break;   /* constants, coefficients, the index: no tangent */
      }
    }
    W[q] = w;
  }
  *out = W[R->nops - 1];
}

/* F over the box X (and G when G != NULL) of a tape problem */
static iv tape_eval(const orc_problem* P, const iv* X, iv* G) {
  tape T;
  if (tape_parse(P, &T) != 0) return entire();
  const int64_t n = P->n;
  iv red[TAPE_MAX_RED];
  tv* E[TAPE_MAX_RED];
  for (int k = 0; k < T.K; ++k) {
    const tape_red* R = &T.red[k];
    E[k] = G ? (tv*)malloc((size_t)(n > 0 ? n : 1) * sizeof(tv)) : NULL;
    int have = 0;
    iv acc = R->kind ? mk(1.0, 1.0) : mk(0.0, 0.0);
    for (int64_t i = R->start; i < R->stop; ++i) {
      tv e;
      elem_eval(&T, R, n, i, X[i], i + 1 < n ? X[i + 1] : X[i], G != NULL, &e);
      if (G) E[k][i] = e;
      acc = have ? (R->kind ? iv_mul(acc, e.v) : iv_add(acc, e.v)) : e.v;
      have = 1;
    }
    red[k] = acc;
  }
  /* scalar program: values, then adjoints in reverse */
  iv V[TAPE_MAX_OPS];
  for (int q = 0; q < T.Q; ++q) V[q] = op_value(&T.sc[q], V, mk(0.0, 0.0), mk(0.0, 0.0), 0, &T, n, red);
  iv F = V[T.Q - 1];
  if (!G) return F;
  iv A[TAPE_MAX_OPS], AR[TAPE_MAX_RED];
  int hA[TAPE_MAX_OPS], hR[TAPE_MAX_RED];
  for (int q = 0; q < T.Q; ++q) { hA[q] = 0; A[q] = mk(0.0, 0.0); }
  for (int k = 0; k < T.K; ++k) { hR[k] = 0; AR[k] = mk(0.0, 0.0); }
  A[T.Q - 1] = mk(1.0, 1.0); hA[T.Q - 1] = 1;
  for (int q = T.Q - 1; q >= 0; --q) {
    if (!hA[q]) continue;
    const tape_op* o = &T.sc[q];
    const iv a = A[q];
    switch (o->code) {
    case T_RED: AR[o->a] = acc_add(AR[o->a], &hR[o->a], a); break;
    case T_ADD: A[o->a] = acc_add(A[o->a], &hA[o->a], a); A[o->b] = acc_add(A[o->b], &hA[o->b], a); break;
    case T_SUB: A[o->a] = acc_add(A[o->a], &hA[o->a], a); A[o->b] = acc_add(A[o->b], &hA[o->b], iv_neg(a)); break;
    case T_MUL:
      A[o->a] = acc_add(A[o->a], &hA[o->a], iv_mul(a, V[o->b]));
      A[o->b] = acc_add(A[o->b], &hA[o->b], iv_mul(a, V[o->a]));
      break;
    case T_DIV: {
      const iv rb = iv_recip(V[o->b]);
      A[o->a] = acc_add(A[o->a], &hA[o->a], iv_mul(a, rb));
      A[o->b] = acc_add(A[o->b], &hA[o->b], iv_neg(iv_mul(a, iv_mul(V[q], rb))));
      break;
    }
    case T_NEG: case T_SQR: case T_SQRT: case T_EXP: case T_COS: case T_SIN: case T_COS2PI: case T_SIN2PI:
    case T_ABS:
      A[o->a] = acc_add(A[o->a], &hA[o->a], iv_mul(a, unary_factor(o->code, V[o->a], V[q])));
      break;
    default: break;
    }
  }
  /* products: left products pre[j] = e(start) ... e(j-1) (left to right) and
   * right products suf[j] = e(j+1) (e(j+2) (... e(stop-1))) */
  iv* PRE[TAPE_MAX_RED];
  iv* SUF[TAPE_MAX_RED];
  for (int k = 0; k < T.K; ++k) {
    PRE[k] = SUF[k] = NULL;
    const tape_red* R = &T.red[k];
    if (R->kind != 1 || R->stop <= R->start) continue;
    PRE[k] = (iv*)malloc((size_t)n * sizeof(iv));
    SUF[k] = (iv*)malloc((size_t)n * sizeof(iv));
    PRE[k][R->start] = mk(1.0, 1.0);   /* empty */
    for (int64_t i = R->start + 1; i < R->stop; ++i)
      PRE[k][i] = i - 1 == R->start ? E[k][i - 1].v : iv_mul(PRE[k][i - 1], E[k][i - 1].v);
    SUF[k][R->stop - 1] = mk(1.0, 1.0);   /* empty */
    for (int64_t i = R->stop - 2; i >= R->start; --i)
      SUF[k][i] = i + 1 == R->stop - 1 ? E[k][i + 1].v : iv_mul(E[k][i + 1].v, SUF[k][i + 1]);
  }
  /* G_j over the reductions, k increasing */
  for (int64_t j = 0; j < n; ++j) {
    int hg = 0;
    iv g = mk(0.0, 0.0);
    for (int k = 0; k < T.K; ++k) {
      if (!hR[k]) continue;
      const tape_red* R = &T.red[k];
      int hd = 0;
      iv d = mk(0.0, 0.0);
      if (R->kind == 0) {
        if (j >= R->start && j < R->stop && E[k][j].has0) d = acc_add(d, &hd, E[k][j].d0);
        if (j - 1 >= R->start && j - 1 < R->stop && E[k][j - 1].has1) d = acc_add(d, &hd, E[k][j - 1].d1);
      } else if (j >= R->start && j < R->stop && E[k][j].has0) {
        const int hp = j > R->start, hs = j < R->stop - 1;
        const iv loo = hp && hs ? iv_mul(PRE[k][j], SUF[k][j]) : (hp ? PRE[k][j] : (hs ? SUF[k][j] : mk(1.0, 1.0)));
        d = iv_mul(E[k][j].d0, loo);
        hd = 1;
      }
      if (hd) g = acc_add(g, &hg, iv_mul(AR[k], d));
    }
    G[j] = g;
  }
  for (int k = 0; k < T.K; ++k) { free(E[k]); free(PRE[k]); free(SUF[k]); }
  return F;
}

/* bisection point of [lo, hi]: 0.5 lo + 0.5 hi rounded up, kept inside */
static double midpoint(double lo, double hi) {
  double m = up_add(up_mul(0.5, lo), up_mul(0.5, hi));
  if (m < lo) m = lo;
  if (m > hi) m = hi;
  return m;
}

typedef struct { iv F; double ub; int mono; } box_eval;

/* upper bound of f at a point (X holds point intervals) */
static double point_hi(const orc_problem* P, const iv* X) {
  return P->family == FAM_TAPE ? tape_eval(P, X, NULL).hi : canonical_sum(P, X).hi;
}

/*
 * Bound one box: F over the box, the first-order test (Sec. 3.1: discard when
 * some DLB_j > 0 and x_j^lo != l_j, or some DUB_j < 0 and x_j^hi != u_j), and
 * the upper bound of f at the box midpoint (the sampling step of Sec. 3.1 with
 * a single sample point).  G receives the gradient enclosure when non-NULL.
 */
static box_eval eval_box(const orc_problem* P, const double* lo, const double* hi, iv* X, iv* G) {
  const int64_t n = P->n;
  box_eval r;
  for (int64_t i = 0; i < n; ++i) X[i] = mk(lo[i], hi[i]);
  r.mono = 0;
  if (P->family == FAM_TAPE) {
    iv* GG = G ? G : (iv*)malloc((size_t)(n > 0 ? n : 1) * sizeof(iv));
    r.F = tape_eval(P, X, GG);
    for (int64_t j = 0; j < n; ++j) {
      const iv g = GG[j];
      if ((g.lo > 0.0 && lo[j] != P->lower[j]) || (g.hi < 0.0 && hi[j] != P->upper[j])) r.mono = 1;
    }
    if (!G) free(GG);
  } else {
    r.F = canonical_sum(P, X);
    for (int64_t j = 0; j < n; ++j) {
      iv g = grad(P, X, j);
      if (G) G[j] = g;
      if ((g.lo > 0.0 && lo[j] != P->lower[j]) || (g.hi < 0.0 && hi[j] != P->upper[j])) r.mono = 1;
    }
  }
  for (int64_t i = 0; i < n; ++i) { double m = midpoint(lo[i], hi[i]); X[i] = mk(m, m); }
  r.ub = point_hi(P, X);
  return r;
}

/* ------------------------------------------------------------------------- */
/* the iteration                                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t split_dims, select_k; int64_t max_sweeps, max_live_boxes;
  int32_t incremental;   /* 1: children bounded from their parent's shared terms (see child_bounds) */
  int32_t reserved;
  int32_t pieces;        /* subintervals per split coordinate: 2 (bisection, default) or 4 (Sec. 4) */
  int32_t samples;       /* 0: one sample, the child midpoint; S > 0: S points on the child's diagonal */
} orc_options;

/*
 * Incremental bounds of the children of one selected box (an option; the
 * paper bounds every subregion from scratch and fixes no summation order).
 * A child differs from its parent only on the split coordinates, so a term t_i
 * that involves none of them (SEP: i not split; CHAIN: neither i nor i+1
 * split) is the parent's.  The canonical sum of those terms (the order of
 * canonical_sum, affected terms left out) is formed once per parent; a child's
 * F is that sum plus its affected terms, added one at a time in increasing i.
 * The midpoint upper bound is formed the same way, from the terms at the
 * midpoints (the midpoint of an unsplit coordinate is the parent's).  The
 * first-order test and the widest side are unchanged: they do not depend on an
 * order of summation.
 */
typedef struct {
  unsigned char* affected;  /* [n_terms] */
  iv base_F;
  double base_ub;
} parent_base;

static void parent_base_form(const orc_problem* P, const double* lo, const double* hi, const int* split_dim,
                             int n_split, iv* X, parent_base* B) {
  const int64_t n = P->n, T = n_terms(P);
  for (int64_t i = 0; i < T; ++i) B->affected[i] = 0;
  for (int q = 0; q < n_split; ++q) {
    const int64_t d = split_dim[q];
    if (d < T) B->affected[d] = 1;                                  /* t_d involves x_d */
    if (P->family == FAM_CHAIN && d >= 1) B->affected[d - 1] = 1;   /* t_{d-1} involves x_d */
  }
  for (int64_t i = 0; i < n; ++i) X[i] = mk(lo[i], hi[i]);
  B->base_F = canonical_sum_except(P, X, B->affected);
  for (int64_t i = 0; i < n; ++i) { double m = midpoint(lo[i], hi[i]); X[i] = mk(m, m); }
  B->base_ub = canonical_sum_except(P, X, B->affected).hi;
}

/* F and the midpoint upper bound of a child from its parent's base */
static void child_bounds(const orc_problem* P, const parent_base* B, const double* lo, const double* hi, iv* X,
                         iv* F, double* ub) {
  const int64_t n = P->n, T = n_terms(P);
  for (int64_t i = 0; i < n; ++i) X[i] = mk(lo[i], hi[i]);
  iv f = B->base_F;
  for (int64_t i = 0; i < T; ++i)
    if (B->affected[i]) f = iv_add(f, term(P, X, i));
  for (int64_t i = 0; i < n; ++i) { double m = midpoint(lo[i], hi[i]); X[i] = mk(m, m); }
  double u = B->base_ub;
  for (int64_t i = 0; i < T; ++i)
    if (B->affected[i]) u = up_add(u, term(P, X, i).hi);
  *F = f;
  *ub = u;
}
/* ------------------------------------------------------------------------- */
/* the schedule of the paper's experiments (Sec. 4): each of the m cycled      */
/* coordinates of the selected box is cut into four equal subintervals        */
/* (Sec. 3.2, Eqs. (8)-(11)), 4^m subregions, and each subregion is sampled   */
/* at points on its diagonal that cut it into S + 1 equal pieces              */
/* ------------------------------------------------------------------------- */

#define MAX_SAMPLES 16

/* The cut points of one coordinate [lo, hi] into `pieces` subintervals:
 * cut[0] = lo, cut[pieces] = hi, and in between (bisection) the midpoint, or
 * (four pieces, Eqs. (10)-(11)) lo + w I with w = (hi - lo) / 4, I = 1, 2, 3,
 * each operation rounded up (exact for the dyadic domains of the experiments),
 * kept inside [previous cut, hi].  Neighbouring subintervals share their cut
 * point and the last one ends at hi itself, so the pieces cover [lo, hi] with
 * no gap whatever the rounding.  Returns 1 when every piece has positive width
 * (the coordinate is split), 0 otherwise (it is then left whole). */
static int make_cuts(double lo, double hi, int pieces, double* cut) {
  cut[0] = lo;
  cut[pieces] = hi;
  if (pieces == 2) {
    cut[1] = midpoint(lo, hi);
  } else {
    double w = up_mul(up_sub(hi, lo), 0.25);
    for (int I = 1; I < pieces; ++I) {
      double c = up_add(lo, up_mul(w, (double)I));
      if (c < cut[I - 1]) c = cut[I - 1];
      if (c > hi) c = hi;
      cut[I] = c;
    }
  }
  for (int I = 0; I < pieces; ++I)
    if (!(cut[I] < cut[I + 1])) return 0;
  return 1;
}

/* digit j of child index r in base `pieces` (little-endian: digit 0 is the
 * first coordinate of the window, Eqs. (8)-(9) read for m coordinates) */
static int digit(int64_t r, int j, int pieces) {
  for (int q = 0; q < j; ++q) r /= pieces;
  return (int)(r % pieces);
}

/* coordinate of diagonal sample s (1..S) of [a, b]: a + (b - a) c_s with c_s
 * the double nearest to s / (S + 1), each operation rounded up, kept in [a, b] */
static double diag_coord(double a, double b, double c) {
  double x = up_add(a, up_mul(up_sub(b, a), c));
  if (x < a) x = a;
  if (x > b) x = b;
  return x;
}

/* F, the first-order flag and the smallest sample upper bound of one box,
 * every term formed over all n coordinates (the reference evaluation) */
static box_eval eval_box_samples(const orc_problem* P, const double* lo, const double* hi, iv* X, int S,
                                 const double* cs) {
  box_eval r = eval_box(P, lo, hi, X, NULL);
  if (S <= 0) return r;
  const int64_t n = P->n;
  double ub = INFINITY;
  for (int s = 0; s < S; ++s) {
    for (int64_t i = 0; i < n; ++i) { double x = diag_coord(lo[i], hi[i], cs[s]); X[i] = mk(x, x); }
    double u = point_hi(P, X);
    if (u < ub) ub = u;
  }
  r.ub = ub;
  return r;
}

/* Incremental bounds of all children of one selected box, memoised per piece.
 * The terms and derivative coordinates that involve a split coordinate are the
 * only ones that differ between children; each of them is evaluated once for
 * every combination of pieces of the coordinates it involves (the same interval
 * operations a child would make), and a child adds, in increasing term index,
 * the entries of its own pieces to the canonical sums of the other terms over
 * the parent (F, and each sample point).  The first-order test is taken over
 * the affected derivative coordinates only: every other coordinate has the
 * parent's interval and derivative, and the parent passed the test there (the
 * root, whose sides lie on the domain's bounds, passes it everywhere). */
typedef struct {
  int n_aff;
  int64_t aff[48];
  int aj[48][2];                   /* window index of the term's coordinates (-1: not split) */
  iv tF[48][16];                   /* term over the pieces (digit of first + pieces * digit of second) */
  double tS[48][16][MAX_SAMPLES];  /* term's upper bound at each sample point */
  int n_g;
  int64_t gc[48];
  int gj[48][3];                   /* window index of g - 1, g, g + 1 (-1: not split or absent) */
  unsigned char gm[48][64];        /* first-order test fails, per combination of pieces */
  iv base_F;
  double base_S[MAX_SAMPLES];
  double wbase;                    /* widest side among the coordinates not split */
} piece_tab;

static int win_of(const int* dim, const int* split, int m, int64_t i) {
  for (int j = 0; j < m; ++j)
    if (split[j] && dim[j] == i) return j;
  return -1;
}

static iv piece_iv(const double* plo, const double* phi, const double (*cut)[5], int j, int64_t i, int d) {
  return j < 0 ? mk(plo[i], phi[i]) : mk(cut[j][d], cut[j][d + 1]);
}

static void piece_tab_form(const orc_problem* P, const double* plo, const double* phi, const int* dim,
                           const int* split, const double (*cut)[5], int m, int pieces, int S, const double* cs,
                           iv* X, unsigned char* affected, piece_tab* B) {
  const int64_t n = P->n, T = n_terms(P);
  const int chain = P->family == FAM_CHAIN;
  for (int64_t i = 0; i < T; ++i) affected[i] = 0;
  for (int j = 0; j < m; ++j) {
    if (!split[j]) continue;
    const int64_t d = dim[j];
    if (d < T) affected[d] = 1;
    if (chain && d >= 1) affected[d - 1] = 1;
  }
  B->n_aff = 0;
  for (int64_t i = 0; i < T; ++i)
    if (affected[i]) {
      int a = B->n_aff++;
      B->aff[a] = i;
      B->aj[a][0] = win_of(dim, split, m, i);
      B->aj[a][1] = chain ? win_of(dim, split, m, i + 1) : -1;
      const int nb = (chain && B->aj[a][1] >= 0) ? pieces : 1, na = B->aj[a][0] >= 0 ? pieces : 1;
      for (int db = 0; db < nb; ++db)
        for (int da = 0; da < na; ++da) {
          const int cb = da + pieces * db;
          X[i] = piece_iv(plo, phi, cut, B->aj[a][0], i, da);
          if (chain) X[i + 1] = piece_iv(plo, phi, cut, B->aj[a][1], i + 1, db);
          B->tF[a][cb] = term(P, X, i);
          iv xa = X[i], xb = chain ? X[i + 1] : X[i];
          for (int s = 0; s < S; ++s) {
            double pa = diag_coord(xa.lo, xa.hi, cs[s]);
            X[i] = mk(pa, pa);
            if (chain) { double pb = diag_coord(xb.lo, xb.hi, cs[s]); X[i + 1] = mk(pb, pb); }
            B->tS[a][cb][s] = term(P, X, i).hi;
          }
        }
    }
  /* derivative coordinates whose interval derivative involves a split coordinate */
  B->n_g = 0;
  for (int64_t g = 0; g < n; ++g) {
    int jm = g >= 1 ? win_of(dim, split, m, g - 1) : -1, j0 = win_of(dim, split, m, g),
        jp = g + 1 < n ? win_of(dim, split, m, g + 1) : -1;
    if (!chain) jm = jp = -1;
    if (jm < 0 && j0 < 0 && jp < 0) continue;
    int k = B->n_g++;
    B->gc[k] = g;
    B->gj[k][0] = jm; B->gj[k][1] = j0; B->gj[k][2] = jp;
    for (int c = 0; c < pieces * pieces * pieces; ++c) {
      const int d0 = c % pieces, d1 = (c / pieces) % pieces, d2 = c / (pieces * pieces);
      if ((jm < 0 && d0) || (j0 < 0 && d1) || (jp < 0 && d2)) { B->gm[k][c] = 0; continue; }
      if (g >= 1) X[g - 1] = piece_iv(plo, phi, cut, jm, g - 1, d0);
      X[g] = piece_iv(plo, phi, cut, j0, g, d1);
      if (g + 1 < n) X[g + 1] = piece_iv(plo, phi, cut, jp, g + 1, d2);
      iv G = grad(P, X, g);
      B->gm[k][c] = (G.lo > 0.0 && X[g].lo != P->lower[g]) || (G.hi < 0.0 && X[g].hi != P->upper[g]);
    }
  }
  /* canonical sums of the unaffected terms over the parent and at its sample points */
  for (int64_t i = 0; i < n; ++i) X[i] = mk(plo[i], phi[i]);
  B->base_F = canonical_sum_except(P, X, affected);
  for (int s = 0; s < S; ++s) {
    for (int64_t i = 0; i < n; ++i) { double x = diag_coord(plo[i], phi[i], cs[s]); X[i] = mk(x, x); }
    B->base_S[s] = canonical_sum_except(P, X, affected).hi;
  }
  B->wbase = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (win_of(dim, split, m, i) < 0) B->wbase = dmax(B->wbase, up_sub(phi[i], plo[i]));
}

/* one child from the tables: F (the base plus the affected terms in increasing
 * index; lower endpoints summed rounding down, upper ones rounding up), the
 * first-order flag, the smallest sample upper bound and the widest side */
static box_eval piece_child(const piece_tab* B, const int* dig, const double (*cut)[5], const int* split, int m,
                            int pieces, int S, double* wmax) {
  box_eval r;
  int cb[48];
  for (int a = 0; a < B->n_aff; ++a) {
    const int ja = B->aj[a][0], jb = B->aj[a][1];
    cb[a] = (ja >= 0 ? dig[ja] : 0) + pieces * (jb >= 0 ? dig[jb] : 0);
  }
  volatile double lo = B->base_F.lo, hi = B->base_F.hi;
  fesetround(FE_DOWNWARD);
  for (int a = 0; a < B->n_aff; ++a) lo = lo + B->tF[a][cb[a]].lo;
  fesetround(FE_UPWARD);
  for (int a = 0; a < B->n_aff; ++a) hi = hi + B->tF[a][cb[a]].hi;
  double ub = INFINITY;
  for (int s = 0; s < S; ++s) {
    volatile double u = B->base_S[s];
    for (int a = 0; a < B->n_aff; ++a) u = u + B->tS[a][cb[a]][s];
    if (u < ub) ub = u;
  }
  fesetround(FE_TONEAREST);
  r.F = fix(mk(lo, hi));
  r.ub = isnan(ub) ? INFINITY : ub;
  r.mono = 0;
  for (int k = 0; k < B->n_g && !r.mono; ++k) {
    const int c = (B->gj[k][0] >= 0 ? dig[B->gj[k][0]] : 0) + pieces * (B->gj[k][1] >= 0 ? dig[B->gj[k][1]] : 0) +
                  pieces * pieces * (B->gj[k][2] >= 0 ? dig[B->gj[k][2]] : 0);
    r.mono = B->gm[k][c];
  }
  double w = B->wbase;
  for (int j = 0; j < m; ++j)
    if (split[j]) w = dmax(w, up_sub(cut[j][dig[j] + 1], cut[j][dig[j]]));
  *wmax = w;
  return r;
}

typedef struct { double f_lo, f_hi; int64_t n_boxes, sweeps, boxes_evaluated; int32_t status; } orc_info;

enum { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_INVALID = -1, ST_NOMEM = -2, ST_INTERNAL = -5 };

typedef struct { double* lo; double* hi; double flo, wmax; int64_t seq; int32_t cyc; } box;

typedef struct {
  int32_t n;
  box* live; int64_t n_live, cap_live;
  double gub;
  orc_info info;
  double* tr_gub; int64_t* tr_nsurv; int64_t* tr_nlive; int64_t* tr_sel; int64_t n_trace, cap_trace;
} solve_state;

static int push_box(solve_state* S, box b) {
  if (S->n_live == S->cap_live) {
    int64_t nc = S->cap_live ? 2 * S->cap_live : 1024;
    box* nb = (box*)realloc(S->live, (size_t)nc * sizeof(box));
    if (!nb) return 0;
    S->live = nb; S->cap_live = nc;
  }
  S->live[S->n_live++] = b;
  return 1;
}
static void free_box(box* b) { free(b->lo); free(b->hi); }

static double box_wmax(int n, const double* lo, const double* hi) {
  double w = 0.0;
  for (int i = 0; i < n; ++i) w = dmax(w, up_sub(hi[i], lo[i]));
  return w;
}

/* (flo, seq) lexicographic order used by the selection */
static int key_less(const box* a, const box* b) {
  if (a->flo != b->flo) return a->flo < b->flo;
  return a->seq < b->seq;
}

/* remove every live box whose lower bound exceeds GUB (Sec. 3.1, "Remove the
 * suboptimal regions"); equality is kept */
static void cutoff(solve_state* S) {
  int64_t w = 0;
  for (int64_t i = 0; i < S->n_live; ++i) {
    if (S->live[i].flo > S->gub) free_box(&S->live[i]);
    else S->live[w++] = S->live[i];
  }
  S->n_live = w;
}

static int cmp_seq(const void* a, const void* b) {
  int64_t x = ((const box*)a)->seq, y = ((const box*)b)->seq;
  return (x > y) - (x < y);
}

void* orc_solve(const orc_problem* P, const orc_options* O, int64_t trace_cap) {
  solve_state* S = (solve_state*)calloc(1, sizeof(solve_state));
  if (!S) return NULL;
  const int n = P->n;
  S->n = n;
  S->cap_trace = trace_cap > 0 ? trace_cap : 0;
  if (S->cap_trace) {
    S->tr_gub = (double*)malloc((size_t)S->cap_trace * sizeof(double));
    S->tr_nsurv = (int64_t*)malloc((size_t)S->cap_trace * sizeof(int64_t));
    S->tr_nlive = (int64_t*)malloc((size_t)S->cap_trace * sizeof(int64_t));
    S->tr_sel = (int64_t*)malloc((size_t)S->cap_trace * sizeof(int64_t));
  }
  const int m = n < O->split_dims ? n : O->split_dims;
  const int K = O->select_k > 0 ? O->select_k : 1;
  const int PC = O->pieces == 4 ? 4 : 2;                            /* subintervals per split coordinate */
  const int NS = O->samples > 0 ? (O->samples < MAX_SAMPLES ? O->samples : MAX_SAMPLES) : 0;
  const int general = PC != 2 || NS > 0;                           /* the schedule of Sec. 4 (or part of it) */
  orc_options O_local = *O;
  if (P->family == FAM_TAPE) O_local.incremental = 0;               /* tapes: every child bounded in full */
  O = &O_local;
  double cs[MAX_SAMPLES];
  for (int q = 0; q < NS; ++q) cs[q] = (double)(q + 1) / (double)(NS + 1);   /* nearest double to q+1 / (S+1) */
  piece_tab* tab = general ? (piece_tab*)malloc(sizeof(piece_tab)) : NULL;
  iv* X = (iv*)malloc((size_t)n * sizeof(iv));
  box* par = (box*)malloc((size_t)K * sizeof(box));
  double* clo = (double*)malloc((size_t)n * sizeof(double));
  double* chi = (double*)malloc((size_t)n * sizeof(double));
  parent_base pb;
  pb.affected = (unsigned char*)malloc((size_t)(n > 0 ? n : 1));

  /* Initialization (Sec. 3.1): L = { whole domain } */
  box root;
  root.lo = (double*)malloc((size_t)n * sizeof(double));
  root.hi = (double*)malloc((size_t)n * sizeof(double));
  memcpy(root.lo, P->lower, (size_t)n * sizeof(double));
  memcpy(root.hi, P->upper, (size_t)n * sizeof(double));
  box_eval e0 = eval_box(P, root.lo, root.hi, X, NULL);
  root.flo = e0.F.lo; root.seq = 0; root.cyc = 0; root.wmax = box_wmax(n, root.lo, root.hi);
  /* with diagonal samples (the schedule of Sec. 4) nothing is sampled before the
   * first iteration, which samples the subregions of the whole domain: GUB
   * starts at +inf; with the midpoint rule the root's midpoint bound starts it */
  S->gub = NS > 0 ? INFINITY : e0.ub;
  S->info.boxes_evaluated = 1;
  int64_t next_seq = 1;
  push_box(S, root);
  cutoff(S);

  int32_t status = ST_NOT_CONVERGED;
  int64_t sweeps = 0;
  for (;;) {
    if (S->n_live == 0) { status = ST_INTERNAL; break; }
    /* GLB = smallest lower bound in L; stopping criteria (Sec. 3.1) */
    double glb = INFINITY, wmax = 0.0;
    for (int64_t i = 0; i < S->n_live; ++i) { glb = dmin(glb, S->live[i].flo); wmax = dmax(wmax, S->live[i].wmax); }
    S->info.f_lo = glb; S->info.f_hi = S->gub;
    if (up_sub(S->gub, glb) <= P->tol_f && (P->tol_x <= 0.0 || wmax < P->tol_x)) { status = ST_OK; break; }
    if (sweeps >= O->max_sweeps) break;
    if (O->max_live_boxes > 0 && S->n_live > O->max_live_boxes) break;

    /* Select: the K boxes with the smallest (lower bound, seq), removed from L */
    int kk = 0;
    for (; kk < K && S->n_live > 0; ++kk) {
      int64_t best = 0;
      for (int64_t i = 1; i < S->n_live; ++i) if (key_less(&S->live[i], &S->live[best])) best = i;
      par[kk] = S->live[best];
      S->live[best] = S->live[--S->n_live];
    }

    /* Partition each parent on m cycled coordinates d_j = (cyc + j) mod n
     * (Sec. 3.2): cut into `pieces` subintervals each (bisection, or the four
     * equal pieces of Eqs. (10)-(11)); child r takes piece digit_j(r) of d_j.
     * A coordinate whose pieces would not all have positive width is not
     * split; children that would take another piece of it are not formed. */
    int64_t nch = 1;
    for (int j = 0; j < m; ++j) nch *= PC;
    int64_t cap_ch = (int64_t)kk * nch;
    double* ch_flo = (double*)malloc((size_t)cap_ch * sizeof(double));
    double* ch_ub = (double*)malloc((size_t)cap_ch * sizeof(double));
    unsigned char* ch_ok = (unsigned char*)malloc((size_t)cap_ch);
    double gub_new = S->gub;
    for (int p = 0; p < kk; ++p) {
      int dim[64], split[64], dig[64];
      double cut[64][5];
      int split_dim[64], n_split = 0;
      for (int j = 0; j < m; ++j) {
        dim[j] = (int)(((int64_t)par[p].cyc + j) % n);
        split[j] = make_cuts(par[p].lo[dim[j]], par[p].hi[dim[j]], PC, cut[j]);
        if (split[j]) split_dim[n_split++] = dim[j];
      }
      if (general && O->incremental)
        piece_tab_form(P, par[p].lo, par[p].hi, dim, split, (const double(*)[5])cut, m, PC, NS, cs, X, pb.affected,
                       tab);
      else if (O->incremental)
        parent_base_form(P, par[p].lo, par[p].hi, split_dim, n_split, X, &pb);
      for (int64_t r = 0; r < nch; ++r) {
        int64_t c = (int64_t)p * nch + r;
        ch_ok[c] = 0;
        int isvoid = 0;
        int64_t rr = r;
        for (int j = 0; j < m; ++j) {   /* the digits of r, as digit() gives them */
          dig[j] = (int)(rr % PC);
          rr /= PC;
          if (dig[j] && !split[j]) isvoid = 1;
        }
        if (isvoid) continue;
        box_eval e;
        if (general && O->incremental) {
          double w;
          e = piece_child(tab, dig, (const double(*)[5])cut, split, m, PC, NS, &w);
        } else {
          memcpy(clo, par[p].lo, (size_t)n * sizeof(double));
          memcpy(chi, par[p].hi, (size_t)n * sizeof(double));
          for (int j = 0; j < m; ++j) {
            if (!split[j]) continue;
            clo[dim[j]] = cut[j][dig[j]];
            chi[dim[j]] = cut[j][dig[j] + 1];
          }
          e = general ? eval_box_samples(P, clo, chi, X, NS, cs) : eval_box(P, clo, chi, X, NULL);
          if (!general && O->incremental) child_bounds(P, &pb, clo, chi, X, &e.F, &e.ub);
        }
        S->info.boxes_evaluated++;
        ch_flo[c] = e.F.lo;
        ch_ub[c] = e.ub;
        ch_ok[c] = e.mono ? 1 : 2;      /* 1: evaluated but fails the first-order test */
        /* Sample: GUB = smallest upper bound seen (Sec. 3.1) */
        if (e.ub < gub_new) gub_new = e.ub;
      }
    }
    S->gub = gub_new;

    /* Insert survivors: lower bound <= GUB and passing the first-order test */
    int64_t nsurv = 0;
    for (int p = 0; p < kk; ++p) {
      int dim[64], split[64];
      double cut[64][5];
      for (int j = 0; j < m; ++j) {
        dim[j] = (int)(((int64_t)par[p].cyc + j) % n);
        split[j] = make_cuts(par[p].lo[dim[j]], par[p].hi[dim[j]], PC, cut[j]);
      }
      for (int64_t r = 0; r < nch; ++r) {
        int64_t c = (int64_t)p * nch + r;
        if (ch_ok[c] != 2 || ch_flo[c] > S->gub) continue;
        box b;
        b.lo = (double*)malloc((size_t)n * sizeof(double));
        b.hi = (double*)malloc((size_t)n * sizeof(double));
        memcpy(b.lo, par[p].lo, (size_t)n * sizeof(double));
        memcpy(b.hi, par[p].hi, (size_t)n * sizeof(double));
        for (int j = 0; j < m; ++j) {
          if (!split[j]) continue;
          const int d = digit(r, j, PC);
          b.lo[dim[j]] = cut[j][d];
          b.hi[dim[j]] = cut[j][d + 1];
        }
        b.flo = ch_flo[c];
        b.seq = next_seq++;
        b.cyc = (int32_t)(((int64_t)par[p].cyc + m) % n);
        b.wmax = box_wmax(n, b.lo, b.hi);
        if (!push_box(S, b)) { status = ST_NOMEM; goto done; }
        nsurv++;
      }
    }
    int64_t sel0 = par[0].seq;
    for (int p = 0; p < kk; ++p) free_box(&par[p]);
    free(ch_flo); free(ch_ub); free(ch_ok);
    cutoff(S);
    sweeps++;
    if (S->n_trace < S->cap_trace) {
      S->tr_gub[S->n_trace] = S->gub;
      S->tr_nsurv[S->n_trace] = nsurv;
      S->tr_nlive[S->n_trace] = S->n_live;
      S->tr_sel[S->n_trace] = sel0;
      S->n_trace++;
    }
  }
done:
  S->info.sweeps = sweeps;
  S->info.status = status;
  S->info.n_boxes = S->n_live;
  S->info.f_hi = S->gub;
  if (S->n_live) {
    double glb = INFINITY;
    for (int64_t i = 0; i < S->n_live; ++i) glb = dmin(glb, S->live[i].flo);
    S->info.f_lo = glb;
  }
  qsort(S->live, (size_t)S->n_live, sizeof(box), cmp_seq);
  free(X); free(par); free(clo); free(chi); free(pb.affected); free(tab);
  return S;
}

int orc_info_get(void* h, orc_info* out) { if (!h) return -1; *out = ((solve_state*)h)->info; return 0; }

int64_t orc_boxes(void* h, double* lo, double* hi, double* flo, int64_t* seq, int64_t cap) {
  solve_state* S = (solve_state*)h;
  int64_t k = S->n_live < cap ? S->n_live : cap;
  for (int64_t i = 0; i < k; ++i) {
    if (lo) memcpy(lo + i * S->n, S->live[i].lo, (size_t)S->n * sizeof(double));
    if (hi) memcpy(hi + i * S->n, S->live[i].hi, (size_t)S->n * sizeof(double));
    if (flo) flo[i] = S->live[i].flo;
    if (seq) seq[i] = S->live[i].seq;
  }
  return k;
}

int64_t orc_trace(void* h, double* gub, int64_t* nsurv, int64_t* nlive, int64_t* sel, int64_t cap) {
  solve_state* S = (solve_state*)h;
  int64_t k = S->n_trace < cap ? S->n_trace : cap;
  for (int64_t i = 0; i < k; ++i) {
    gub[i] = S->tr_gub[i]; nsurv[i] = S->tr_nsurv[i]; nlive[i] = S->tr_nlive[i]; sel[i] = S->tr_sel[i];
  }
  return k;
}

void orc_free(void* h) {
  solve_state* S = (solve_state*)h;
  if (!S) return;
  for (int64_t i = 0; i < S->n_live; ++i) free_box(&S->live[i]);
  free(S->live);
  free(S->tr_gub); free(S->tr_nsurv); free(S->tr_nlive); free(S->tr_sel);
  free(S);
}

/* ------------------------------------------------------------------------- */
/* per-box and per-operation entry points used by the tests                  */
/* ------------------------------------------------------------------------- */

/* F[nb][2], ub[nb], mono[nb], G[nb][n][2] (G may be NULL) */
int orc_eval_boxes(const orc_problem* P, int64_t nb, const double* lo, const double* hi,
                   double* F, double* ub, unsigned char* mono, double* G) {
  const int64_t n = P->n;
  iv* X = (iv*)malloc((size_t)n * sizeof(iv));
  iv* GG = (iv*)malloc((size_t)n * sizeof(iv));
  for (int64_t b = 0; b < nb; ++b) {
    box_eval e = eval_box(P, lo + b * n, hi + b * n, X, GG);
    F[2 * b] = e.F.lo; F[2 * b + 1] = e.F.hi;
    ub[b] = e.ub;
    mono[b] = (unsigned char)e.mono;
    if (G) for (int64_t j = 0; j < n; ++j) { G[(b * n + j) * 2] = GG[j].lo; G[(b * n + j) * 2 + 1] = GG[j].hi; }
  }
  free(X); free(GG);
  return 0;
}

/* op codes shared with the test suite (values chosen here) */
enum { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_SQRT = 4, OP_SQR = 5, OP_ABS = 6,
       OP_RECIP = 7, OP_COS2PI = 8, OP_SIN2PI = 9, OP_DABS = 10, OP_EXP = 11, OP_COS = 12, OP_SIN = 13 };

/* a, b, out are [cnt][2] (lo, hi) arrays; b is ignored by the unary ops */
int orc_iv_op(int op, int64_t cnt, const double* a, const double* b, double* out) {
  for (int64_t i = 0; i < cnt; ++i) {
    iv x = mk(a[2 * i], a[2 * i + 1]);
    iv y = b ? mk(b[2 * i], b[2 * i + 1]) : mk(0.0, 0.0);
    iv r;
    switch (op) {
    case OP_ADD: r = iv_add(x, y); break;
    case OP_SUB: r = iv_sub(x, y); break;
    case OP_MUL: r = iv_mul(x, y); break;
    case OP_DIV: r = iv_div(x, y); break;
    case OP_SQRT: r = iv_sqrt(x); break;
    case OP_SQR: r = iv_sqr(x); break;
    case OP_ABS: r = iv_abs(x); break;
    case OP_RECIP: r = iv_recip(x); break;
    case OP_COS2PI: r = iv_cos2pi(x); break;
    case OP_SIN2PI: r = iv_sin2pi(x); break;
    case OP_DABS: r = iv_dabs(x); break;
    case OP_EXP: r = iv_exp(x); break;
    case OP_COS: r = iv_cos(x); break;
    case OP_SIN: r = iv_sin(x); break;
    default: return -1;
    }
    out[2 * i] = r.lo; out[2 * i + 1] = r.hi;
  }
  return 0;
}

/* point enclosures: fn 0 = cos(2 pi y), 1 = sin(2 pi y); out [cnt][2] */
int orc_point_trig(int fn, int64_t cnt, const double* y, double* out) {
  for (int64_t i = 0; i < cnt; ++i) pt_trig2pi(fn, y[i], &out[2 * i], &out[2 * i + 1]);
  return 0;
}

/* midpoint rule, exposed for the tests */
double orc_midpoint(double lo, double hi) { return midpoint(lo, hi); }
