// ivl.hpp -- outward-rounded interval arithmetic for gfx950 wavefronts.
//
// Every kernel that includes this header switches its wave to round-toward-+inf
// (MODE.FP_ROUND = +inf for both f32 and f64) as its first statement, and
// represents an interval [lo, hi] as the pair (n, h) = (-lo, hi).  Then every
// endpoint is a single hardware operation rounded up:
//   lower endpoint of a sum   RD(a + b)  = -RU((-a) + (-b))  ->  n = n_a + n_b
//   upper endpoint            RU(a + b)                      ->  h = h_a + h_b
// and a product whose lower endpoint needs RD(x*y) uses RU(-(x*y)), issued as
// one multiply with a negated source operand.  This is the outward rounding of
// Sec. 2.1 (lower endpoint rounded down, upper rounded up), with Eqs. (3)-(6)
// written for the negated lower endpoint.
//
// The compiler assumes round-to-nearest and may legally move a negation across
// a multiply (-(x*y) == (-x)*y under round-to-nearest, not under round-up).  So
// no code here negates the result or an operand of a multiply, divide or fma in
// plain C++: such negations go through the opaque helpers below (one VALU
// instruction each, or a source modifier), and constants are hex literals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibb {

// -------------------------------------------------------------------------
// rounding mode and opaque helpers
// -------------------------------------------------------------------------

// MODE[3:0] = FP_ROUND: bits 1:0 f32, bits 3:2 f64/f16; 1 = toward +inf.
__device__ __forceinline__ void round_up_mode() {
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 4), 5\n\ts_nop 3" ::: "memory");
}

// RU(-(a*b))
__device__ __forceinline__ double mul_neg(double a, double b) {
  double r;
  asm("v_mul_f64 %0, -%1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// -a, exact, invisible to the optimiser
__device__ __forceinline__ double neg(double a) {
  double r;
  asm("v_mul_f64 %0, %1, -1.0" : "=v"(r) : "v"(a));
  return r;
}
// RU(a*b - c); exact when the result is representable (residuals of products)
__device__ __forceinline__ double fms(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, -%3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
// RU(c - a*b)
__device__ __forceinline__ double fnma(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

__device__ __forceinline__ double hexd(uint64_t u) { return __builtin_bit_cast(double, u); }
__device__ __forceinline__ double dmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return __builtin_fmin(a, b); }

// next double up / down (finite arguments)
__device__ __forceinline__ double next_up(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  if (x == 0.0) return hexd(1ull);
  u = (int64_t)u >= 0 ? u + 1 : u - 1;
  return __builtin_bit_cast(double, u);
}
__device__ __forceinline__ double next_down(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  if (x == 0.0) return hexd(0x8000000000000001ull);
  u = (int64_t)u >= 0 ? u - 1 : u + 1;
  return __builtin_bit_cast(double, u);
}

// -------------------------------------------------------------------------
// intervals: I{n, h} is [-n, h]
// -------------------------------------------------------------------------
struct I {
  double n, h;
};

__device__ __forceinline__ I point(double x) { return I{neg(x), x}; }
__device__ __forceinline__ double lo_of(I a) { return neg(a.n); }

// Eq. (3)
__device__ __forceinline__ I add(I a, I b) { return I{a.n + b.n, a.h + b.h}; }
// Eq. (4): [a.lo - b.hi, a.hi - b.lo]
__device__ __forceinline__ I sub(I a, I b) { return I{a.n + b.h, a.h + b.n}; }
// a - c for a scalar c
__device__ __forceinline__ I sub_s(I a, double c) { return I{a.n + c, a.h - c}; }
// c - a for a scalar c
__device__ __forceinline__ I s_sub(double c, I a) { return I{a.h - c, c + a.n}; }

// s * a for a scalar s (Eq. (5) with a degenerate first factor)
__device__ __forceinline__ I scale(double s, I a) {
  double as = __builtin_fabs(s);
  double p = as * a.n, q = as * a.h;
  return s >= 0.0 ? I{p, q} : I{q, p};
}

// Eq. (5): lower = min of the four products rounded down, upper = max rounded up
__device__ __forceinline__ I mul(I a, I b) {
  // products of (lo_a, hi_a) x (lo_b, hi_b) with lo = -n:
  //   lo_a lo_b = n_a n_b,  lo_a hi_b = -(n_a h_b),  hi_a lo_b = -(h_a n_b),  hi_a hi_b
  double hi = dmax(dmax(a.n * b.n, a.h * b.h), dmax(mul_neg(a.n, b.h), mul_neg(a.h, b.n)));
  double nl = dmax(dmax(a.n * b.h, a.h * b.n), dmax(mul_neg(a.n, b.n), mul_neg(a.h, b.h)));
  return I{nl, hi};
}

// x^2 as one operation
__device__ __forceinline__ I sqr(I a) {
  const bool nonneg = a.n <= 0.0;   // lo >= 0
  const bool nonpos = a.h <= 0.0;   // hi <= 0
  double p = nonneg ? a.n : a.h;    // endpoint nearest zero (up to sign)
  double q = nonneg ? a.h : (nonpos ? a.n : dmax(a.n, a.h));
  double nl = (nonneg || nonpos) ? mul_neg(p, p) : 0.0;
  return I{nl, q * q};
}

__device__ __forceinline__ I iabs(I a) {
  if (a.n <= 0.0) return a;                 // lo >= 0
  if (a.h <= 0.0) return I{a.h, a.n};       // [-hi, -lo]
  return I{0.0, dmax(a.n, a.h)};
}

// enclosure of the generalized derivative of |x|
__device__ __forceinline__ I dabs(I a) {
  if (a.n < 0.0) return I{-1.0, 1.0};       // lo > 0: {1}
  if (a.h < 0.0) return I{1.0, -1.0};       // hi < 0: {-1}
  return I{1.0, 1.0};                       // [-1, 1]
}

// --- division and square root (directed results by residual correction) ---

// smallest double >= x / y  (y != 0, finite operands, no underflow)
__device__ inline double div_ru(double x, double y) {
  double q = x / y;
  // residual r = x - q y (exact for q within an ulp); q < x/y  <=>  r / y > 0
  for (int it = 0; it < 4; ++it) {
    double r = fnma(q, y, x);
    bool below = (y > 0.0) ? (r > 0.0) : (r < 0.0);
    if (!below) break;
    q = next_up(q);
  }
  for (int it = 0; it < 4; ++it) {
    double p = next_down(q);
    double r = fnma(p, y, x);
    bool p_ok = (y > 0.0) ? (r <= 0.0) : (r >= 0.0);   // p >= x / y
    if (!p_ok) break;
    q = p;
  }
  return q;
}
// largest double <= x / y
__device__ inline double div_rd(double x, double y) {
  double q = x / y;
  for (int it = 0; it < 4; ++it) {
    double r = fnma(q, y, x);
    bool above = (y > 0.0) ? (r < 0.0) : (r > 0.0);
    if (!above) break;
    q = next_down(q);
  }
  for (int it = 0; it < 4; ++it) {
    double p = next_up(q);
    double r = fnma(p, y, x);
    bool p_ok = (y > 0.0) ? (r >= 0.0) : (r <= 0.0);   // p <= x / y
    if (!p_ok) break;
    q = p;
  }
  return q;
}
__device__ inline double sqrt_ru(double x) {
  if (x <= 0.0) return 0.0;
  double s = __builtin_sqrt(x);
  for (int it = 0; it < 4; ++it) { if (!(fnma(s, s, x) > 0.0)) break; s = next_up(s); }
  for (int it = 0; it < 4; ++it) { double p = next_down(s); if (!(p >= 0.0 && fnma(p, p, x) <= 0.0)) break; s = p; }
  return s;
}
__device__ inline double sqrt_rd(double x) {
  if (x <= 0.0) return 0.0;
  double s = __builtin_sqrt(x);
  for (int it = 0; it < 4; ++it) { if (!(fnma(s, s, x) < 0.0)) break; s = next_down(s); }
  for (int it = 0; it < 4; ++it) { double p = next_up(s); if (!(fnma(p, p, x) >= 0.0)) break; s = p; }
  return s;
}

__device__ __forceinline__ I entire() { return I{__builtin_inf(), __builtin_inf()}; }

__device__ inline I recip(I b) {
  if (!(b.n < 0.0 || b.h < 0.0)) return entire();     // 0 in b
  double lo = div_rd(1.0, b.h), hi = div_ru(1.0, lo_of(b));
  return I{neg(lo), hi};
}
// Eq. (6)
__device__ inline I div(I a, I b) {
  I r = recip(b);
  if (r.n == __builtin_inf()) return r;
  return mul(a, r);
}
__device__ inline I isqrt(I a) {
  if (a.h < 0.0) return entire();
  double lo = a.n < 0.0 ? sqrt_rd(lo_of(a)) : 0.0;
  return I{neg(lo), sqrt_ru(a.h)};
}

// -------------------------------------------------------------------------
// cos(2 pi y), sin(2 pi y)
//
// Reduction (exact): f = |y| - nearest integer (via floor), a = |f|, and one
// reduced argument g with |g| <= 1/8 serves both functions:
//   a <= 1/8:        cos = C(a),          sin = sgn(y) sgn(f) S(a)
//   1/8 < a <= 3/8:  cos = S(1/4 - a),    sin = sgn(y) sgn(f) C(1/4 - a)
//   a > 3/8:         cos = -C(1/2 - a),   sin = sgn(y) sgn(f) S(1/2 - a)
// with S(g) = sin(2 pi g), C(g) = cos(2 pi g).
//
// S(g) = A0 g + A1 g^3 + g^5 P(g^2), A_k = (-1)^k (2pi)^(2k+1) / (2k+1)!
// C(g) = 1 + B1 g^2 + g^4 Q(g^2),    B_k = (-1)^k (2pi)^(2k) / (2k)!
// The first two terms of each are carried as an unevaluated sum w + t (A0,
// A1 and B1 split into two doubles, products split exactly with fma, the
// rounding error of the leading addition recovered exactly by Sterbenz), the
// tail in plain round-up arithmetic.  The result w + t is within about
// 0.02 * 2^-52 |w| (S) or 0.07 * 2^-52 (C) of the true value, the Taylor
// truncation (degree 17 / 18) below 2^-62.  The enclosure adds a margin E
// (2^-55 |w| for S, 2^-54 for C) on each side and rounds outward, so it holds
// the true value, holds any enclosure of the form [v - 2^-58 |v|, v + 2^-58 |v|]
// with v within 2^-62 relative of the truth, and is at most two doubles wider
// than that on each side.
// -------------------------------------------------------------------------

struct TrigEnc {
  I c, s;   // enclosures of cos(2 pi y) and sin(2 pi y)
};

__device__ __forceinline__ TrigEnc sincos2pi_point(double y) {
  // reduce |y| with floor (exact, independent of the rounding mode):
  // fr in [0, 1), f in (-1/2, 1/2];  cos is even, sin odd in y
  const double ay = __builtin_fabs(y);
  const double fr = ay - __builtin_floor(ay);
  const double f = fr > 0.5 ? fr - 1.0 : fr;
  const double a = __builtin_fabs(f);
  const bool oct0 = a <= 0.125, oct1 = a <= 0.375;
  const double g = oct0 ? a : (oct1 ? 0.25 - a : 0.5 - a);   // exact, |g| <= 1/8
  // exact square: z + zl = g^2
  const double z = g * g;
  const double zl = fms(g, g, z);

  // ---- S(g) ----
  const double A0h = hexd(0x401921fb54442d18ull), A0l = hexd(0x3cb1a62633145c07ull);
  const double A1h = hexd(0xc044abbce625be53ull), A1l = hexd(0x3ce05511c68476a8ull);
  // p + pe = A0h g exactly
  const double p = A0h * g;
  const double pe = fms(A0h, g, p);
  // g^3 = r1 + r1e + g zl (r1 + r1e = g z exactly)
  const double r1 = g * z;
  const double r1e = fms(g, z, r1);
  // A1 g^3 ~= q + qe + (A1h (r1e + g zl) + A1l r1)
  const double q = A1h * r1;
  const double qe = fms(A1h, r1, q);
  // leading sum p + q, |q| <= 0.103 |p|, opposite signs: error recovered exactly
  const double ws = p + q;
  const double ds = q - (ws - p);
  // tail A2 g^5 + ... + A8 g^17 = g z^2 (A2 + z (A3 + ...))
  double ts = hexd(0x3fbaaec32af93359ull);                  // A8
  ts = __builtin_fma(z, ts, hexd(0xbfe6fadb9f155744ull));   // A7
  ts = __builtin_fma(z, ts, hexd(0x400e8f434d018d63ull));   // A6
  ts = __builtin_fma(z, ts, hexd(0xc02e3074fde8871full));   // A5
  ts = __builtin_fma(z, ts, hexd(0x40450783487ee782ull));   // A4
  ts = __builtin_fma(z, ts, hexd(0xc0532d2cce62bd86ull));   // A3
  ts = __builtin_fma(z, ts, hexd(0x405466bc6775aae2ull));   // A2
  const double g5 = r1 * z;
  double lo_s = ds + pe;
  lo_s = lo_s + qe;
  lo_s = __builtin_fma(A0l, g, lo_s);
  lo_s = __builtin_fma(A1h, __builtin_fma(g, zl, r1e), lo_s);
  lo_s = __builtin_fma(A1l, r1, lo_s);
  lo_s = __builtin_fma(g5, ts, lo_s);
  const double Es = __builtin_fabs(ws) * hexd(0x3c80000000000000ull);   // 2^-55 |w|
  // enclosure: [w + t - E, w + t + E] rounded outward
  I S{(Es - lo_s) - ws, ws + (lo_s + Es)};
  // |g| < 2^-900: the split products above are no longer exact near the
  // subnormal range; there 2 pi g (1 - 2^-54) < sin(2 pi g) <= 2 pi g, so
  // [RD(PI2_LO g), RU(PI2_HI g)] (g >= 0; odd for g < 0) encloses S
  if (__builtin_fabs(g) < hexd(0x07b0000000000000ull)) {
    const double ag = __builtin_fabs(g);
    const double lo_m = mul_neg(hexd(0x401921fb54442d18ull), ag);   // -RD(PI2_LO |g|)
    const double hi_m = hexd(0x401921fb54442d19ull) * ag;            //  RU(PI2_HI |g|)
    S = g >= 0.0 ? I{lo_m, hi_m} : I{hi_m, lo_m};
  }

  // ---- C(g) ----
  const double B1h = hexd(0xc033bd3cc9be45deull), B1l = hexd(0xbcd692b71366cc04ull);
  // B1 g^2 ~= u + ue + (B1h zl + B1l z)
  const double u = B1h * z;
  const double ue = fms(B1h, z, u);
  const double wc = 1.0 + u;                // in [0.69, 1]
  const double dc = u - (wc - 1.0);         // exact
  double tc = hexd(0xbfa2a0c591af8314ull);                   // B9
  tc = __builtin_fma(z, tc, hexd(0x3fd20c62c2f2d7f5ull));    // B8
  tc = __builtin_fma(z, tc, hexd(0xbffb6e24f44b128full));    // B7
  tc = __builtin_fma(z, tc, hexd(0x401f9d38a3763cc3ull));    // B6
  tc = __builtin_fma(z, tc, hexd(0xc03a6d1f2a204a8cull));    // B5
  tc = __builtin_fma(z, tc, hexd(0x404e1f506891babbull));    // B4
  tc = __builtin_fma(z, tc, hexd(0xc0555d3c7e3cbffaull));    // B3
  tc = __builtin_fma(z, tc, hexd(0x40503c1f081b5ac4ull));    // B2
  const double z2 = z * z;
  double lo_c = dc + ue;
  lo_c = __builtin_fma(B1h, zl, lo_c);
  lo_c = __builtin_fma(B1l, z, lo_c);
  lo_c = __builtin_fma(z2, tc, lo_c);
  const double Ec = (g == 0.0) ? 0.0 : hexd(0x3c90000000000000ull);   // 2^-54
  I C{(Ec - lo_c) - wc, wc + (lo_c + Ec)};

  // ---- assemble by octant and sign ----
  TrigEnc r;
  // cos: C, S, or -C
  r.c = oct0 ? C : (oct1 ? S : I{C.h, C.n});
  // sin: sgn(f) * (S, C, S)
  I sv = (oct0 || !oct1) ? S : C;
  r.s = ((f < 0.0) != (y < 0.0)) ? I{sv.h, sv.n} : sv;
  // clamp to [-1, 1]
  r.c.n = dmin(r.c.n, 1.0); r.c.h = dmin(r.c.h, 1.0);
  r.s.n = dmin(r.s.n, 1.0); r.s.h = dmin(r.s.h, 1.0);
  return r;
}

// does [-n, h] hold an integer?  ceil(lo) <= floor(hi)  <=>  floor(n) + floor(h) >= 0
__device__ __forceinline__ bool has_int(double n, double h) {
  return __builtin_floor(n) + __builtin_floor(h) >= 0.0;
}

// interval cos(2 pi Y) and sin(2 pi Y) together (they share the reduction)
struct TrigIv {
  I c, s;
};
__device__ __forceinline__ TrigIv sincos2pi(I y, bool want_cos, bool want_sin) {
  TrigIv r;
  const I whole{1.0, 1.0};
  if (!(y.n + y.h < 1.0)) {                 // width (rounded up) >= 1 period, or NaN
    r.c = whole; r.s = whole;
    return r;
  }
  TrigEnc ea = sincos2pi_point(lo_of(y));
  TrigEnc eb = sincos2pi_point(y.h);
  r.c = I{dmax(ea.c.n, eb.c.n), dmax(ea.c.h, eb.c.h)};
  r.s = I{dmax(ea.s.n, eb.s.n), dmax(ea.s.h, eb.s.h)};
  if (want_cos) {
    if (has_int(y.n, y.h)) r.c.h = 1.0;                       // max at y in Z
    if (has_int(y.n + 0.5, y.h - 0.5)) r.c.n = 1.0;           // min at y in Z + 1/2
  }
  if (want_sin) {
    if (has_int(y.n + 0.25, y.h - 0.25)) r.s.h = 1.0;         // max at y in Z + 1/4
    if (has_int(y.n - 0.25, y.h + 0.25)) r.s.n = 1.0;         // min at y in Z - 1/4
  }
  return r;
}

// -------------------------------------------------------------------------
// exp, and cos / sin of an argument in radians (the generic family's
// elementary functions; Sec. 2.1 asks every operation to round outward)
//
// exp at a double x: x = k ln2 + r with k = rint(x log2 e); r is enclosed from
// ln2 = LN2_HI + LN2_LO + d (LN2_HI has 42 bits, so k LN2_HI is exact for
// |k| < 2^11; |d| < 2^-102, so |k d| < 2^-91 is covered by a margin of 2^-90);
// e^r, |r| < 0.36, by interval Horner over the Taylor coefficients 1/j!,
// j <= 16, each the pair of doubles around it, plus the truncation bound
// |r|^17 e^|r| / 17! < 2^-72; then the exact scaling by 2^k.  Outside
// [-700, 709] the bounds are e^-700 < 1e-304 and e^709 > 8.2e307.
// cos x and sin x: cos(2 pi y), sin(2 pi y) of y = x [1 / (2 pi)], the factor
// enclosed by the two doubles around 1 / (2 pi).
// -------------------------------------------------------------------------
__device__ inline I exp_point(double x) {
  if (x == 0.0) return I{-1.0, 1.0};
  if (x != x) return entire();
  if (x > 709.0) return I{-8.2e307, __builtin_inf()};
  if (x < -700.0) return I{0.0, 1e-304};
  const double kd = __builtin_rint(x * hexd(0x3ff71547652b82feull));   // any integer near x / ln2
  const I kI = point(kd);
  I r = sub(point(x), mul(kI, point(hexd(0x3fe62e42fefa3800ull))));    // x - k LN2_HI
  r = sub(r, mul(kI, point(hexd(0x3d2ef35793c76730ull))));            // - k LN2_LO
  const double m90 = hexd(0x3a50000000000000ull);                      // 2^-90
  r = I{r.n + m90, r.h + m90};
  // 1/j!, j = 0 .. 16: (lower, upper)
  const uint64_t cl[17] = {0x3ff0000000000000ull, 0x3ff0000000000000ull, 0x3fe0000000000000ull,
                           0x3fc5555555555555ull, 0x3fa5555555555555ull, 0x3f81111111111111ull,
                           0x3f56c16c16c16c16ull, 0x3f2a01a01a01a01aull, 0x3efa01a01a01a01aull,
                           0x3ec71de3a556c733ull, 0x3e927e4fb7789f5cull, 0x3e5ae64567f544e3ull,
                           0x3e21eed8eff8d897ull, 0x3de6124613a86d09ull, 0x3da93974a8c07c9dull,
                           0x3d6ae7f3e733b81full, 0x3d2ae7f3e733b81full};
  const uint64_t ch[17] = {0x3ff0000000000000ull, 0x3ff0000000000000ull, 0x3fe0000000000000ull,
                           0x3fc5555555555556ull, 0x3fa5555555555556ull, 0x3f81111111111112ull,
                           0x3f56c16c16c16c17ull, 0x3f2a01a01a01a01bull, 0x3efa01a01a01a01bull,
                           0x3ec71de3a556c734ull, 0x3e927e4fb7789f5dull, 0x3e5ae64567f544e4ull,
                           0x3e21eed8eff8d898ull, 0x3de6124613a86d0aull, 0x3da93974a8c07c9eull,
                           0x3d6ae7f3e733b820ull, 0x3d2ae7f3e733b820ull};
  I p{neg(hexd(cl[16])), hexd(ch[16])};
  for (int j = 15; j >= 0; --j) p = add(mul(p, r), I{neg(hexd(cl[j])), hexd(ch[j])});
  const double m72 = hexd(0x3b70000000000000ull);                      // 2^-72
  p = I{p.n + m72, p.h + m72};
  return scale(__builtin_ldexp(1.0, (int)kd), p);                      // exact power of two
}
__device__ inline I iexp(I a) {
  if (a.n != a.n || a.h != a.h) return I{-0.0, __builtin_inf()};
  const I l = exp_point(neg(a.n)), h = exp_point(a.h);
  return I{dmin(l.n, 0.0), h.h};   // the lower end is never below 0
}
__device__ __forceinline__ I inv_two_pi() { return I{neg(hexd(0x3fc45f306dc9c882ull)), hexd(0x3fc45f306dc9c883ull)}; }

// ordered 64-bit key of a double: key(x) < key(y) <=> x < y (for x, y not NaN, -0 < +0)
__host__ __device__ __forceinline__ uint64_t okey(double x) {
  uint64_t u = __builtin_bit_cast(uint64_t, x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double okey_inv(uint64_t k) {
  uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __builtin_bit_cast(double, u);
}

}  // namespace ibb

// =========================================================================
// Single precision: the FP32 filter.  Same representation [-n, h] and the same
// round-up MODE (its f32 field is set too).  A double interval is enclosed in
// single precision with the conversion's rounding checked, so the enclosure
// holds whatever rounding the conversion used.
// =========================================================================
namespace ibb {

__device__ __forceinline__ float mul_neg32(float a, float b) {
  float r;
  asm("v_mul_f32 %0, -%1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float neg32(float a) {
  float r;
  asm("v_mul_f32 %0, %1, -1.0" : "=v"(r) : "v"(a));
  return r;
}
__device__ __forceinline__ float next_up32(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if (x == 0.0f) return __builtin_bit_cast(float, 1u);
  u = (int32_t)u >= 0 ? u + 1 : u - 1;
  return __builtin_bit_cast(float, u);
}
__device__ __forceinline__ float f32max(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ float f32min(float a, float b) { return __builtin_fminf(a, b); }

struct J {
  float n, h;
};

// smallest float >= x (checked after the conversion)
__device__ __forceinline__ float up32(double x) {
  float f = (float)x;
  if ((double)f < x) f = next_up32(f);
  return f;
}
__device__ __forceinline__ J to32(I x) { return J{up32(x.n), up32(x.h)}; }

__device__ __forceinline__ J add32(J a, J b) { return J{a.n + b.n, a.h + b.h}; }
__device__ __forceinline__ J sub32(J a, J b) { return J{a.n + b.h, a.h + b.n}; }
__device__ __forceinline__ J s_sub32(float c, J a) { return J{a.h - c, c + a.n}; }   // exact scalar c
__device__ __forceinline__ J scale32(float s, J a) {                                // exact scalar s
  const float as = __builtin_fabsf(s);
  const float p = as * a.n, q = as * a.h;
  return s >= 0.0f ? J{p, q} : J{q, p};
}
__device__ __forceinline__ J mul32(J a, J b) {
  const float hi = f32max(f32max(a.n * b.n, a.h * b.h), f32max(mul_neg32(a.n, b.h), mul_neg32(a.h, b.n)));
  const float nl = f32max(f32max(a.n * b.h, a.h * b.n), f32max(mul_neg32(a.n, b.n), mul_neg32(a.h, b.h)));
  return J{nl, hi};
}
__device__ __forceinline__ J sqr32(J a) {
  const bool nonneg = a.n <= 0.0f, nonpos = a.h <= 0.0f;
  const float p = nonneg ? a.n : a.h;
  const float q = nonneg ? a.h : (nonpos ? a.n : f32max(a.n, a.h));
  const float nl = (nonneg || nonpos) ? mul_neg32(p, p) : 0.0f;
  return J{nl, q * q};
}
__device__ __forceinline__ J abs32(J a) {
  if (a.n <= 0.0f) return a;
  if (a.h <= 0.0f) return J{a.h, a.n};
  return J{0.0f, f32max(a.n, a.h)};
}
__device__ __forceinline__ J dabs32(J a) {
  if (a.n < 0.0f) return J{-1.0f, 1.0f};
  if (a.h < 0.0f) return J{1.0f, -1.0f};
  return J{1.0f, 1.0f};
}

// cos(2 pi y), sin(2 pi y) at a float y: the exact reduction of sincos2pi_point,
// then degree-9 / degree-10 Taylor polynomials in single precision (round-up).
// Their rounding error is below 3 * 2^-23 relative (sine) and absolute (cosine),
// the truncation below 2^-28; the enclosure adds a margin of 2^-19 (plus 2^-126
// absolute on the sine, which covers a subnormal product).
struct TrigEnc32 {
  J c, s;
};
__device__ __forceinline__ TrigEnc32 sincos2pi_point32(float y) {
  const float ay = __builtin_fabsf(y);
  const float fr = ay - __builtin_floorf(ay);
  const float f = fr > 0.5f ? fr - 1.0f : fr;
  const float a = __builtin_fabsf(f);
  const bool oct0 = a <= 0.125f, oct1 = a <= 0.375f;
  const float g = oct0 ? a : (oct1 ? 0.25f - a : 0.5f - a);
  const float z = g * g;
  // A_k = (-1)^k (2pi)^(2k+1)/(2k+1)!,  B_k = (-1)^k (2pi)^(2k)/(2k)!  (rounded to float)
  float ps = __builtin_bit_cast(float, 0x42283c1au);            // A4  42.06
  ps = __builtin_fmaf(z, ps, __builtin_bit_cast(float, 0xc2996966u));   // A3 -76.71
  ps = __builtin_fmaf(z, ps, __builtin_bit_cast(float, 0x42a335e3u));   // A2  81.61
  ps = __builtin_fmaf(z, ps, __builtin_bit_cast(float, 0xc2255de7u));   // A1 -41.34
  ps = __builtin_fmaf(z, ps, __builtin_bit_cast(float, 0x40c90fdbu));   // A0   6.283
  const float sv = g * ps;
  float pc = __builtin_bit_cast(float, 0xc1d368f9u);            // B5 -26.43
  pc = __builtin_fmaf(z, pc, __builtin_bit_cast(float, 0x4270fa83u));   // B4  60.24
  pc = __builtin_fmaf(z, pc, __builtin_bit_cast(float, 0xc2aae9e4u));   // B3 -85.46
  pc = __builtin_fmaf(z, pc, __builtin_bit_cast(float, 0x4281e0f8u));   // B2  64.94
  pc = __builtin_fmaf(z, pc, __builtin_bit_cast(float, 0xc19de9e6u));   // B1 -19.74
  const float cv = __builtin_fmaf(z, pc, 1.0f);
  const float Es = __builtin_fmaf(__builtin_fabsf(sv), 0x1p-19f, 0x1p-126f);
  const float Ec = g == 0.0f ? 0.0f : 0x1p-19f;
  const J S{Es - sv, sv + Es};
  const J C{Ec - cv, cv + Ec};
  TrigEnc32 r;
  r.c = oct0 ? C : (oct1 ? S : J{C.h, C.n});
  const J sv2 = (oct0 || !oct1) ? S : C;
  r.s = ((f < 0.0f) != (y < 0.0f)) ? J{sv2.h, sv2.n} : sv2;
  r.c.n = f32min(r.c.n, 1.0f); r.c.h = f32min(r.c.h, 1.0f);
  r.s.n = f32min(r.s.n, 1.0f); r.s.h = f32min(r.s.h, 1.0f);
  return r;
}
__device__ __forceinline__ bool has_int32(float n, float h) { return __builtin_floorf(n) + __builtin_floorf(h) >= 0.0f; }

struct TrigIv32 {
  J c, s;
};
__device__ __forceinline__ TrigIv32 sincos2pi32(J y, bool want_cos, bool want_sin) {
  TrigIv32 r;
  const J whole{1.0f, 1.0f};
  if (!(y.n + y.h < 1.0f)) { r.c = whole; r.s = whole; return r; }
  const TrigEnc32 ea = sincos2pi_point32(neg32(y.n));
  const TrigEnc32 eb = sincos2pi_point32(y.h);
  r.c = J{f32max(ea.c.n, eb.c.n), f32max(ea.c.h, eb.c.h)};
  r.s = J{f32max(ea.s.n, eb.s.n), f32max(ea.s.h, eb.s.h)};
  if (want_cos) {
    if (has_int32(y.n, y.h)) r.c.h = 1.0f;
    if (has_int32(y.n + 0.5f, y.h - 0.5f)) r.c.n = 1.0f;
  }
  if (want_sin) {
    if (has_int32(y.n + 0.25f, y.h - 0.25f)) r.s.h = 1.0f;
    if (has_int32(y.n - 0.25f, y.h + 0.25f)) r.s.n = 1.0f;
  }
  return r;
}

}  // namespace ibb
