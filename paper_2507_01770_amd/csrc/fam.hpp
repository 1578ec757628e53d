// fam.hpp -- natural interval extensions of the three objective families, their
// interval gradients and their point upper bounds, one coordinate at a time.
//
// Expression trees (the natural interval extension of Sec. 2.1: every real
// operation replaced by its outward-rounded interval operation):
//   SEP_COS      D = X_i - c_i, Y = k_i D
//                t_i = a_i sqr(D) + b_i (1 - cos2pi(Y))
//                G_i = (2 a_i) D + [2 pi k_i b_i] sin2pi(Y)
//   SEP_ABS_SIN2 D = X_i - c_i, H = (k_i / 2) D, Y = k_i D
//                t_i = s_i |D| + b_i sqr(sin2pi(H))
//                G_i = s_i dabs(D) + [pi k_i b_i] sin2pi(Y)
//   CHAIN        R_i = X_{i+1} - sqr(X_i), E_i = X_i - 1
//                t_i = alpha_i sqr(R_i) + beta_i sqr(E_i)                 (i < n-1)
//                G_j = ((-4 alpha_j) X_j) R_j + (2 beta_j) E_j            (j < n-1)
//                    (+) (2 alpha_{j-1}) R_{j-1}                          (j >= 1)
// cos2pi(y) = cos(2 pi y), sin2pi(y) = sin(2 pi y).  [c pi k b] are intervals
// built once per problem from the two doubles around pi.
#pragma once
#include "ivl.hpp"

namespace ibb {

enum { FAM_SEP_COS = 1, FAM_CHAIN = 2, FAM_SEP_ABS_SIN2 = 3 };

// per-coordinate coefficients of the separable families
struct alignas(16) CoefSep {
  double a, b, k, c;   // a (SEP_COS) or s (SEP_ABS_SIN2), b, k, c
  I pkb;               // [2 pi k b] (SEP_COS) or [pi k b] (SEP_ABS_SIN2)
};
struct alignas(16) CoefChain {
  double al, be;       // alpha_i, beta_i (zero past the last term)
};

// t_i and G_i of a separable family on the interval X
template <int FAM>
__device__ __forceinline__ void sep_box(const CoefSep& cf, I X, I& t, I& G) {
  const I D = sub_s(X, cf.c);
  if (FAM == FAM_SEP_COS) {
    const I Y = scale(cf.k, D);
    const TrigIv cs = sincos2pi(Y, true, true);
    t = add(scale(cf.a, sqr(D)), scale(cf.b, s_sub(1.0, cs.c)));
    G = add(scale(2.0 * cf.a, D), mul(cf.pkb, cs.s));
  } else {
    const I H = scale(0.5 * cf.k, D);
    const TrigIv sh = sincos2pi(H, false, true);
    t = add(scale(cf.a, iabs(D)), scale(cf.b, sqr(sh.s)));
    const I Y = scale(cf.k, D);
    const TrigIv sy = sincos2pi(Y, false, true);
    G = add(scale(cf.a, dabs(D)), mul(cf.pkb, sy.s));
  }
}

// t_i alone (the same operations as in sep_box)
template <int FAM>
__device__ __forceinline__ I sep_term(const CoefSep& cf, I X) {
  const I D = sub_s(X, cf.c);
  if (FAM == FAM_SEP_COS) {
    const TrigIv cs = sincos2pi(scale(cf.k, D), true, false);
    return add(scale(cf.a, sqr(D)), scale(cf.b, s_sub(1.0, cs.c)));
  } else {
    const TrigIv sh = sincos2pi(scale(0.5 * cf.k, D), false, true);
    return add(scale(cf.a, iabs(D)), scale(cf.b, sqr(sh.s)));
  }
}

// upper endpoint of t_i at the point x (the point interval [x, x])
template <int FAM>
__device__ __forceinline__ double sep_point_hi(const CoefSep& cf, double x) {
  const I D = sub_s(point(x), cf.c);
  if (FAM == FAM_SEP_COS) {
    const I Y = scale(cf.k, D);
    const TrigIv cs = sincos2pi(Y, true, false);
    return add(scale(cf.a, sqr(D)), scale(cf.b, s_sub(1.0, cs.c))).h;
  } else {
    const I H = scale(0.5 * cf.k, D);
    const TrigIv sh = sincos2pi(H, false, true);
    return add(scale(cf.a, iabs(D)), scale(cf.b, sqr(sh.s))).h;
  }
}

// CHAIN: term i from X_i, X_{i+1}; also returns R_i and E_i for the gradient
__device__ __forceinline__ I chain_term(const CoefChain& cf, I Xi, I Xi1, I& R, I& E) {
  R = sub(Xi1, sqr(Xi));
  E = sub_s(Xi, 1.0);
  return add(scale(cf.al, sqr(R)), scale(cf.be, sqr(E)));
}

// CHAIN: G_j from X_{j-1}, X_j, X_{j+1} (has_prev: j >= 1, has_next: j <= n-2)
__device__ __forceinline__ I chain_grad(const CoefChain& cprev, const CoefChain& cj, I Xp, I Xj, I Xn,
                                        bool has_prev, bool has_next) {
  I g{0.0, 0.0};
  if (has_next) {
    const I R = sub(Xn, sqr(Xj));
    const I E = sub_s(Xj, 1.0);
    g = add(mul(scale(-4.0 * cj.al, Xj), R), scale(2.0 * cj.be, E));
  }
  if (has_prev) {
    const I Rp = sub(Xj, sqr(Xp));
    const I B = scale(2.0 * cprev.al, Rp);
    g = has_next ? add(g, B) : B;
  }
  return g;
}

}  // namespace ibb

// ---- the same trees in single precision (the FP32 filter) --------------------
// Coefficients are enclosed in float intervals once per problem; k and k/2 are
// exact (the filter is used only when every k_i <= 2^24).
namespace ibb {

struct alignas(16) CoefSep32 {
  J a, b, c, pkb;      // [a] (or [s]), [b], [c], [2 pi k b] (or [pi k b])
  float k, hk;         // k, k/2
  float pad0, pad1;
};
struct alignas(16) CoefChain32 {
  J al, be;            // [alpha_i], [beta_i] (zero past the last term)
};

template <int FAM>
__device__ __forceinline__ void sep_box32(const CoefSep32& cf, J X, J& t, J& G) {
  const J D = sub32(X, cf.c);
  if (FAM == FAM_SEP_COS) {
    const TrigIv32 cs = sincos2pi32(scale32(cf.k, D), true, true);
    t = add32(mul32(cf.a, sqr32(D)), mul32(cf.b, s_sub32(1.0f, cs.c)));
    G = add32(mul32(scale32(2.0f, cf.a), D), mul32(cf.pkb, cs.s));
  } else {
    const TrigIv32 sh = sincos2pi32(scale32(cf.hk, D), false, true);
    t = add32(mul32(cf.a, abs32(D)), mul32(cf.b, sqr32(sh.s)));
    const TrigIv32 sy = sincos2pi32(scale32(cf.k, D), false, true);
    G = add32(mul32(cf.a, dabs32(D)), mul32(cf.pkb, sy.s));
  }
}

__device__ __forceinline__ J chain_term32(const CoefChain32& cf, J Xi, J Xi1) {
  const J R = sub32(Xi1, sqr32(Xi));
  const J E = add32(Xi, J{1.0f, -1.0f});
  return add32(mul32(cf.al, sqr32(R)), mul32(cf.be, sqr32(E)));
}

__device__ __forceinline__ J chain_grad32(const CoefChain32& cprev, const CoefChain32& cj, J Xp, J Xj, J Xn,
                                          bool has_prev, bool has_next) {
  J g{0.0f, 0.0f};
  if (has_next) {
    const J R = sub32(Xn, sqr32(Xj));
    const J E = add32(Xj, J{1.0f, -1.0f});
    g = add32(mul32(mul32(scale32(-4.0f, cj.al), Xj), R), mul32(scale32(2.0f, cj.be), E));
  }
  if (has_prev) {
    const J B = mul32(scale32(2.0f, cprev.al), sub32(Xj, sqr32(Xp)));
    g = has_next ? add32(g, B) : B;
  }
  return g;
}

}  // namespace ibb
