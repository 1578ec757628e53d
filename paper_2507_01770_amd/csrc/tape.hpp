// Generic closed-form f (the problem's coefficient array holds an expression
// tape): f = g(R_1, ..., R_K), each R_k a sum or a product over a range of i
// of an element program in x_i, x_{i+1}, i and coefficient columns, g a scalar
// program of the R_k.  This covers the benchmark functions of the paper's SI
// Appendix A (Eqs. S1-S21) and Appendix D (Eq. S22).
//
// Bounds (Sec. 2.1: every operation outward rounded; Sec. 3.1: F, the
// first-order test, sample upper bounds), in this order, which defines them:
//   R_k: element values left to right over i (the first term taken as is);
//   g: ops in order; its adjoints in reverse op order, starting from [1, 1],
//      each contribution added to its operand's adjoint as it is met;
//   element tangents d/dx_i (d0) and d/dx_{i+1} (d1) carried forward;
//   dR_k/dx_j: sum: d0 e_k(j) + d1 e_k(j-1) (the parts that exist);
//              product: d0 e_k(j) * L_k(j), L_k(j) the product of the other
//              terms, (e(start) ... e(j-1)) left to right times
//              (e(j+1) (e(j+2) (... e(stop-1)))) nested from the right;
//   G_j = sum over k (increasing) of adj(R_k) dR_k/dx_j.
// A NaN endpoint from any op makes that op's value the whole line.
#pragma once

#include "kern.hpp"

namespace ibb {

enum : int32_t {
  T_CONST = 0, T_X = 1, T_XNEXT = 2, T_COEF = 3, T_ADD = 4, T_SUB = 5, T_MUL = 6, T_DIV = 7, T_NEG = 8,
  T_SQR = 9, T_SQRT = 10, T_EXP = 11, T_COS = 12, T_SIN = 13, T_COS2PI = 14, T_SIN2PI = 15, T_ABS = 16,
  T_RED = 17, T_INDEX = 18
};

__device__ __forceinline__ I nanfix(I r) {
  return (__builtin_isnan(r.n) || __builtin_isnan(r.h)) ? entire() : r;
}
__device__ __forceinline__ I ineg(I a) { return I{a.h, a.n}; }
__device__ __forceinline__ I icos(I a) { return sincos2pi(mul(a, inv_two_pi()), true, false).c; }
__device__ __forceinline__ I isin(I a) { return sincos2pi(mul(a, inv_two_pi()), false, true).s; }
__device__ __forceinline__ I two_pi_iv() {   // [2 pi] from the doubles around pi (exact doubling)
  return I{neg(2.0 * hexd(0x400921fb54442d18ull)), 2.0 * hexd(0x400921fb54442d19ull)};
}

// the value of one op from its operands' values
__device__ __forceinline__ I tape_value(const TapeOp& o, const I* V, I x0, I x1, int i, const double* cols, int n,
                                        const I* red) {
  switch (o.code) {
    case T_CONST: return I{neg(o.lo), o.hi};
    case T_X: return x0;
    case T_XNEXT: return x1;
    case T_COEF: return point(cols[(int64_t)o.a * n + i]);
    case T_INDEX: return point((double)(i + 1));
    case T_RED: return red[o.a];
    case T_ADD: return nanfix(add(V[o.a], V[o.b]));
    case T_SUB: return nanfix(sub(V[o.a], V[o.b]));
    case T_MUL: return nanfix(mul(V[o.a], V[o.b]));
    case T_DIV: return nanfix(div(V[o.a], V[o.b]));
    case T_NEG: return ineg(V[o.a]);
    case T_SQR: return nanfix(sqr(V[o.a]));
    case T_SQRT: return nanfix(isqrt(V[o.a]));
    case T_EXP: return iexp(V[o.a]);
    case T_COS: return icos(V[o.a]);
    case T_SIN: return isin(V[o.a]);
    case T_COS2PI: return sincos2pi(V[o.a], true, false).c;
    case T_SIN2PI: return sincos2pi(V[o.a], false, true).s;
    case T_ABS: return iabs(V[o.a]);
  }
  return entire();
}

// dh/da of a unary op u = h(a), from the operand's value a and the op's value v
__device__ __forceinline__ I tape_unary_factor(int code, I a, I v) {
  switch (code) {
    case T_NEG: return I{1.0, -1.0};
    case T_SQR: return scale(2.0, a);
    case T_SQRT: return recip(scale(2.0, v));
    case T_EXP: return v;
    case T_COS: return ineg(isin(a));
    case T_SIN: return icos(a);
    case T_COS2PI: return ineg(nanfix(mul(two_pi_iv(), sincos2pi(a, false, true).s)));
    case T_SIN2PI: return nanfix(mul(two_pi_iv(), sincos2pi(a, true, false).c));
    case T_ABS: return dabs(a);
  }
  return entire();
}

__device__ __forceinline__ I acc_add(I s, bool& has, I t) {
  if (has) return nanfix(add(s, t));
  has = true;
  return t;
}

// one element program at index i: values only (TAN = false) or with tangents
template <bool TAN>
__device__ void tape_elem(const TapeOp* ops, int nops, const double* cols, int n, int i, I x0, I x1, I* V, I* D0,
                          I* D1, uint8_t* fl, I& v_out, I& d0_out, I& d1_out, uint8_t& fl_out) {
  for (int q = 0; q < nops; ++q) {
    const TapeOp o = ops[q];
    const I v = tape_value(o, V, x0, x1, i, cols, n, nullptr);
    V[q] = v;
    if (TAN) {
      uint8_t f = 0;
      I d0{0.0, 0.0}, d1{0.0, 0.0};
      switch (o.code) {
        case T_X: d0 = I{-1.0, 1.0}; f = 1; break;
        case T_XNEXT: d1 = I{-1.0, 1.0}; f = 2; break;
        case T_ADD: case T_SUB: {
          const bool s = o.code == T_SUB;
          bool h0 = false, h1 = false;
          if (fl[o.a] & 1) d0 = acc_add(d0, h0, D0[o.a]);
          if (fl[o.a] & 2) d1 = acc_add(d1, h1, D1[o.a]);
          if (fl[o.b] & 1) d0 = acc_add(d0, h0, s ? ineg(D0[o.b]) : D0[o.b]);
          if (fl[o.b] & 2) d1 = acc_add(d1, h1, s ? ineg(D1[o.b]) : D1[o.b]);
          f = (h0 ? 1 : 0) | (h1 ? 2 : 0);
          break;
        }
        case T_MUL: {
          bool h0 = false, h1 = false;
          if (fl[o.a] & 1) d0 = acc_add(d0, h0, nanfix(mul(D0[o.a], V[o.b])));
          if (fl[o.a] & 2) d1 = acc_add(d1, h1, nanfix(mul(D1[o.a], V[o.b])));
          if (fl[o.b] & 1) d0 = acc_add(d0, h0, nanfix(mul(V[o.a], D0[o.b])));
          if (fl[o.b] & 2) d1 = acc_add(d1, h1, nanfix(mul(V[o.a], D1[o.b])));
          f = (h0 ? 1 : 0) | (h1 ? 2 : 0);
          break;
        }
        case T_DIV: {
          const I rb = recip(V[o.b]);
          for (int s = 0; s < 2; ++s) {
            const uint8_t bit = s ? 2 : 1;
            const bool ha = fl[o.a] & bit, hb = fl[o.b] & bit;
            if (!ha && !hb) continue;
            const I da = s ? D1[o.a] : D0[o.a], db = s ? D1[o.b] : D0[o.b];
            I num;
            if (ha && hb) num = nanfix(sub(da, nanfix(mul(v, db))));
            else if (ha) num = da;
            else num = ineg(nanfix(mul(v, db)));
            const I d = nanfix(mul(num, rb));
            if (s) d1 = d; else d0 = d;
            f |= bit;
          }
          break;
        }
        case T_NEG: case T_SQR: case T_SQRT: case T_EXP: case T_COS: case T_SIN: case T_COS2PI: case T_SIN2PI:
        case T_ABS: {
          if (!(fl[o.a] & 3)) break;
          const I k = tape_unary_factor(o.code, V[o.a], v);
          if (fl[o.a] & 1) d0 = nanfix(mul(k, D0[o.a]));
          if (fl[o.a] & 2) d1 = nanfix(mul(k, D1[o.a]));
          f = fl[o.a] & 3;
          break;
        }
        default: break;
      }
      D0[q] = d0;
      D1[q] = d1;
      fl[q] = f;
    }
  }
  v_out = V[nops - 1];
  if (TAN) {
    d0_out = D0[nops - 1];
    d1_out = D1[nops - 1];
    fl_out = fl[nops - 1];
  }
}

// point rows for the sample upper bounds: the midpoint (c < 0) or the diagonal
// point lo + (hi - lo) c of every coordinate of the box X
template <class ROW>
struct PointRow {
  const ROW& X;
  double c;
  __device__ __forceinline__ I get(int i) const {
    const I x = X.get(i);
    return point(c < 0.0 ? midpoint(x) : diag_coord(x, c));
  }
};

// F over the box X; with TEST also the first-order test (Sec. 3.1) against the
// domain [nl, u], and with G != nullptr the gradient ([n][2] real endpoints).
// ws: n intervals per product reduction for this thread (the right products).
// cut: with no gradient asked for, a box whose lower bound exceeds it skips the
// test (mono stays false): the caller discards such a box anyway.
template <class ROW, bool TEST>
__device__ I tape_box(const TapeDev& T, const double* cols, int n, const ROW& X, const double* nl, const double* u,
                      I* ws, bool& mono, double* G, double cut = __builtin_inf()) {
  I V[kTapeMaxOps], D0[kTapeMaxOps], D1[kTapeMaxOps];
  uint8_t fl[kTapeMaxOps];
  I red[kTapeMaxRed];
  I d0, d1;
  uint8_t f;
  for (int k = 0; k < T.K; ++k) {
    const TapeRed R = T.red[k];
    I acc = R.kind ? I{-1.0, 1.0} : I{0.0, 0.0};
    bool have = false;
    for (int i = R.start; i < R.stop; ++i) {
      I v;
      tape_elem<false>(T.op + R.first, R.nops, cols, n, i, X.get(i), i + 1 < n ? X.get(i + 1) : X.get(i), V, D0, D1,
                       fl, v, d0, d1, f);
      acc = have ? (R.kind ? nanfix(mul(acc, v)) : nanfix(add(acc, v))) : v;
      have = true;
    }
    red[k] = acc;
  }
  I SV[kTapeMaxOps];
  const TapeOp* sc = T.op + T.sc_first;
  for (int q = 0; q < T.Q; ++q) SV[q] = tape_value(sc[q], SV, I{0.0, 0.0}, I{0.0, 0.0}, 0, cols, n, red);
  const I F = SV[T.Q - 1];
  mono = false;
  if (!TEST && !G) return F;
  if (!G && lo_or_ninf(neg(F.n)) > cut) return F;
  // adjoints of the scalar program, in reverse op order
  I A[kTapeMaxOps], AR[kTapeMaxRed];
  bool hA[kTapeMaxOps], hR[kTapeMaxRed];
  for (int q = 0; q < T.Q; ++q) { hA[q] = false; A[q] = I{0.0, 0.0}; }
  for (int k = 0; k < T.K; ++k) { hR[k] = false; AR[k] = I{0.0, 0.0}; }
  A[T.Q - 1] = I{-1.0, 1.0};
  hA[T.Q - 1] = true;
  for (int q = T.Q - 1; q >= 0; --q) {
    if (!hA[q]) continue;
    const TapeOp o = sc[q];
    const I a = A[q];
    switch (o.code) {
      case T_RED: AR[o.a] = acc_add(AR[o.a], hR[o.a], a); break;
      case T_ADD: A[o.a] = acc_add(A[o.a], hA[o.a], a); A[o.b] = acc_add(A[o.b], hA[o.b], a); break;
      case T_SUB: A[o.a] = acc_add(A[o.a], hA[o.a], a); A[o.b] = acc_add(A[o.b], hA[o.b], ineg(a)); break;
      case T_MUL:
        A[o.a] = acc_add(A[o.a], hA[o.a], nanfix(mul(a, SV[o.b])));
        A[o.b] = acc_add(A[o.b], hA[o.b], nanfix(mul(a, SV[o.a])));
        break;
      case T_DIV: {
        const I rb = recip(SV[o.b]);
        A[o.a] = acc_add(A[o.a], hA[o.a], nanfix(mul(a, rb)));
        A[o.b] = acc_add(A[o.b], hA[o.b], ineg(nanfix(mul(a, nanfix(mul(SV[q], rb))))));
        break;
      }
      case T_NEG: case T_SQR: case T_SQRT: case T_EXP: case T_COS: case T_SIN: case T_COS2PI: case T_SIN2PI:
      case T_ABS:
        A[o.a] = acc_add(A[o.a], hA[o.a], nanfix(mul(a, tape_unary_factor(o.code, SV[o.a], SV[q]))));
        break;
      default: break;
    }
  }
  // right products of the product reductions, from the right end
  int kp = 0;
  for (int k = 0; k < T.K; ++k) {
    const TapeRed R = T.red[k];
    if (R.kind != 1) continue;
    I* suf = ws + (int64_t)kp * n;
    ++kp;
    if (!hR[k] || R.stop <= R.start) continue;
    I s{0.0, 0.0};
    for (int j = R.stop - 2; j >= R.start; --j) {
      I e;
      tape_elem<false>(T.op + R.first, R.nops, cols, n, j + 1, X.get(j + 1), X.get(j + 1), V, D0, D1, fl, e, d0, d1,
                       f);
      s = j + 1 == R.stop - 1 ? e : nanfix(mul(e, s));
      suf[j] = s;
    }
  }
  // G_j, j increasing: per reduction the element tangents at j (and, for a sum,
  // the x_{i+1} tangent of the term at j - 1 kept from the step before)
  I pd1[kTapeMaxRed], pre[kTapeMaxRed];
  bool hpd1[kTapeMaxRed], hpre[kTapeMaxRed];
  for (int k = 0; k < T.K; ++k) { hpd1[k] = false; hpre[k] = false; pd1[k] = I{0.0, 0.0}; pre[k] = I{0.0, 0.0}; }
  for (int j = 0; j < n; ++j) {
    bool hg = false;
    I g{0.0, 0.0};
    kp = 0;
    for (int k = 0; k < T.K; ++k) {
      const TapeRed R = T.red[k];
      const int kpk = kp;
      if (R.kind == 1) ++kp;
      const bool inr = j >= R.start && j < R.stop;
      I e{0.0, 0.0}, e0{0.0, 0.0}, e1{0.0, 0.0};
      uint8_t ef = 0;
      if (inr)
        tape_elem<true>(T.op + R.first, R.nops, cols, n, j, X.get(j), j + 1 < n ? X.get(j + 1) : X.get(j), V, D0, D1,
                        fl, e, e0, e1, ef);
      if (hR[k]) {
        bool hd = false;
        I d{0.0, 0.0};
        if (R.kind == 0) {
          if (inr && (ef & 1)) d = acc_add(d, hd, e0);
          if (hpd1[k]) d = acc_add(d, hd, pd1[k]);
        } else if (inr && (ef & 1)) {
          const bool hs = j < R.stop - 1;
          const I sj = hs ? ws[(int64_t)kpk * n + j] : I{0.0, 0.0};
          const I loo = hpre[k] && hs ? nanfix(mul(pre[k], sj)) : (hpre[k] ? pre[k] : (hs ? sj : I{-1.0, 1.0}));
          d = nanfix(mul(e0, loo));
          hd = true;
        }
        if (hd) g = acc_add(g, hg, nanfix(mul(AR[k], d)));
      }
      // carried to j + 1
      hpd1[k] = R.kind == 0 && inr && (ef & 2);
      pd1[k] = e1;
      if (R.kind == 1 && inr) {
        pre[k] = hpre[k] ? nanfix(mul(pre[k], e)) : e;
        hpre[k] = true;
      }
    }
    if (G) {
      G[2 * j] = hg ? neg(g.n) : 0.0;
      G[2 * j + 1] = hg ? g.h : 0.0;
    }
    if (TEST && hg) {
      const I x = X.get(j);
      if ((g.n < 0.0 && x.n != nl[j]) || (g.h < 0.0 && x.h != u[j])) mono = true;
    }
  }
  return F;
}

}  // namespace ibb
