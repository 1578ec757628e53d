"""Expression tapes: the paper's benchmark functions (SI Appendix A, Eqs. S1-S21,
and Appendix D, Eq. S22) as inputs for the generic family (inputs only: no
interval arithmetic lives here).

A tape describes f = g(R_1, ..., R_K): each R_k is a sum (kind 0) or a product
(kind 1) over i in a range of an element program in x_i, x_{i+1}, i and
per-coordinate coefficient columns; g is a scalar program over the R_k and
constants.  The encoding (float64, the problem's coefficient array):

  [1, K, Q, C]
  per reduction: [kind, s_off, s_end, t_off, t_end, L] + L ops
                 (i from s_off + (s_end ? n : 0) to t_off + (t_end ? n : 0), exclusive)
  Q scalar ops, the last one's value being f
  C columns of n coefficients
  each op: [code, a, b, c_lo, c_hi]  (a, b: earlier ops of the same program;
           CONST is the interval [c_lo, c_hi]; COEF reads column a at i; RED
           reads reduction a)

Constants that are not doubles (pi, e, 0.1, 1/n, ...) enter as the two
doubles around them, so the tape encloses the function as printed.
"""
from __future__ import annotations

import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

from .problems import Problem

TAPE = 4
(T_CONST, T_X, T_XNEXT, T_COEF, T_ADD, T_SUB, T_MUL, T_DIV, T_NEG, T_SQR, T_SQRT, T_EXP, T_COS, T_SIN,
 T_COS2PI, T_SIN2PI, T_ABS, T_RED, T_INDEX) = range(19)

getcontext().prec = 60
_PI = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
_E = Decimal("2.71828182845904523536028747135266249775724709369995957496696763")


def _down(d: Decimal) -> float:
    f = float(d)
    return f if Decimal(f) <= d else math.nextafter(f, -math.inf)


def _up(d: Decimal) -> float:
    f = float(d)
    return f if Decimal(f) >= d else math.nextafter(f, math.inf)


def enclose(v) -> tuple[float, float]:
    """The doubles around a real given exactly (int, Fraction, or a finite
    decimal string); exact values give a point."""
    if isinstance(v, Fraction):
        lo, hi = float(v), float(v)
        if Fraction(lo) > v:
            lo = math.nextafter(lo, -math.inf)
        if Fraction(hi) < v:
            hi = math.nextafter(hi, math.inf)
        return lo, hi
    d = Decimal(v)
    return _down(d), _up(d)


def enclose_irrational(d: Decimal) -> tuple[float, float]:
    """An irrational known to 60 digits: the doubles around it, one more each way."""
    return math.nextafter(_down(d), -math.inf), math.nextafter(_up(d), math.inf)


class Prog:
    """One program (element or scalar): ops appended in order, each returning its index."""

    def __init__(self):
        self.ops: list[tuple] = []

    def _op(self, code, a=-1, b=-1, lo=0.0, hi=0.0):
        self.ops.append((float(code), float(a), float(b), float(lo), float(hi)))
        return len(self.ops) - 1

    def const(self, lo, hi=None):
        return self._op(T_CONST, lo=lo, hi=lo if hi is None else hi)

    def cenc(self, v):               # a real constant, enclosed
        return self.const(*enclose(v))

    def x(self):
        return self._op(T_X)

    def xnext(self):
        return self._op(T_XNEXT)

    def coef(self, col):
        return self._op(T_COEF, a=col)

    def index(self):                 # i + 1 (the paper's 1-based index)
        return self._op(T_INDEX)

    def red(self, k):
        return self._op(T_RED, a=k)

    def add(self, a, b):
        return self._op(T_ADD, a, b)

    def sub(self, a, b):
        return self._op(T_SUB, a, b)

    def mul(self, a, b):
        return self._op(T_MUL, a, b)

    def div(self, a, b):
        return self._op(T_DIV, a, b)

    def neg(self, a):
        return self._op(T_NEG, a)

    def sqr(self, a):
        return self._op(T_SQR, a)

    def sqrt(self, a):
        return self._op(T_SQRT, a)

    def exp(self, a):
        return self._op(T_EXP, a)

    def cos(self, a):
        return self._op(T_COS, a)

    def sin(self, a):
        return self._op(T_SIN, a)

    def cos2pi(self, a):
        return self._op(T_COS2PI, a)

    def sin2pi(self, a):
        return self._op(T_SIN2PI, a)

    def abs(self, a):
        return self._op(T_ABS, a)


def encode(reductions, scalar: Prog, columns=()) -> np.ndarray:
    """reductions: list of (kind, (s_off, s_end), (t_off, t_end), Prog)."""
    out = [1.0, float(len(reductions)), float(len(scalar.ops)), float(len(columns))]
    for kind, (s_off, s_end), (t_off, t_end), prog in reductions:
        out += [float(kind), float(s_off), float(s_end), float(t_off), float(t_end), float(len(prog.ops))]
        for o in prog.ops:
            out += list(o)
    for o in scalar.ops:
        out += list(o)
    for col in columns:
        out += [float(v) for v in col]
    return np.array(out, dtype=np.float64)


ALL = (0, False), (0, True)       # i = 0 .. n-1
CHAINED = (0, False), (-1, True)  # i = 0 .. n-2 (uses x_{i+1})


def _problem(name, n, coef, lo, hi, x_star, f_star, tol_f=1e-6, tol_x=0.0):
    p = Problem(TAPE, n, coef, np.full(n, float(lo)), np.full(n, float(hi)), tol_f=tol_f, tol_x=tol_x,
                x_star=np.full(n, float(x_star)))
    p.tape_name = name
    p.f_star = f_star
    return p


def ackley(n):
    """Eq. S1 on [-35, 40]^n (Eq. S2); f(0) = 0."""
    e0 = Prog(); e0.sqr(e0.x())
    e1 = Prog(); e1.cos2pi(e1.x())
    g = Prog()
    inv_n = g.cenc(Fraction(1, n))
    r = g.sqrt(g.mul(g.red(0), inv_n))
    t1 = g.mul(g.const(-20.0), g.exp(g.mul(g.cenc("-0.02"), r)))
    t2 = g.exp(g.mul(g.red(1), inv_n))
    c = g.const(*enclose_irrational(20 + _E))
    g.add(g.sub(t1, t2), c)
    return _problem("ackley", n, encode([(0, *ALL, e0), (0, *ALL, e1)], g), -35, 40, 0.0, 0.0)


def belegundu(n):
    """Eq. S3 on [-10, 11]^n (Eq. S4); f(5) = -1."""
    e = Prog(); e.sqr(e.sub(e.x(), e.const(5.0)))
    g = Prog()
    s = g.red(0)
    g.sub(g.mul(g.cenc("0.1"), s), g.cos(g.mul(g.const(5.0), g.sqrt(s))))
    return _problem("belegundu", n, encode([(0, *ALL, e)], g), -10, 11, 5.0, -1.0)


def breiman(n):
    """Eq. S5 on [-1, 2]^n (Eq. S6); f(0) = -0.1 n.  cos(5 pi x) = cos(2 pi (2.5 x))."""
    e = Prog()
    x = e.x()
    e.add(e.mul(e.cenc("-0.1"), e.cos2pi(e.mul(e.const(2.5), x))), e.sqr(x))
    g = Prog(); g.red(0)
    return _problem("breiman", n, encode([(0, *ALL, e)], g), -1, 2, 0.0, float(Fraction(-n, 10)))


def fu(n):
    """Eq. S7 on [-10, 10]^n (Eq. S8); f(0.9) = 1."""
    e = Prog()
    d = e.sqr(e.sub(e.x(), e.cenc("0.9")))
    a = e.mul(e.const(8.0), e.sqr(e.sin(e.mul(e.const(7.0), d))))
    b = e.mul(e.const(6.0), e.sqr(e.sin(e.mul(e.const(14.0), d))))
    e.add(e.add(a, b), d)
    g = Prog(); g.add(g.const(1.0), g.red(0))
    return _problem("fu", n, encode([(0, *ALL, e)], g), -10, 10, 0.9, 1.0)


def griewank(n):
    """Eq. S9 on [-100, 110]^n (Eq. S10); f(0) = 0."""
    e0 = Prog(); e0.mul(e0.sqr(e0.x()), e0.cenc(Fraction(1, 4000)))
    e1 = Prog(); e1.cos(e1.div(e1.x(), e1.sqrt(e1.index())))
    g = Prog(); g.sub(g.add(g.const(1.0), g.red(0)), g.red(1))
    return _problem("griewank", n, encode([(0, *ALL, e0), (1, *ALL, e1)], g), -100, 110, 0.0, 0.0)


def levy(n):
    """Eqs. S11-S12 on [-10, 10]^n (Eq. S13); f(1) = 0.  sin(pi y) = sin(2 pi (y / 2))."""
    def y(p, v):
        return p.add(p.const(1.0), p.mul(p.const(0.25), p.sub(v, p.const(1.0))))

    def s2(p, v):   # sin^2(pi y)
        return p.sqr(p.sin2pi(p.mul(p.const(0.5), v)))
    e0 = Prog(); e0.mul(e0.const(10.0), s2(e0, y(e0, e0.x())))
    e1 = Prog(); e1.sqr(e1.sub(y(e1, e1.x()), e1.const(1.0)))
    e2 = Prog()
    a = e2.sqr(e2.sub(y(e2, e2.x()), e2.const(1.0)))
    e2.mul(a, e2.add(e2.const(1.0), e2.mul(e2.const(10.0), s2(e2, y(e2, e2.xnext())))))
    g = Prog()
    s = g.add(g.add(g.red(0), g.red(1)), g.red(2))
    g.mul(g.mul(g.const(*enclose_irrational(_PI)), g.cenc(Fraction(1, n))), s)
    reds = [(0, (0, False), (1, False), e0), (0, (-1, True), (0, True), e1), (0, *CHAINED, e2)]
    return _problem("levy", n, encode(reds, g), -10, 10, 1.0, 0.0)


def rastrigin(n):
    """Eq. S14 on [-5.5, 6]^n (Eq. S15), written as printed: 10 n + sum (x^2 - 10 cos(2 pi x)); f(0) = 0."""
    e = Prog()
    x = e.x()
    e.sub(e.sqr(x), e.mul(e.const(10.0), e.cos2pi(x)))
    g = Prog(); g.add(g.const(10.0 * n), g.red(0))
    return _problem("rastrigin", n, encode([(0, *ALL, e)], g), -5.5, 6, 0.0, 0.0)


def salomon(n):
    """Eq. S16 on [-100, 110]^n (Eq. S17); f(0) = 0.  cos(2 pi r) with r = sqrt(sum x^2)."""
    e = Prog(); e.sqr(e.x())
    g = Prog()
    r = g.sqrt(g.red(0))
    g.add(g.sub(g.const(1.0), g.cos2pi(r)), g.mul(g.cenc("0.1"), r))
    return _problem("salomon", n, encode([(0, *ALL, e)], g), -100, 110, 0.0, 0.0)


def styblinski(n):
    """Eq. S18 on [-10, 11]^n (Eq. S19), as printed; f(0) = -4 n."""
    e0 = Prog(); e0.sqr(e0.x())
    e1 = Prog(); e1.cos(e1.x())
    g = Prog()
    g.sub(g.mul(g.cenc(Fraction(1, 2 * n)), g.red(0)), g.mul(g.const(4.0 * n), g.red(1)))
    return _problem("styblinski", n, encode([(0, *ALL, e0), (1, *ALL, e1)], g), -10, 11, 0.0, -4.0 * n)


def zabinsky(n):
    """Eq. S20 on [0, pi]^n (Eq. S21; the upper end is the double below pi); f(2 pi / 3) = -3.5."""
    pi6 = enclose_irrational(_PI / 6)
    e0 = Prog(); e0.sin(e0.sub(e0.x(), e0.const(*pi6)))
    e1 = Prog(); e1.sin(e1.mul(e1.const(5.0), e1.sub(e1.x(), e1.const(*pi6))))
    g = Prog(); g.sub(g.mul(g.const(-2.5), g.red(0)), g.red(1))
    p = _problem("zabinsky", n, encode([(1, *ALL, e0), (1, *ALL, e1)], g), 0.0, math.pi, 0.0, -3.5)
    p.x_star = np.full(n, float(2 * _PI / 3))
    return p


def rosenbrock(n):
    """Eq. S22 on [-30, 30]^n (Eq. S23); f(1) = 0."""
    e = Prog()
    x = e.x()
    e.add(e.mul(e.const(100.0), e.sqr(e.sub(e.sqr(x), e.xnext()))), e.sqr(e.sub(x, e.const(1.0))))
    g = Prog(); g.red(0)
    return _problem("rosenbrock", n, encode([(0, *CHAINED, e)], g), -30, 30, 1.0, 0.0)


def sep_cos_tape(p: Problem) -> Problem:
    """The separable cosine family with p's coefficients, as a tape (columns a, b, k, c)."""
    n = p.n
    e = Prog()
    d = e.sub(e.x(), e.coef(3))
    t = e.add(e.mul(e.coef(0), e.sqr(d)), e.mul(e.coef(1), e.sub(e.const(1.0), e.cos2pi(e.mul(e.coef(2), d)))))
    del t
    g = Prog(); g.red(0)
    cols = [p.coef[j * n:(j + 1) * n] for j in range(4)]
    q = Problem(TAPE, n, encode([(0, *ALL, e)], g, cols), p.lower.copy(), p.upper.copy(), tol_f=p.tol_f,
                tol_x=p.tol_x, x_star=p.x_star)
    q.tape_name = "sep_cos_tape"
    q.f_star = 0.0
    return q


PAPER_FUNCTIONS = {"ackley": ackley, "belegundu": belegundu, "breiman": breiman, "fu": fu, "griewank": griewank,
                   "levy": levy, "rastrigin": rastrigin, "salomon": salomon, "styblinski": styblinski,
                   "zabinsky": zabinsky, "rosenbrock": rosenbrock}
