"""Pins for the oracle's interval primitives, against exact rational arithmetic.

Sec. 2.1 of the paper defines the interval operations (Eqs. 3-6) and optimal
outward rounding: the lower endpoint is the largest double <= the exact lower
bound, the upper endpoint the smallest double >= the exact upper bound.  These
tests compute the exact range with Python ``fractions`` and round it outward by
comparing neighbouring doubles, so they share nothing with the oracle's
fesetround arithmetic.  Division is Eq. (6) (multiplication by the rounded
reciprocal), which is not optimal: it is pinned by containment of the exact
range and a bound on the excess.
"""
import math
from fractions import Fraction as Q

import numpy as np
import pytest

from oracle import oracle as O


MAXD = Q(1.7976931348623157e308)


def _near(x: Q) -> float:
    if x > MAXD:
        return math.inf
    if x < -MAXD:
        return -math.inf
    return float(x)


def rd(x: Q) -> float:
    """largest double <= x (-inf below the range)"""
    d = _near(x)
    if d == math.inf:
        return 1.7976931348623157e308
    if d != -math.inf and Q(d) > x:
        d = math.nextafter(d, -math.inf)
    return d


def ru(x: Q) -> float:
    """smallest double >= x (+inf above the range)"""
    d = _near(x)
    if d == -math.inf:
        return -1.7976931348623157e308
    if d != math.inf and Q(d) < x:
        d = math.nextafter(d, math.inf)
    return d


def rand_doubles(g, cnt):
    """Doubles of mixed sign and magnitude, with exact small values and zeros."""
    kind = g.integers(0, 6, cnt)
    mant = 1.0 + g.random(cnt)
    e = g.integers(-60, 60, cnt)
    v = np.ldexp(mant, e)
    v = np.where(kind == 0, np.round(g.uniform(-40, 40, cnt)) * 0.125, v)
    v = np.where(kind == 1, np.ldexp(mant, g.integers(-1000, 1000, cnt)), v)
    v = np.where(kind == 2, 0.0, v)
    sign = np.where(g.random(cnt) < 0.5, -1.0, 1.0)
    return v * sign


def rand_intervals(g, cnt):
    a = rand_doubles(g, cnt)
    b = np.where(g.random(cnt) < 0.15, a, rand_doubles(g, cnt))  # some point intervals
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return np.stack([lo, hi], axis=1)


CNT = 4000


@pytest.fixture(scope="module")
def ab():
    g = np.random.default_rng(20250701)
    return rand_intervals(g, CNT), rand_intervals(g, CNT)


def test_add_sub_optimal(ab):
    A, B = ab
    ra, rs = O.iv_op("add", A, B), O.iv_op("sub", A, B)
    for i in range(CNT):
        al, ah = map(Q, A[i]); bl, bh = map(Q, B[i])
        assert ra[i, 0] == rd(al + bl) and ra[i, 1] == ru(ah + bh), i
        assert rs[i, 0] == rd(al - bh) and rs[i, 1] == ru(ah - bl), i


def test_mul_optimal(ab):
    A, B = ab
    r = O.iv_op("mul", A, B)
    for i in range(CNT):
        P = [Q(x) * Q(y) for x in A[i] for y in B[i]]
        assert r[i, 0] == rd(min(P)) and r[i, 1] == ru(max(P)), i


def test_sqr_abs_optimal(ab):
    A, _ = ab
    rs, ra = O.iv_op("sqr", A), O.iv_op("abs", A)
    for i in range(CNT):
        lo, hi = map(Q, A[i])
        sq_hi = max(lo * lo, hi * hi)
        sq_lo = Q(0) if lo <= 0 <= hi else min(lo * lo, hi * hi)
        assert rs[i, 0] == rd(sq_lo) and rs[i, 1] == ru(sq_hi), i
        ab_lo = Q(0) if lo <= 0 <= hi else min(abs(lo), abs(hi))
        assert ra[i, 0] == float(ab_lo) and ra[i, 1] == float(max(abs(lo), abs(hi))), i


def test_recip_optimal_and_div_contains(ab):
    A, B = ab
    rr, rq = O.iv_op("recip", B), O.iv_op("div", A, B)
    for i in range(CNT):
        bl, bh = map(Q, B[i])
        if bl <= 0 <= bh:
            assert rr[i, 0] == -math.inf and rr[i, 1] == math.inf
            assert rq[i, 0] == -math.inf and rq[i, 1] == math.inf
            continue
        assert rr[i, 0] == rd(1 / bh) and rr[i, 1] == ru(1 / bl), i
        Qs = [Q(x) / Q(y) for x in A[i] for y in B[i]]
        lo, hi = min(Qs), max(Qs)
        assert rq[i, 0] == -math.inf or Q(rq[i, 0]) <= lo, i
        assert rq[i, 1] == math.inf or hi <= Q(rq[i, 1]), i
        # two outward roundings: at most a few units in the last place beyond optimal
        if rq[i, 0] != 0.0 and math.isfinite(rq[i, 0]) and rd(lo) != 0.0:
            assert abs(rq[i, 0] - rd(lo)) <= 4 * math.ulp(rd(lo)), i
        if rq[i, 1] != 0.0 and math.isfinite(rq[i, 1]) and ru(hi) != 0.0:
            assert abs(rq[i, 1] - ru(hi)) <= 4 * math.ulp(ru(hi)), i


def _isqrt_rd(x: Q) -> float:
    """largest double d >= 0 with d*d <= x"""
    d = math.sqrt(float(x))
    while Q(d) * Q(d) > x:
        d = math.nextafter(d, -math.inf)
    while Q(math.nextafter(d, math.inf)) ** 2 <= x:
        d = math.nextafter(d, math.inf)
    return d


def test_sqrt_optimal():
    g = np.random.default_rng(7)
    v = np.abs(rand_doubles(g, 2 * CNT))
    v = np.concatenate([v, [0.0, 1.0, 2.0, 4.0, 0.25, 1e-300, 2.0 ** -1074]])
    w = v * (1.0 + g.random(v.shape[0]))
    A = np.stack([v, np.maximum(v, w)], axis=1)
    r = O.iv_op("sqrt", A)
    for i in range(A.shape[0]):
        lo, hi = map(Q, A[i])
        dl = _isqrt_rd(lo)
        du = _isqrt_rd(hi)
        if Q(du) * Q(du) < hi:
            du = math.nextafter(du, math.inf)
        assert r[i, 0] == dl and r[i, 1] == du, i


def test_dabs_cases():
    A = np.array([[1.0, 2.0], [-3.0, -1.0], [-1.0, 1.0], [0.0, 1.0], [-1.0, 0.0], [0.0, 0.0]])
    r = O.iv_op("dabs", A)
    assert r.tolist() == [[1, 1], [-1, -1], [-1, 1], [-1, 1], [-1, 1], [-1, 1]]


def test_midpoint_rule():
    # rounded-up midpoint, kept inside [lo, hi]; exact when 0.5 lo + 0.5 hi is a double
    assert O.midpoint(-5.0, 5.0) == 0.0
    assert O.midpoint(0.0, 1.0) == 0.5
    a, b = 1.0, math.nextafter(1.0, 2.0)
    assert O.midpoint(a, b) == b          # exact mid lies between: rounded up
    a = math.nextafter(1.0, 0.0)
    assert O.midpoint(a, 1.0) == 1.0
    g = np.random.default_rng(3)
    for _ in range(2000):
        x, y = sorted(rand_doubles(g, 2))
        m = O.midpoint(x, y)
        assert x <= m <= y
        exact = (Q(x) + Q(y)) / 2
        assert m == min(max(ru(exact), x), y)
