"""Pins for the oracle's bounds on the three synthetic families.

Each family is a closed form with known minimum 0.  The tests evaluate f and
its partial derivatives at sample points with mpmath (100-bit real arithmetic
on the closed form, not on interval trees) and require the oracle's
enclosures to contain them; they also pin exact values at special points, the
canonical summation (no term lost or counted twice), and the first-order test.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

mpmath.mp.prec = 100


def f_true(p, x):
    """f(x) in mpmath from the closed form of the family."""
    n, cf = p.n, p.coef
    x = [mpmath.mpf(v) for v in x]
    s = mpmath.mpf(0)
    if p.family == PR.SEP_COS:
        a, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        for i in range(n):
            d = x[i] - mpmath.mpf(c[i])
            s += mpmath.mpf(a[i]) * d * d + mpmath.mpf(b[i]) * (1 - mpmath.cospi(2 * mpmath.mpf(k[i]) * d))
    elif p.family == PR.CHAIN:
        al, be = cf[:n - 1], cf[n - 1:]
        for i in range(n - 1):
            s += mpmath.mpf(al[i]) * (x[i + 1] - x[i] ** 2) ** 2 + mpmath.mpf(be[i]) * (x[i] - 1) ** 2
    else:
        sc, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        for i in range(n):
            d = x[i] - mpmath.mpf(c[i])
            s += mpmath.mpf(sc[i]) * abs(d) + mpmath.mpf(b[i]) * mpmath.sinpi(mpmath.mpf(k[i]) * d) ** 2
    return s


def grad_true(p, x, j):
    h = mpmath.mpf(2) ** -40

    def fj(t):
        y = list(map(mpmath.mpf, x))
        y[j] = t
        return f_true(p, y)
    return mpmath.diff(fj, mpmath.mpf(x[j]), h=h)


PROBS = [PR.sep_cos(5, 1), PR.chain(6, 2), PR.sep_abs_sin2(5, 3)]


@pytest.mark.parametrize("p", PROBS, ids=lambda p: p.name)
def test_F_contains_f_and_ub_bounds_midpoint(p):
    lo, hi = PR.random_boxes(p, 60, seed=p.n, max_width_frac=0.3)
    F, ub, mono = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi)
    g = np.random.default_rng(9)
    for b in range(lo.shape[0]):
        assert 0.0 <= F[b, 0] <= F[b, 1]             # every term is non-negative
        for _ in range(4):
            x = lo[b] + g.random(p.n) * (hi[b] - lo[b])
            v = f_true(p, x)
            assert mpmath.mpf(F[b, 0]) <= v <= mpmath.mpf(F[b, 1]), (p.name, b)
        mid = [O.midpoint(lo[b, i], hi[b, i]) for i in range(p.n)]
        fm = f_true(p, mid)
        assert fm <= mpmath.mpf(ub[b])
        assert mpmath.mpf(ub[b]) <= fm + abs(fm) * mpmath.mpf(2) ** -40 + mpmath.mpf(2) ** -1000
        assert F[b, 0] <= ub[b]


@pytest.mark.parametrize("p", PROBS, ids=lambda p: p.name)
def test_G_contains_derivative(p):
    lo, hi = PR.random_boxes(p, 25, seed=100 + p.n, max_width_frac=0.05)
    F, ub, mono, G = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi, want_grad=True)
    g = np.random.default_rng(10)
    for b in range(lo.shape[0]):
        x = lo[b] + (0.05 + 0.9 * g.random(p.n)) * (hi[b] - lo[b])
        for j in range(p.n):
            d = grad_true(p, x, j)
            tol = mpmath.mpf(2) ** -30 * (1 + abs(d))   # numerical differentiation slack
            assert mpmath.mpf(G[b, j, 0]) - tol <= d <= mpmath.mpf(G[b, j, 1]) + tol, (p.name, b, j)


@pytest.mark.parametrize("p", PROBS, ids=lambda p: p.name)
def test_F_width_shrinks_on_small_boxes(p):
    # a box of width w around a point: F must be at most (slope * w * n + rounding) wide;
    # catches a trig enclosure or an operation that ignores its argument
    g = np.random.default_rng(4)
    for _ in range(10):
        x = p.lower + g.random(p.n) * (p.upper - p.lower)
        w = 1e-9
        F, ub, mono = O.eval_boxes(p.family, p.coef, p.lower, p.upper, (x - w)[None], (x + w)[None])
        assert F[0, 1] - F[0, 0] <= 2e-4 * p.n


def test_exact_values_at_minimiser():
    for p in PROBS:
        x = p.x_star
        F, ub, mono = O.eval_boxes(p.family, p.coef, p.lower, p.upper, x[None], x[None])
        assert F[0].tolist() == [0.0, 0.0] and ub[0] == 0.0, p.name


def _unit_sep_cos(n, ones_at=None):
    # a=1, b=0, k=1, c=0 on x = 1: every term equals exactly 1 (or 4 where x = 2)
    coef = np.concatenate([np.ones(n), np.zeros(n), np.ones(n), np.zeros(n)])
    x = np.ones(n)
    if ones_at is not None:
        x[ones_at] = 2.0
    return coef, x


def test_canonical_sum_counts_every_term_once():
    for n in [1, 63, 64, 65, 1000]:
        coef, x = _unit_sep_cos(n)
        F, ub, _ = O.eval_boxes(PR.SEP_COS, coef, -np.ones(n) * 5, np.ones(n) * 5, x[None], x[None])
        assert F[0].tolist() == [n, n] and ub[0] == n
    n = 130
    for j in range(n):
        coef, x = _unit_sep_cos(n, ones_at=j)
        F, _, _ = O.eval_boxes(PR.SEP_COS, coef, -np.ones(n) * 5, np.ones(n) * 5, x[None], x[None])
        assert F[0].tolist() == [n + 3, n + 3], j


def test_first_order_test():
    p = PR.sep_cos(3, 5)
    a, b, k, c = (p.coef[i * 3:(i + 1) * 3] for i in range(4))
    g = np.random.default_rng(8)
    checked = 0
    for _ in range(400):
        x = p.lower + 0.1 + g.random(3) * (p.upper - p.lower - 0.2)
        lo, hi = x - 1e-7, x + 1e-7
        F, ub, mono = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo[None], hi[None])
        d = [float(grad_true(p, x, j)) for j in range(3)]
        if max(abs(v) for v in d) > 1e-2:
            assert mono[0], (x, d)        # a clearly non-zero slope inside the domain
            checked += 1
    assert checked > 300
    # f = (x + 10)^2 on [-5, 5]: slope > 0 everywhere, so the minimum sits on the
    # lower edge; a box touching x = l must stay, the same box moved inward must go
    coef = np.array([1.0, 0.0, 1.0, -10.0])
    lo_d, hi_d = np.array([-5.0]), np.array([5.0])
    for left, pruned in [(-5.0, False), (-4.0, True), (4.0 - 1e-9, True)]:
        lo = np.array([[left]]); hi = lo + 1e-9
        _, _, mono = O.eval_boxes(PR.SEP_COS, coef, lo_d, hi_d, lo, hi)
        assert bool(mono[0]) == pruned, left
    # f = (x - 10)^2: slope < 0, the minimum is on the upper edge
    coef = np.array([1.0, 0.0, 1.0, 10.0])
    for right, pruned in [(5.0, False), (4.0, True)]:
        hi = np.array([[right]]); lo = hi - 1e-9
        _, _, mono = O.eval_boxes(PR.SEP_COS, coef, lo_d, hi_d, lo, hi)
        assert bool(mono[0]) == pruned, right
