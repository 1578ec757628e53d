"""Pins of the oracle's generic family (an expression tape: sums and products over
the coordinates, an outer scalar expression, forward tangents in the element
programs and adjoints in the scalar one) on the benchmark functions of the
paper's SI Appendix A (Eqs. S1-S21) and Appendix D (Eq. S22):

  * the values the paper prints: under the schedule of Sec. 4 (four pieces per
    cycled coordinate, ten diagonal samples, stop at width 1e-4) every Appendix A
    function gives one output region and (n / m) * L iterations, L being the
    iterations of Tables S2-S10 and Table 2 per pass over 10 coordinates; the
    oracle reproduces L for all ten functions (n = 4, m = 2) and several
    regions for Rosenbrock, as Table S11 reports;
  * the closed-form minima f(x*) of Appendix A, inside the point enclosure;
  * the true value (mpmath, 50 digits, from the equations as printed) at random
    points, inside the point enclosure, and at points of random boxes, inside F;
  * the true partial derivatives (mpmath) at a box's centre, inside G (this
    checks the element tangents, the scalar adjoints and the leave-one-out
    products of the product reductions);
  * a one-term separable cosine tape, whose op sequence is the family's tree,
    gives the family's F and midpoint bound bit for bit;
  * n = 2 solves enclose the known minimum, and a brute-force grid agrees;
  * a malformed tape gives the whole real line, never a false enclosure.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR
from paper_2507_01770_amd import tapes as TP

mp.mp.dps = 50
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_schedule_results.txt")


def f_exact(name, x):
    """The functions of Appendix A / D as printed, in mpmath (sin(pi t), cos(pi t)
    through sinpi / cospi, exact at rational t)."""
    n = len(x)
    x = [v if isinstance(v, mp.mpf) else mp.mpf(float(v)) for v in x]
    pi = mp.pi
    if name == "ackley":
        return (-20 * mp.e ** (mp.mpf("-0.02") * mp.sqrt(sum(v * v for v in x) / n))
                - mp.e ** (sum(mp.cospi(2 * v) for v in x) / n) + 20 + mp.e)
    if name == "belegundu":
        s = sum((v - 5) ** 2 for v in x)
        return mp.mpf("0.1") * s - mp.cos(5 * mp.sqrt(s))
    if name == "breiman":
        return -mp.mpf("0.1") * sum(mp.cospi(5 * v) for v in x) + sum(v * v for v in x)
    if name == "fu":
        return 1 + sum(8 * mp.sin(7 * (v - mp.mpf("0.9")) ** 2) ** 2 + 6 * mp.sin(14 * (v - mp.mpf("0.9")) ** 2) ** 2
                       + (v - mp.mpf("0.9")) ** 2 for v in x)
    if name == "griewank":
        p = mp.mpf(1)
        for i, v in enumerate(x):
            p *= mp.cos(v / mp.sqrt(i + 1))
        return 1 + sum(v * v for v in x) / 4000 - p
    if name == "levy":
        y = [1 + (v - 1) / 4 for v in x]
        s = 10 * mp.sinpi(y[0]) ** 2 + (y[-1] - 1) ** 2
        s += sum((y[i] - 1) ** 2 * (1 + 10 * mp.sinpi(y[i + 1]) ** 2) for i in range(n - 1))
        return pi / n * s
    if name == "rastrigin":
        return 10 * n + sum(v * v - 10 * mp.cospi(2 * v) for v in x)
    if name == "salomon":
        r = mp.sqrt(sum(v * v for v in x))
        return 1 - mp.cospi(2 * r) + mp.mpf("0.1") * r
    if name == "styblinski":
        p = mp.mpf(1)
        for v in x:
            p *= mp.cos(v)
        return sum(v * v for v in x) / (2 * n) - 4 * n * p
    if name == "zabinsky":
        p1 = p2 = mp.mpf(1)
        for v in x:
            p1 *= mp.sin(v - pi / 6)
            p2 *= mp.sin(5 * (v - pi / 6))
        return -mp.mpf("2.5") * p1 - p2
    if name == "rosenbrock":
        return sum(100 * (x[i] ** 2 - x[i + 1]) ** 2 + (x[i] - 1) ** 2 for i in range(n - 1))
    raise KeyError(name)


NAMES = list(TP.PAPER_FUNCTIONS)


def ev(p, lo, hi, grad=False):
    return O.eval_boxes(p.family, p.coef, p.lower, p.upper, np.atleast_2d(lo), np.atleast_2d(hi), want_grad=grad)


def contains(lo, hi, v):
    return mp.mpf(lo) <= v <= mp.mpf(hi)


def paper_rows():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.lstrip().startswith("#"):
                fn, n, it, reg, src = line.split()
                rows[(fn, int(n))] = (int(it), int(reg))
    return rows


@pytest.mark.parametrize("name", NAMES)
def test_closed_form_minimum_and_point_values(name):
    for n in (1, 3, 5):
        if name in ("levy", "rosenbrock") and n < 2:
            continue
        p = TP.PAPER_FUNCTIONS[name](n)
        F, ub, mono = ev(p, p.x_star, p.x_star)
        assert F[0, 0] <= p.f_star <= F[0, 1], (n, F[0], p.f_star)
        assert contains(F[0, 0], F[0, 1], f_exact(name, p.x_star))
        rng = np.random.default_rng(17 + n)
        for _ in range(8):
            x = p.lower + rng.uniform(0, 1, n) * (p.upper - p.lower)
            F, ub, mono = ev(p, x, x)
            v = f_exact(name, x)
            assert contains(F[0, 0], F[0, 1], v), (name, n, x, F[0], v)
            assert F[0, 1] - F[0, 0] <= 1e-9 * (1 + abs(float(v))) and ub[0] == F[0, 1]


@pytest.mark.parametrize("name", NAMES)
def test_box_enclosure_holds_sampled_values(name):
    n = 4
    p = TP.PAPER_FUNCTIONS[name](n)
    rng = np.random.default_rng(29)
    for b in range(6):
        w = (p.upper - p.lower) * rng.uniform(1e-6, 0.2, n)
        lo = p.lower + rng.uniform(0, 1, n) * (p.upper - p.lower - w)
        hi = lo + w
        F, ub, mono = ev(p, lo, hi)
        for _ in range(10):
            x = lo + rng.uniform(0, 1, n) * (hi - lo)
            assert contains(F[0, 0], F[0, 1], f_exact(name, x)), (name, b)


@pytest.mark.parametrize("name", NAMES)
def test_gradient_encloses_the_derivative(name):
    n = 4
    p = TP.PAPER_FUNCTIONS[name](n)
    rng = np.random.default_rng(41)
    for b in range(3):
        c = p.lower + rng.uniform(0.05, 0.95, n) * (p.upper - p.lower)
        h = (p.upper - p.lower) * 1e-3
        lo, hi = c - h, c + h
        F, ub, mono, G = ev(p, lo, hi, grad=True)
        for j in range(n):
            def fj(t, j=j):
                x = list(c)
                x[j] = t
                return f_exact(name, x)
            d = mp.diff(fj, mp.mpf(float(c[j])))
            assert contains(G[0, j, 0], G[0, j, 1], d), (name, b, j, G[0, j], d)


def test_one_term_cosine_tape_is_the_family_bit_for_bit():
    base = PR.sep_cos(1, 3)
    tape = TP.sep_cos_tape(base)
    lo, hi = PR.random_boxes(base, 40, seed=5, max_width_frac=0.5)
    F1, u1, m1 = O.eval_boxes(base.family, base.coef, base.lower, base.upper, lo, hi)
    F2, u2, m2 = O.eval_boxes(tape.family, tape.coef, tape.lower, tape.upper, lo, hi)
    assert np.array_equal(F1, F2) and np.array_equal(u1, u2)


@pytest.mark.parametrize("name", NAMES)
def test_paper_schedule_iterations_and_regions(name):
    # Tables S2-S10, Table 2 (n = 50 and 100, m = 10): iterations = (n / 10) L and
    # one region; the same L per pass over the cycled coordinates at n = 4, m = 2
    n, m = 4, 2
    p = TP.PAPER_FUNCTIONS[name](n)
    o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e300, tol_x=1e-4, split_dims=m, max_sweeps=2000,
                pieces=4, samples=10)
    assert o.status == O.ST_OK
    assert np.any(np.all((o.lo <= p.x_star) & (p.x_star <= o.hi), axis=1))
    assert np.all(o.hi - o.lo < 1e-4)
    rows = paper_rows()
    if name == "rosenbrock":   # Table S11: several output regions (9 at n = 50)
        assert rows[("rosenbrock", 50)][1] > 1 and len(o.flo) > 1
        return
    for n_table in (50, 100):
        it, reg = rows[(name, n_table)]
        L = it // (n_table // 10)
        assert it == (n_table // 10) * L and reg == 1
        assert o.sweeps == (n // m) * L, (name, o.sweeps, L)
        assert len(o.flo) == reg


@pytest.mark.parametrize("name", NAMES)
def test_two_dimensional_solve_and_grid(name):
    p = TP.PAPER_FUNCTIONS[name](2)
    o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=20000)
    assert o.status == O.ST_OK and o.f_lo <= p.f_star <= o.f_hi and o.f_hi - o.f_lo <= 1e-6
    # a 201 x 201 grid (double evaluation is enough here): its smallest value is >= GLB
    g = np.linspace(p.lower[0], p.upper[0], 201)
    best = min(float(f_exact(name, [a, b])) for a in g[::10] for b in g[::10])
    assert o.f_lo <= best + 1e-12


def test_malformed_tape_gives_the_whole_line():
    p = TP.ackley(3)
    bad = p.coef.copy()
    bad[0] = 2.0   # unknown format
    F, ub, mono = O.eval_boxes(p.family, bad, p.lower, p.upper, p.lower[None], p.upper[None])
    assert F[0, 0] == -math.inf and F[0, 1] == math.inf
    bad = p.coef.copy()
    bad[4 + 6 + 5 + 1] = 7.0   # an operand that is not an earlier op
    F, ub, mono = O.eval_boxes(p.family, bad, p.lower, p.upper, p.lower[None], p.upper[None])
    assert F[0, 0] == -math.inf and F[0, 1] == math.inf
