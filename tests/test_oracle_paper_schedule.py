"""Pins of the oracle's version of the schedule the paper's experiments use
(Sec. 4): the m cycled coordinates of the selected region cut into four equal
subintervals (Sec. 3.2, Eqs. (8)-(11)), each subregion sampled at S points that
cut its diagonal into S + 1 equal pieces, and the region-width stopping rule.

  * Rastrigin (Eqs. S14-S15) is the separable cosine family with a = 1, b = 10,
    k = 1, c = 0 on [-5.5, 6]^n.  The paper prints 45 iterations and one output
    region at n = 50 (Table S7, fixture tests/golden/paper_schedule_results.txt);
    the closed form behind it, (n / 10) * ceil(log_4(11.5 / 1e-4)) iterations, is
    checked at n = 10, 20, 30 as well.
  * The children of one selected box are the 4^m products of the four pieces,
    in digit order (Eq. (8): I_1 = r mod 4, Eq. (9): I_2 = r div 4), each piece
    [lo + w I, lo + w (I + 1)], and a child is kept exactly when its bound does
    not exceed the new GUB and it passes the first-order test (checked with the
    oracle's box evaluation on all 16 children of a 2-coordinate window).
  * GUB after the first sweep is the smallest value of f at the diagonal sample
    points of the children, up to the outward rounding of the point evaluation:
    f is evaluated there in exact rational arithmetic (chained family, a
    polynomial), at sample coordinates a + (b - a) c_s (c_s the double nearest
    s / (S + 1), each operation rounded up) computed here independently.
  * The memoised incremental bounds take the same decisions as the reference
    evaluation of every child over all n terms.
"""
import math
import os
from fractions import Fraction as Q

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_schedule_results.txt")
PAPER = dict(pieces=4, samples=10, tol_f=1e300, tol_x=1e-4)


def paper_rows():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.lstrip().startswith("#"):
                fn, n, it, reg, src = line.split()
                rows[(fn, int(n))] = (int(it), int(reg), src)
    return rows


def rastrigin(n):
    coef = np.concatenate([np.ones(n), 10.0 * np.ones(n), np.ones(n), np.zeros(n)])
    return coef, np.full(n, -5.5), np.full(n, 6.0)


def test_fixture_is_the_closed_form():
    # every Rastrigin row of the fixture follows (n / 10) ceil(log_4(11.5 / 1e-4))
    levels = math.ceil(math.log(11.5 / 1e-4, 4))
    for (fn, n), (it, reg, src) in paper_rows().items():
        if fn == "rastrigin":
            assert it == n // 10 * levels and reg == 1 and src == "table_S7"


@pytest.mark.parametrize("n", [10, 20, 30, 50])
def test_rastrigin_iterations_and_regions(n):
    coef, lo, hi = rastrigin(n)
    o = O.solve(PR.SEP_COS, coef, lo, hi, incremental=True, max_sweeps=100000, **PAPER)
    want = paper_rows().get(("rastrigin", n))
    it = want[0] if want else n // 10 * math.ceil(math.log(11.5 / 1e-4, 4))
    assert o.status == O.ST_OK and o.sweeps == it
    assert len(o.flo) == (want[1] if want else 1)
    assert np.all(o.hi - o.lo < 1e-4)
    assert np.all((o.lo <= 0.0) & (0.0 <= o.hi))          # the region holds the minimiser
    assert o.f_lo <= 0.0 <= o.f_hi


def _rd(q):
    f = float(q)
    return f if Q(f) <= q else math.nextafter(f, -math.inf)


def _ru(q):
    f = float(q)
    return f if Q(f) >= q else math.nextafter(f, math.inf)


def _diag(a, b, c):
    x = _ru(Q(a) + Q(_ru(Q(_ru(Q(b) - Q(a))) * Q(c))))
    return min(max(x, a), b)


def _chain_f(coef, x):
    n = len(x)
    al, be = coef[:n - 1], coef[n - 1:]
    return sum(Q(al[i]) * (Q(x[i + 1]) - Q(x[i]) ** 2) ** 2 + Q(be[i]) * (Q(x[i]) - 1) ** 2 for i in range(n - 1))


def _children(lo, hi, dims, pieces=4):
    """The 4^m children of [lo, hi] split on dims, in child-index order, with their digits."""
    m = len(dims)
    cuts = []
    for d in dims:
        w = _ru(Q(_ru(Q(hi[d]) - Q(lo[d]))) * Q(1, 4))
        c = [lo[d]] + [min(max(_ru(Q(lo[d]) + Q(_ru(Q(w) * I))), lo[d]), hi[d]) for I in (1, 2, 3)] + [hi[d]]
        cuts.append(c)
    out = []
    for r in range(pieces ** m):
        digs = [(r // pieces ** j) % pieces for j in range(m)]
        clo, chi = lo.copy(), hi.copy()
        for j, d in enumerate(dims):
            clo[d], chi[d] = cuts[j][digs[j]], cuts[j][digs[j] + 1]
        out.append((digs, clo, chi))
    return out


def test_children_digit_order_pruning_and_samples():
    # chained family, n = 3, two coordinates split per sweep: one sweep from the root
    # ([-2, 2.5]: the pieces' endpoints are exact, so Eqs. (10)-(11) hold as printed)
    p = PR.chain(3, 505, lo=-2.0, hi=2.5)
    coef = p.coef
    S = 10
    o1 = O.solve(p.family, coef, p.lower, p.upper, split_dims=2, max_sweeps=1, incremental=True, **PAPER)
    kids = _children(p.lower.copy(), p.upper.copy(), [0, 1])
    # Eqs. (10)-(11): pieces of width (hi - lo) / 4 (exact here), I_1 = r mod 4, I_2 = r div 4
    w = (p.upper - p.lower) / 4
    for r, (digs, clo, chi) in enumerate(kids):
        assert digs == [r % 4, r // 4]
        for j in range(2):
            assert clo[j] == p.lower[j] + w[j] * digs[j] and chi[j] == p.lower[j] + w[j] * (digs[j] + 1)
    # GUB after the sweep: the smallest f over the children's diagonal points
    cs = [(s + 1) / (S + 1) for s in range(S)]
    best = min(_chain_f(coef, [_diag(clo[i], chi[i], c) for i in range(3)]) for _, clo, chi in kids for c in cs)
    gub = o1.trace_gub[0]
    assert Q(gub) >= best and gub <= _ru(best) * (1 + 1e-12) + 1e-300
    # kept exactly when F.lo <= GUB and the first-order test passes, in child-index order
    los = np.array([k[1] for k in kids])
    his = np.array([k[2] for k in kids])
    F, ub, mono = O.eval_boxes(p.family, coef, p.lower, p.upper, los, his)
    keep = [r for r in range(16) if F[r, 0] <= gub and not mono[r]]
    assert o1.trace_nsurv[0] == len(keep) == len(o1.flo)
    for q, r in enumerate(keep):     # o1's boxes come in insertion order
        assert np.array_equal(o1.lo[q], los[r]) and np.array_equal(o1.hi[q], his[r])


@pytest.mark.parametrize("n,m,hi", [(6, 3, 2.3), (5, 2, 2.0), (4, 4, 2.3)])
def test_memoised_incremental_bounds_take_the_reference_decisions(n, m, hi):
    p = PR.chain(n, 505, hi=hi)
    kw = dict(split_dims=m, max_sweeps=8, **PAPER)
    a = O.solve(p.family, p.coef, p.lower, p.upper, incremental=False, **kw)
    b = O.solve(p.family, p.coef, p.lower, p.upper, incremental=True, **kw)
    assert a.sweeps == b.sweeps and a.status == b.status
    assert np.array_equal(a.trace_nsurv, b.trace_nsurv) and np.array_equal(a.trace_sel, b.trace_sel)
    assert np.array_equal(a.trace_nlive, b.trace_nlive)
    assert np.array_equal(a.lo, b.lo) and np.array_equal(a.hi, b.hi) and np.array_equal(a.seq, b.seq)
    assert np.allclose(a.trace_gub, b.trace_gub, rtol=1e-13, atol=0) and np.allclose(a.flo, b.flo, rtol=1e-13, atol=1e-300)
