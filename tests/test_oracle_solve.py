"""Pins for the oracle's branch-and-bound iteration (Sec. 3.1-3.3 of the paper).

* completeness: the known minimiser lies in a surviving box after every sweep,
  and the final [GLB, GUB] contains the known minimum 0 at the stated width;
* brute force: for n <= 3 a dense grid (numpy float64) plus a Lipschitz bound
  brackets the true minimum; GLB/GUB must be consistent with the bracket and
  the known minimiser must lie in a surviving box;
* determinism (Sec. 4: no random variation is involved) and budget exits.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR


def inside_some_box(x, lo, hi, slack=0.0):
    return bool(np.any(np.all((lo - slack <= x) & (x <= hi + slack), axis=1)))


def test_workload0_encloses_zero():
    p = PR.config(0)
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6)
    assert r.status == O.ST_OK
    assert r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6
    assert inside_some_box(p.x_star, r.lo, r.hi)


@pytest.mark.parametrize("p", [PR.sep_cos(3, 11), PR.chain(3, 12), PR.sep_abs_sin2(3, 13),
                               PR.sep_cos(12, 14), PR.sep_abs_sin2(12, 15)], ids=lambda p: p.name)
def test_minimiser_never_cut(p):
    full = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=4000)
    assert full.status == O.ST_OK, full.status
    assert full.f_lo <= 0.0 <= full.f_hi and full.f_hi - full.f_lo <= 1e-6
    # the iteration is deterministic, so stopping after s sweeps shows the list at sweep s
    for s in sorted(set(np.linspace(1, full.sweeps, 12).astype(int))):
        r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=int(s))
        assert r.sweeps == s
        assert inside_some_box(p.x_star, r.lo, r.hi), s
        assert r.f_lo <= 0.0 <= r.f_hi
        assert np.array_equal(r.trace_gub, full.trace_gub[:s])


def lipschitz(p):
    """per-coordinate bound on |df/dx_i| over the domain"""
    n, cf = p.n, p.coef
    W = np.maximum(np.abs(p.lower), np.abs(p.upper))
    if p.family == PR.SEP_COS:
        a, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        return 2 * a * (W + np.abs(c)) + 2 * np.pi * k * b
    if p.family == PR.SEP_ABS_SIN2:
        s, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        return s + np.pi * k * b
    al, be = np.append(cf[:n - 1], 0.0), np.append(cf[n - 1:], 0.0)
    alp = np.insert(cf[:n - 1], 0, 0.0)
    R = W + W * W
    return 4 * al * W * R + 2 * be * (W + 1) + 2 * alp * R


def f_grid(p, X):
    """f on points X [..., n] in float64 (closed form)"""
    n, cf = p.n, p.coef
    if p.family == PR.SEP_COS:
        a, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        d = X - c
        return np.sum(a * d * d + b * (1 - np.cos(2 * np.pi * k * d)), axis=-1)
    if p.family == PR.SEP_ABS_SIN2:
        s, b, k, c = cf[:n], cf[n:2 * n], cf[2 * n:3 * n], cf[3 * n:]
        d = X - c
        return np.sum(s * np.abs(d) + b * np.sin(np.pi * k * d) ** 2, axis=-1)
    al, be = cf[:n - 1], cf[n - 1:]
    return np.sum(al * (X[..., 1:] - X[..., :-1] ** 2) ** 2 + be * (X[..., :-1] - 1) ** 2, axis=-1)


@pytest.mark.parametrize("fam,n", list(itertools.product([PR.SEP_COS, PR.CHAIN, PR.SEP_ABS_SIN2], [2, 3])))
def test_brute_force_grid(fam, n):
    p = PR.make(fam, n, 200 + 10 * fam + n)
    pts = 1001 if n == 2 else 121
    axes = [np.linspace(p.lower[i], p.upper[i], pts) for i in range(n)]
    h = (p.upper - p.lower) / (pts - 1)
    G = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, n)
    vals = f_grid(p, G)
    gmin = float(vals.min())
    slack = float(np.sum(lipschitz(p) * h / 2)) + 1e-9
    # the known minimum 0 sits in the grid bracket: checks f and the generator
    assert gmin - slack <= 0.0 <= gmin + 1e-12
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=20000)
    assert r.status == O.ST_OK
    assert r.f_lo <= gmin + 1e-12          # GLB below the true minimum, hence below the grid minimum
    assert r.f_hi >= gmin - slack          # GUB above the true minimum
    assert r.f_hi - r.f_lo <= 1e-6
    assert inside_some_box(p.x_star, r.lo, r.hi)


def test_deterministic_and_select_k():
    p = PR.sep_cos(8, 31)
    a = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6)
    b = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6)
    assert a.f_lo == b.f_lo and a.f_hi == b.f_hi and a.sweeps == b.sweeps
    assert np.array_equal(a.lo, b.lo) and np.array_equal(a.seq, b.seq)
    for k in [2, 7]:
        r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, select_k=k)
        assert r.status == O.ST_OK and r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6
        assert inside_some_box(p.x_star, r.lo, r.hi)


def test_budget_exit_is_still_rigorous():
    p = PR.sep_cos(20, 32)
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=5)
    assert r.status == O.ST_NOT_CONVERGED and r.sweeps == 5
    assert r.f_lo <= 0.0 <= r.f_hi
    assert inside_some_box(p.x_star, r.lo, r.hi)


def test_box_width_criterion():
    p = PR.sep_cos(4, 33)
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, tol_x=1e-4, max_sweeps=20000)
    assert r.status == O.ST_OK
    assert np.all(r.hi - r.lo < 1e-4)
    assert inside_some_box(p.x_star, r.lo, r.hi)


@pytest.mark.parametrize("make,incremental", [(lambda: PR.sep_cos(8, 34), False), (lambda: PR.chain(6, 35, hi=2.3), True),
                                              (lambda: PR.sep_abs_sin2(5, 36), True)])
def test_selection_takes_the_smallest_lower_bound(make, incremental):
    # Sec. 3.1: each iteration takes the listed box with the smallest lower bound
    # (ties: the earlier insertion).  The list after t sweeps is the output of a
    # run stopped there; the box the next sweep selects must be its minimum, and
    # the reported GLB is that minimum's lower bound.
    p = make()
    runs = [O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-9, max_sweeps=t, incremental=incremental)
            for t in range(1, 16)]
    checked = 0
    for a, b in zip(runs, runs[1:]):
        if a.status != O.ST_NOT_CONVERGED or b.sweeps <= a.sweeps:
            break
        assert np.array_equal(b.trace_sel[: a.sweeps], a.trace_sel)   # the same iteration up to there
        best = min(range(a.flo.size), key=lambda i: (a.flo[i], a.seq[i]))
        assert b.trace_sel[a.sweeps] == a.seq[best]
        assert a.f_lo == a.flo[best] and a.f_lo <= a.f_hi
        # cutoff: no listed box has a lower bound above GUB, which never increases
        assert np.all(a.flo <= a.f_hi) and b.f_hi <= a.f_hi and a.f_hi == a.trace_gub[-1]
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("make", [lambda: PR.sep_cos(6, 37), lambda: PR.chain(5, 38, hi=2.3)])
def test_stops_at_the_first_sweep_that_meets_the_tolerance(make):
    # stop as soon as GUB - GLB <= tol_f: one sweep fewer does not meet it
    p = make()
    full = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=100000)
    assert full.status == O.ST_OK and full.f_hi - full.f_lo <= 1e-6 and full.sweeps > 1
    short = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-6, max_sweeps=full.sweeps - 1)
    assert short.status == O.ST_NOT_CONVERGED and short.sweeps == full.sweeps - 1
    assert short.f_hi - short.f_lo > 1e-6
    assert short.f_lo <= full.f_lo and full.f_hi <= short.f_hi   # the enclosure only tightens


@pytest.mark.parametrize("make", [lambda: PR.sep_cos(8, 34), lambda: PR.chain(7, 39, hi=2.3)])
def test_trace_bookkeeping(make):
    # per sweep t: nsurv children enter the list, the selected box leaves it, and a
    # lower GUB may cut listed boxes; with GUB unchanged nothing else leaves.  The
    # live count after sweep t is the size of the output of a run stopped there.
    p = make()
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-9, max_sweeps=40)
    nl, ns, g = r.trace_nlive, r.trace_nsurv, r.trace_gub
    assert nl.size == ns.size == g.size == r.sweeps >= 12
    assert nl[0] == ns[0]
    same_gub = 0
    for t in range(1, r.sweeps):
        assert nl[t] <= nl[t - 1] - 1 + ns[t]
        if g[t] == g[t - 1]:
            assert nl[t] == nl[t - 1] - 1 + ns[t]
            same_gub += 1
    assert same_gub >= 1
    for k in (1, 4, 9):
        s = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-9, max_sweeps=k)
        assert s.flo.size == nl[k - 1] and np.array_equal(s.trace_nlive, nl[:k])


def test_live_box_limit_stops_the_run():
    # the run stops (not converged, enclosure still rigorous) at the first sweep
    # that leaves more live boxes than the limit
    p = PR.sep_cos(8, 34)
    free = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-9, max_sweeps=40)
    nl = free.trace_nlive
    limit = 900
    first = int(np.nonzero(nl > limit)[0][0])
    assert first >= 1
    r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-9, max_sweeps=40, max_live_boxes=limit)
    assert r.status == O.ST_NOT_CONVERGED and r.sweeps == first + 1
    assert r.flo.size == nl[first] and np.array_equal(r.trace_nlive, nl[: first + 1])
    assert r.f_lo <= 0.0 <= r.f_hi


def test_width_criterion_stops_at_the_first_sweep_that_meets_both():
    # with tol_x > 0 the run stops when GUB - GLB <= tol_f and every listed box is
    # narrower than tol_x; one sweep fewer meets only the first or neither
    p = PR.chain(5, 505, hi=2.3)
    base = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, max_sweeps=100000)
    full = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, tol_x=1e-4, max_sweeps=100000)
    assert full.status == O.ST_OK and full.sweeps > base.sweeps
    assert np.all(full.hi - full.lo < 1e-4) and full.f_hi - full.f_lo <= p.tol_f
    short = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, tol_x=1e-4, max_sweeps=full.sweeps - 1)
    assert short.status == O.ST_NOT_CONVERGED
    assert np.any(short.hi - short.lo >= 1e-4) or short.f_hi - short.f_lo > p.tol_f


@pytest.mark.parametrize("lo,hi,n", [(1.0, 2.3, 6), (-3.0, 1.0, 9)])
def test_minimiser_on_the_domain_boundary_is_kept(lo, hi, n):
    # chained family, x* = (1, ..., 1) on the lower (upper) face of the domain: the
    # gradient does not vanish there, and the first-order test must not drop the
    # boxes on that face (Sec. 3.1: a sign of the derivative rules a box out only
    # when the box does not touch the bound on the descending side)
    p = PR.chain(n, 505, lo=lo, hi=hi)
    for incremental in (False, True):
        r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, max_sweeps=3000, incremental=incremental)
        assert r.status == O.ST_OK and r.f_lo <= 0.0 <= r.f_hi
        assert inside_some_box(np.ones(n), r.lo, r.hi)


def test_stop_test_comes_before_the_first_selection():
    # Sec. 3.1: the list starts as the whole domain; when the root already meets
    # the tolerance (or no sweep is allowed) the output is the domain itself, with
    # GLB its lower bound and GUB its midpoint bound
    p = PR.chain(4, 505, hi=2.3)
    F, ub, _ = O.eval_boxes(p.family, p.coef, p.lower, p.upper, p.lower[None], p.upper[None])
    for tol_f, budget, status in ((1e6, 100, O.ST_OK), (1e-6, 0, O.ST_NOT_CONVERGED)):
        r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=tol_f, max_sweeps=budget)
        assert r.status == status and r.sweeps == 0 and r.boxes_evaluated == 1
        assert np.array_equal(r.lo, p.lower[None]) and np.array_equal(r.hi, p.upper[None])
        assert r.f_lo == F[0, 0] and r.f_hi == ub[0] and r.trace_gub.size == 0
