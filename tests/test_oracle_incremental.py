"""Pins of the oracle's incremental child bounds (children bounded from their
parent's shared terms plus the terms that involve a split coordinate).

The incremental order only reassociates the sum of the same terms, so:
  * where every operation is exact (chained family, power-of-two coefficients,
    a few sweeps of dyadic boxes) the incremental run must equal the full run
    bit for bit; a term left out, counted twice or taken from the wrong box
    would change the sums;
  * elsewhere both runs enclose the known minimum 0 within the tolerance and
    keep the minimiser in a live box, and their enclosures differ by at most a
    few rounding steps.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR


def run(p, **kw):
    return O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, **kw)


@pytest.mark.parametrize("n,m", [(4, 4), (6, 3), (7, 5)])
def test_exact_chain_runs_identical(n, m):
    # alpha_i, beta_i powers of two, domain [-2, 2.5] (the minimiser x = 1 is not a
    # bisection point, so the run does not stop early): endpoints after s
    # bisections carry at most s + 5 significant bits, so squares and sums stay
    # exact for a few sweeps
    alpha = np.array([2.0 ** (i % 3) for i in range(n - 1)])
    beta = np.array([0.5 * 2.0 ** (i % 2) for i in range(n - 1)])
    p = dataclasses.replace(PR.chain(n, 1, hi=2.5), coef=np.concatenate([alpha, beta]))
    a = run(p, max_sweeps=6, split_dims=m)
    b = run(p, max_sweeps=6, split_dims=m, incremental=True)
    assert a.sweeps == b.sweeps == 6
    assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.trace_nsurv, b.trace_nsurv)
    assert np.array_equal(a.trace_sel, b.trace_sel)
    assert np.array_equal(a.flo, b.flo) and np.array_equal(a.lo, b.lo) and np.array_equal(a.hi, b.hi)


@pytest.mark.parametrize("make", [lambda: PR.sep_cos(2, 101), lambda: PR.sep_cos(9, 2),
                                  lambda: PR.chain(5, 505, hi=2.3), lambda: PR.sep_abs_sin2(12, 4),
                                  lambda: PR.chain(3, 7, hi=2.3)])
def test_incremental_encloses_minimum(make):
    p = make()
    a = run(p, max_sweeps=3000)
    b = run(p, max_sweeps=3000, incremental=True)
    assert b.status == 0 and b.f_lo <= 0.0 <= b.f_hi and b.f_hi - b.f_lo <= p.tol_f
    inside = np.all((b.lo <= p.x_star) & (p.x_star <= b.hi), axis=1)
    assert inside.any()
    # same terms, another order of the additions: a few rounding steps apart
    assert abs(a.f_hi - b.f_hi) <= 1e-12 and abs(a.f_lo - b.f_lo) <= 1e-12


def test_incremental_split_fewer_than_all():
    # coordinates that cannot be split stay unaffected: a box pinned to a point
    # in one coordinate (lower == upper is not allowed, so use a float-width interval)
    p = PR.sep_cos(3, 5)
    lo = p.lower.copy(); hi = p.upper.copy()
    lo[1] = 0.25; hi[1] = np.nextafter(0.25, 1.0)
    q = dataclasses.replace(p, lower=lo, upper=hi, x_star=None)
    a = run(q, max_sweeps=25)
    b = run(q, max_sweeps=25, incremental=True)
    assert a.sweeps == b.sweeps
    assert np.all(np.abs(a.trace_gub - b.trace_gub) <= 1e-12 * (1 + np.abs(a.trace_gub)))
