"""The partition of a selected box, read off the oracle's output boxes.

Child indexing (Sec. 3.1, Eqs. 8-11, with two pieces per coordinate instead of
four): digit j of the child index r (base 2, least significant first) picks
the half of the j-th coordinate of the split window, and the children enter the
list in increasing r.

Variable cycling (Sec. 3.2): a box whose lineage has been split k times has had
the coordinates s mod n, s = 0 .. k*m - 1, bisected once each (split windows of
m consecutive coordinates in index order, wrapping to the first coordinate
after the last).  The worked example of Sec. 3.2 is the fixture
tests/golden/variable_cycling.txt."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "variable_cycling.txt")


def fixture_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.lstrip().startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


def window(n, m, index_in):
    """1-based dimensions split at cycling index index_in, and the children's index"""
    dims = [(index_in - 1 + j) % n + 1 for j in range(m)]
    return dims, (index_in - 1 + m) % n + 1


def test_fixture_is_the_cycling_rule():
    rows = fixture_rows()
    assert len(rows) == 2
    for n, m, index_in, first, last, index_out in rows:
        dims, nxt = window(n, m, index_in)
        assert (dims[0], dims[-1], nxt) == (first, last, index_out)
        assert dims == list(range(first, last + 1))


def split_depths(p, o):
    """times each coordinate of each output box was halved"""
    w0 = p.upper - p.lower
    d = np.log2(w0[None, :] / (o.hi - o.lo))
    di = np.rint(d).astype(np.int64)
    assert np.all(np.abs(d - di) < 1e-9)   # bisection at midpoints: widths are w0 / 2^k
    return di


def check_pattern(p, o, m):
    n = p.upper.shape[0]
    D = split_depths(p, o)
    ks = []
    for d in D:
        tot = int(d.sum())
        assert tot % m == 0
        k = tot // m
        expect = np.bincount(np.arange(k * m) % n, minlength=n)
        assert np.array_equal(d, expect), (k, d)
        ks.append(k)
    return max(ks)


def test_first_row_at_the_example_size():
    # n = 1000, 10 dimensions per iteration: the root (index 1) is split in x1..x10,
    # its children carry index 11, so the second split covers x11..x20
    n, m, index_in, first, last, index_out = fixture_rows()[0]
    p = PR.sep_cos(n, 3)
    o1 = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=1, incremental=True)
    D1 = split_depths(p, o1)
    assert np.all(D1[:, first - 1:last] == 1) and np.all(np.delete(D1, np.s_[first - 1:last], axis=1) == 0)
    o2 = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=2, incremental=True)
    D2 = split_depths(p, o2)
    second = D2[D2.sum(1) == 2 * m]
    assert second.shape[0] > 0
    assert np.all(second[:, : index_out - 1 + m] == 1) and np.all(second[:, index_out - 1 + m:] == 0)


@pytest.mark.parametrize("n,sweeps,min_k", [(30, 60, 4), (25, 60, 4)])
def test_wrap_to_the_first_window(n, sweeps, min_k):
    # the second row (index 991 of 1000 -> x991..x1000, then index 1) needs 99
    # levels at n = 1000; the same rule is checked here with 3 windows (n = 30)
    # and with a window that wraps inside itself (n = 25, m = 10: x21..x25 and
    # x1..x5, then index 6)
    m = 10
    p = PR.sep_cos(n, 5)
    o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=sweeps, incremental=True)
    assert check_pattern(p, o, m) >= min_k
    f = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=sweeps, incremental=False)
    assert check_pattern(p, f, m) >= min_k



def children_of(parent_lo, parent_hi, lo, hi, window):
    """child index of each box (rows of lo/hi) cut from the parent box, from the
    halves it takes in the window's coordinates (Eqs. 8-11 with two pieces)"""
    rs = np.zeros(lo.shape[0], dtype=np.int64)
    outside = np.setdiff1d(np.arange(lo.shape[1]), window)
    assert np.array_equal(lo[:, outside], np.broadcast_to(parent_lo[outside], lo[:, outside].shape))
    assert np.array_equal(hi[:, outside], np.broadcast_to(parent_hi[outside], hi[:, outside].shape))
    for j, c in enumerate(window):
        upper = lo[:, c] != parent_lo[c]
        # lower half [lo, mid], upper half [mid, hi], one split point for all children
        mids = np.concatenate([hi[~upper, c], lo[upper, c]])
        assert np.all(mids == mids[0])
        mid = mids[0]
        assert parent_lo[c] < mid < parent_hi[c]
        assert abs(mid - 0.5 * (parent_lo[c] + parent_hi[c])) <= 2.0 ** -50 * (parent_hi[c] - parent_lo[c])
        assert np.all(hi[upper, c] == parent_hi[c]) and np.all(lo[~upper, c] == parent_lo[c])
        rs |= upper.astype(np.int64) << j
    return rs


@pytest.mark.parametrize("seed", [5, 6])
def test_children_follow_eqs_8_to_11(seed):
    n, m = 12, 10
    p = PR.sep_cos(n, seed)
    o1 = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=1, incremental=True)
    o2 = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=2, incremental=True)
    # sweep 1: the root (cycling index 1) is cut along x1..x10
    order = np.argsort(o1.seq)
    r1 = children_of(p.lower, p.upper, o1.lo[order], o1.hi[order], np.arange(m))
    assert np.all(np.diff(r1) > 0) and o1.lo.shape[0] > 1
    # sweep 2: the box selected then (index 11) is cut along x11, x12, x1..x8
    par = np.nonzero(o1.seq == o2.trace_sel[1])[0]
    assert par.size == 1
    new = o2.seq > o1.seq.max()
    order = np.argsort(o2.seq[new])
    window = (np.arange(m) + m) % n
    r2 = children_of(o1.lo[par[0]], o1.hi[par[0]], o2.lo[new][order], o2.hi[new][order], window)
    assert np.all(np.diff(r2) > 0) and r2.size > 1


def test_one_ulp_coordinates_are_never_split():
    # a coordinate one ulp wide has its split point on an endpoint: it is not
    # split, and the children that would take its upper half are not formed
    p = PR.chain(6, 505, hi=2.3)
    p.lower[2], p.upper[2] = 1.0, np.nextafter(1.0, 2.0)
    p.lower[4], p.upper[4] = 0.5, np.nextafter(0.5, 1.0)
    one = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=6, max_sweeps=1)
    assert one.boxes_evaluated == 1 + 2 ** 4
    for incremental in (False, True):
        r = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, max_sweeps=3000, incremental=incremental)
        assert r.status == O.ST_OK and r.f_hi - r.f_lo <= p.tol_f
        for c in (2, 4):
            assert np.all(r.lo[:, c] == p.lower[c]) and np.all(r.hi[:, c] == p.upper[c])
