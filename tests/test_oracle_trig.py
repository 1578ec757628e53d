"""Pins for the oracle's cos(2 pi y) / sin(2 pi y) enclosures, against mpmath.

The point enclosure must contain the true value (computed by mpmath at 200
bits) and be at most one double wider on each side than the tightest outward
rounding.  The interval versions must contain every sampled value and must
include the extremum (+1 or -1) exactly when the interval may hold an integer
or a half-integer (cos) / a quarter point (sin).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O

mpmath.mp.prec = 200


def true_val(fn, y):
    t = 2 * mpmath.mpf(y)   # exact; cospi/sinpi reduce the argument exactly
    return mpmath.cospi(t) if fn == "cos2pi" else mpmath.sinpi(t)


def rd(v):
    d = float(v)
    if mpmath.mpf(d) > v:
        d = math.nextafter(d, -math.inf)
    return d


def ru(v):
    d = float(v)
    if mpmath.mpf(d) < v:
        d = math.nextafter(d, math.inf)
    return d


def sample_points(seed, cnt):
    g = np.random.default_rng(seed)
    pts = [g.uniform(-3, 3, cnt), g.uniform(-1e4, 1e4, cnt // 4),
           np.ldexp(g.random(cnt // 4), -g.integers(1, 60, cnt // 4))]
    quarters = np.round(g.uniform(-400, 400, cnt // 4)) * 0.125
    nudge = np.array([math.nextafter(q, math.inf) for q in quarters] + [math.nextafter(q, -math.inf) for q in quarters])
    special = np.array([0.0, -0.0, 0.125, 0.25, 0.375, 0.5, 0.75, 1.0, -0.25, -0.5, 2.0 ** 52, 2.0 ** 60,
                        2.0 ** 52 + 0.5 * 0 + 1, 1e300, -1e300, 0.1, 1 / 3, 2.0 ** -1074])
    return np.concatenate(pts + [quarters, nudge, special])


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_point_enclosure_contains_and_tight(fn):
    y = sample_points(11 if fn == "cos2pi" else 12, 1200)
    enc = O.point_trig(fn, y)
    for i, yi in enumerate(y):
        v = true_val(fn, yi)
        lo, hi = enc[i]
        assert mpmath.mpf(lo) <= v <= mpmath.mpf(hi), (fn, yi, lo, hi)
        tl, th = max(rd(v), -1.0), min(ru(v), 1.0)
        assert lo >= math.nextafter(tl, -math.inf) and hi <= math.nextafter(th, math.inf), (fn, yi)


def test_point_enclosure_exact_values():
    c = O.point_trig("cos2pi", np.array([0.0, 0.25, 0.5, 1.0, -0.75, 3.0, 2.0 ** 53]))
    assert c.tolist() == [[1, 1], [0, 0], [-1, -1], [1, 1], [0, 0], [1, 1], [1, 1]]
    s = O.point_trig("sin2pi", np.array([0.0, 0.25, 0.5, -0.25, 7.5, 2.0 ** 60]))
    assert s.tolist() == [[0, 0], [1, 1], [0, 0], [-1, -1], [0, 0], [0, 0]]


def _rand_ivals(seed, cnt):
    g = np.random.default_rng(seed)
    a = g.uniform(-6, 6, cnt)
    w = np.exp(g.uniform(np.log(1e-12), np.log(1.5), cnt))
    return np.stack([a, a + w], axis=1)


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_interval_contains_samples_and_extrema(fn):
    Y = _rand_ivals(21 if fn == "cos2pi" else 22, 600)
    R = O.iv_op(fn, Y)
    g = np.random.default_rng(5)
    shift = 0.0 if fn == "cos2pi" else 0.25   # phase of the maximum
    for i in range(Y.shape[0]):
        a, b = Y[i]
        lo, hi = R[i]
        assert -1.0 <= lo <= hi <= 1.0
        for t in np.concatenate([[a, b], g.uniform(a, b, 6)]):
            v = true_val(fn, t)
            assert mpmath.mpf(lo) <= v <= mpmath.mpf(hi), (fn, a, b, t)
        # a maximum inside <=> hi == 1 (up to the enclosure rounding of the endpoints)
        has_max = math.floor(b - shift) >= math.ceil(a - shift)
        has_min = math.floor(b - shift - 0.5) >= math.ceil(a - shift - 0.5)
        if b - a >= 1.0:
            assert (lo, hi) == (-1.0, 1.0)
            continue
        if has_max:
            assert hi == 1.0
        else:
            tmax = max(true_val(fn, a), true_val(fn, b))
            assert hi <= min(1.0, math.nextafter(ru(tmax), math.inf))
        if has_min:
            assert lo == -1.0
        else:
            tmin = min(true_val(fn, a), true_val(fn, b))
            assert lo >= max(-1.0, math.nextafter(rd(tmin), -math.inf))


def test_interval_width_rule():
    R = O.iv_op("cos2pi", np.array([[0.3, 1.3], [0.3, 1.2999999], [-1e9, 1e9]]))
    assert R[0].tolist() == [-1, 1] and R[2].tolist() == [-1, 1]
    assert R[1, 1] == 1.0 and R[1, 0] == -1.0   # holds 0.5 and 1.0
