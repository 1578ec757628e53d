"""GPU interval arithmetic against the oracle, through the C ABI.

+, -, x, sqr, abs, reciprocal, / (Eq. 6) and sqrt must match the oracle bit for
bit (compared as values, so -0 == +0).  The cos(2 pi y) / sin(2 pi y)
enclosures must contain the oracle's and be at most two doubles wider on each
side; they must also contain the true value (mpmath).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def rand_doubles(g, cnt, emin=-300, emax=300):
    kind = g.integers(0, 5, cnt)
    mant = 1.0 + g.random(cnt)
    v = np.ldexp(mant, g.integers(-60, 60, cnt))
    v = np.where(kind == 0, np.round(g.uniform(-40, 40, cnt)) * 0.125, v)
    v = np.where(kind == 1, np.ldexp(mant, g.integers(emin, emax, cnt)), v)
    v = np.where(kind == 2, 0.0, v)
    return v * np.where(g.random(cnt) < 0.5, -1.0, 1.0)


def rand_intervals(g, cnt, **kw):
    a, b = rand_doubles(g, cnt, **kw), rand_doubles(g, cnt, **kw)
    b = np.where(g.random(cnt) < 0.1, a, b)
    return np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)


def gpu_op(op, A, B=None):
    a = torch.from_numpy(A).cuda()
    b = None if B is None else torch.from_numpy(B).cuda()
    r = ibb.interval_op(op, a, b)
    torch.cuda.synchronize()
    return r.cpu().numpy()


N = 1 << 18


@pytest.mark.parametrize("op", ["add", "sub", "mul", "sqr", "abs", "dabs"])
def test_bit_exact_basic(op):
    g = np.random.default_rng(100 + len(op))
    A, B = rand_intervals(g, N), rand_intervals(g, N)
    print(f"case {op} n={N}", flush=True)
    ref = O.iv_op(op, A, B if op in ("add", "sub", "mul") else None)
    got = gpu_op(op, A, B if op in ("add", "sub", "mul") else None)
    bad = ~((got == ref) | (np.isnan(got) & np.isnan(ref)))
    idx = np.argwhere(bad.any(axis=1)).ravel()
    assert idx.size == 0, (op, A[idx[:3]], B[idx[:3]], got[idx[:3]], ref[idx[:3]])


@pytest.mark.parametrize("op", ["recip", "div", "sqrt"])
def test_bit_exact_div_sqrt(op):
    # operands kept away from the underflow range, where residual correction is not exact
    g = np.random.default_rng(200 + len(op))
    A, B = rand_intervals(g, N, emin=-400, emax=400), rand_intervals(g, N, emin=-400, emax=400)
    if op == "sqrt":
        A = np.abs(A)
        A.sort(axis=1)
    print(f"case {op} n={N}", flush=True)
    args = (A, B) if op == "div" else (A if op == "sqrt" else B,)
    ref = O.iv_op(op, *args)
    got = gpu_op(op, *args)
    bad = ~((got == ref) | (np.isnan(got) & np.isnan(ref)))
    idx = np.argwhere(bad.any(axis=1)).ravel()
    assert idx.size == 0, (op, got[idx[:3]], ref[idx[:3]])


def _okey(x):
    """ordered integer key of doubles: key(a) < key(b) <=> a < b, -0 == +0"""
    b = np.ascontiguousarray(x).view(np.int64)
    return np.where(b < 0, -(b & 0x7fffffffffffffff), b)


def ulps_beyond(outer, inner):
    """how many doubles outer's endpoints lie beyond inner's (per side; <0 = not containing).
    Differences are clipped to +-2^40 so that far-apart values cannot overflow."""
    def steps(a, b):  # number of doubles from a up to b
        ka, kb = _okey(a), _okey(b)
        same_sign = (ka >= 0) == (kb >= 0)
        d = np.where(same_sign, kb - ka, np.sign(kb - ka.astype(np.float64)) * 2 ** 40)
        return np.clip(d, -2 ** 40, 2 ** 40).astype(np.int64)
    return steps(outer[:, 0], inner[:, 0]), steps(inner[:, 1], outer[:, 1])


def report(y, got, ref, dl, dh, limit=5):
    bad = np.argwhere((dl < 0) | (dh < 0) | (dl > 2) | (dh > 2)).ravel()
    return [(float(y[i]).hex(), got[i].tolist(), ref[i].tolist(), int(dl[i]), int(dh[i])) for i in bad[:limit]]


def trig_points(seed, cnt):
    g = np.random.default_rng(seed)
    parts = [g.uniform(-3, 3, cnt), g.uniform(-500, 500, cnt), np.ldexp(g.random(cnt), -g.integers(1, 60, cnt)),
             np.round(g.uniform(-4000, 4000, cnt)) * 0.125]
    q = parts[-1]
    parts += [np.nextafter(q, np.inf), np.nextafter(q, -np.inf), np.nextafter(np.nextafter(q, np.inf), np.inf)]
    parts.append(np.array([0.0, -0.0, 0.125, 0.25, 0.375, 0.5, 1.0, 2.0 ** 52, 2.0 ** 60, 1e300, -1e300, 1 / 3]))
    return np.concatenate(parts)


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_point_trig_contains_oracle_within_two_ulps(fn):
    y = trig_points(7 if fn == "cos2pi" else 8, 1 << 17)
    print(f"case point {fn} n={y.size}", flush=True)
    ref = O.point_trig(fn, y)
    got = ibb.point_trig(fn, torch.from_numpy(y).cuda()).cpu().numpy()
    dl, dh = ulps_beyond(got, ref)
    assert dl.min() >= 0 and dh.min() >= 0, ("GPU enclosure must contain the oracle's", report(y, got, ref, dl, dh))
    assert dl.max() <= 2 and dh.max() <= 2, report(y, got, ref, dl, dh)
    # and the true value (a sample, at 200 bits)
    mpmath.mp.prec = 200
    for i in np.random.default_rng(1).choice(y.size, 400, replace=False):
        t = 2 * mpmath.mpf(y[i])
        v = mpmath.cospi(t) if fn == "cos2pi" else mpmath.sinpi(t)
        assert mpmath.mpf(got[i, 0]) <= v <= mpmath.mpf(got[i, 1])


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_interval_trig_contains_oracle_within_two_ulps(fn):
    g = np.random.default_rng(11 if fn == "cos2pi" else 12)
    a = np.concatenate([g.uniform(-8, 8, 1 << 16), np.round(g.uniform(-64, 64, 1 << 14)) * 0.25])
    w = np.exp(g.uniform(np.log(1e-15), np.log(1.2), a.size))
    w[: 1 << 12] = 0.0
    Y = np.stack([a, a + w], axis=1)
    print(f"case interval {fn} n={Y.shape[0]}", flush=True)
    ref = O.iv_op(fn, Y)
    got = gpu_op(fn, Y)
    dl, dh = ulps_beyond(got, ref)
    assert dl.min() >= 0 and dh.min() >= 0, report(Y[:, 0], got, ref, dl, dh)
    assert dl.max() <= 2 and dh.max() <= 2, report(Y[:, 0], got, ref, dl, dh)


@pytest.mark.parametrize("fn", ["exp", "cos", "sin"])
def test_exp_and_radian_trig_contain_oracle(fn):
    # the generic family's elementary functions: the GPU enclosure holds the
    # oracle's (same argument reduction constants, wider margins) with at most
    # 4 (exp) or 2 (cos, sin) doubles more on each side, and the true value
    g = np.random.default_rng(21 if fn == "exp" else 22)
    a = np.concatenate([g.uniform(-40, 40, 1 << 15), g.uniform(-690, 700, 1 << 12),
                        np.ldexp(g.uniform(-1, 1, 1 << 12), -g.integers(1, 60, 1 << 12)),
                        np.array([0.0, -0.0, 0.5, -0.5, 1.0, np.log(2.0) / 2, -np.log(2.0) / 2])])
    if fn != "exp":
        a = a[np.abs(a) < 1e4]
    w = np.exp(g.uniform(np.log(1e-15), np.log(0.5), a.size)) * (1 + np.abs(a))
    w[: 1 << 12] = 0.0
    Y = np.stack([a, a + w], axis=1)
    print(f"case interval {fn} n={Y.shape[0]}", flush=True)
    ref = O.iv_op(fn, Y)
    got = gpu_op(fn, Y)
    dl, dh = ulps_beyond(got, ref)
    assert dl.min() >= 0 and dh.min() >= 0, ("GPU enclosure must contain the oracle's", report(Y[:, 0], got, ref, dl, dh))
    lim = 4 if fn == "exp" else 2
    assert dl.max() <= lim and dh.max() <= lim, report(Y[:, 0], got, ref, dl, dh)
    mpmath.mp.prec = 200
    f = {"exp": mpmath.exp, "cos": mpmath.cos, "sin": mpmath.sin}[fn]
    for i in np.random.default_rng(2).choice(a.size, 300, replace=False):
        v = f(mpmath.mpf(a[i]))
        assert mpmath.mpf(got[i, 0]) <= v <= mpmath.mpf(got[i, 1])
