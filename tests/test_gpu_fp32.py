"""The FP32 filter on the GPU (ibb_interval_op32, ibb_point_trig32, ibb_eval_boxes
with IBB_FP32_BULK, ibb_solve with IBB_FP32_BULK).

The paper bounds in FP64 throughout; the filter is an addition whose results are
rigorous but not defined bit for bit by the paper, so it is checked against
what the mathematics fixes rather than against the oracle's bits:
  * +, -, x, sqr and |.| in single precision must give the tightest float
    enclosure of the exact result (computed with rationals);
  * cos(2 pi y), sin(2 pi y) enclosures must contain the value computed with
    120-bit mpmath and stay narrow;
  * box bounds must contain f and grad f at sample points of the box (whose
    values the oracle encloses in FP64 on point boxes);
  * whole solves must still enclose the known minimum 0 within the tolerance,
    keep the minimiser in a live box, and be deterministic and the same alone
    and in a batch.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402

mpmath = pytest.importorskip("mpmath")

F32 = np.float32


def _down(q: Fraction) -> np.float32:
    """largest float <= q"""
    f = F32(float(q))
    while Fraction(float(f)) > q:
        f = np.nextafter(f, F32(-np.inf))
    while Fraction(float(np.nextafter(f, F32(np.inf)))) <= q:
        f = np.nextafter(f, F32(np.inf))
    return f


def _up(q: Fraction) -> np.float32:
    return -_down(-q)


def _rand_intervals(rng, count):
    mags = rng.choice([1e-30, 1e-3, 1.0, 7.0, 1e5, 1e15], size=(count, 2))
    v = (rng.standard_normal((count, 2)) * mags).astype(F32)
    lo, hi = np.minimum(v[:, 0], v[:, 1]), np.maximum(v[:, 0], v[:, 1])
    k = rng.integers(0, 6, size=count)
    lo[k == 0] = 0.0                      # touching zero
    hi[k == 1] = lo[k == 1]               # points
    lo[k == 2] = -hi[k == 2]              # symmetric
    return np.stack([lo, hi], axis=1).astype(F32)


def _exact(op, a, b):
    al, ah = Fraction(float(a[0])), Fraction(float(a[1]))
    if op == "add":
        return al + Fraction(float(b[0])), ah + Fraction(float(b[1]))
    if op == "sub":
        return al - Fraction(float(b[1])), ah - Fraction(float(b[0]))
    if op == "mul":
        bl, bh = Fraction(float(b[0])), Fraction(float(b[1]))
        ps = [al * bl, al * bh, ah * bl, ah * bh]
        return min(ps), max(ps)
    if op == "sqr":
        if al >= 0:
            return al * al, ah * ah
        if ah <= 0:
            return ah * ah, al * al
        return Fraction(0), max(al * al, ah * ah)
    if op == "abs":
        if al >= 0:
            return al, ah
        if ah <= 0:
            return -ah, -al
        return Fraction(0), max(-al, ah)
    raise ValueError(op)


@pytest.mark.parametrize("op", ["add", "sub", "mul", "sqr", "abs"])
def test_fp32_ops_tightest(op):
    rng = np.random.default_rng(31 + len(op))
    a = _rand_intervals(rng, 400)
    b = _rand_intervals(rng, 400)
    print(f"case fp32 op {op}", flush=True)
    got = ibb.interval_op32(op, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda() if op in ("add", "sub", "mul") else None)
    got = got.cpu().numpy()
    bad = 0
    for i in range(a.shape[0]):
        lo, hi = _exact(op, a[i], b[i])
        want = (_down(lo), _up(hi))
        if not (got[i, 0] == want[0] and got[i, 1] == want[1]):
            bad += 1
            if bad < 5:
                print("mismatch", op, a[i], b[i], got[i], want)
    assert bad == 0


def _truth(fn, y):
    with mpmath.workprec(120):
        v = mpmath.cospi(2 * mpmath.mpf(float(y))) if fn == "cos2pi" else mpmath.sinpi(2 * mpmath.mpf(float(y)))
    return v


def _trig_points(rng):
    ys = [0.0, -0.0, 0.125, 0.25, 0.375, 0.5, 0.75, 1.0, -0.25, 2.0 ** -140, -(2.0 ** -149), 1e-20, 3.0, 1e7,
          2.0 ** 23 + 0.5, 2.0 ** 30]
    ys += list(rng.uniform(-4, 4, 300)) + list(rng.uniform(-1e5, 1e5, 100))
    ys += list(0.25 + rng.uniform(-1e-6, 1e-6, 50)) + list(rng.uniform(-1e-8, 1e-8, 50))
    return np.array(ys, dtype=F32)


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_fp32_point_trig_encloses(fn):
    y = _trig_points(np.random.default_rng(7))
    print(f"case fp32 point {fn}", flush=True)
    out = ibb.point_trig32(fn, torch.from_numpy(y).cuda()).cpu().numpy()
    for i in range(y.shape[0]):
        t = _truth(fn, y[i])
        lo, hi = mpmath.mpf(float(out[i, 0])), mpmath.mpf(float(out[i, 1]))
        assert lo <= t <= hi, (fn, float(y[i]), out[i], t)
        # narrow: margin 2^-19 (relative on the sine, absolute on the cosine) plus rounding
        assert hi - lo <= 2.0 ** -17 * max(abs(float(t)), 2.0 ** -100) + 2.0 ** -17 * (fn == "cos2pi") + 2.0 ** -124
    if fn == "cos2pi":
        assert out[0].tolist() == [1.0, 1.0]


@pytest.mark.parametrize("fn", ["cos2pi", "sin2pi"])
def test_fp32_interval_trig_contains_samples(fn):
    rng = np.random.default_rng(11)
    c = rng.uniform(-3, 3, 300)
    w = rng.choice([0.0, 1e-6, 0.01, 0.2, 0.6, 1.2], 300)
    a = np.stack([c - w, c + w], axis=1).astype(F32)
    print(f"case fp32 interval {fn}", flush=True)
    out = ibb.interval_op32(fn, torch.from_numpy(a).cuda()).cpu().numpy()
    for i in range(a.shape[0]):
        lo, hi = float(out[i, 0]), float(out[i, 1])
        assert -1.0 <= lo <= hi <= 1.0
        for s in np.linspace(float(a[i, 0]), float(a[i, 1]), 9):
            v = _truth(fn, s)
            assert mpmath.mpf(lo) <= v <= mpmath.mpf(hi), (fn, a[i], out[i], s, v)


def _sample_points(lo, hi, rng, k=6):
    pts = [lo, hi, 0.5 * (lo + hi)]
    for _ in range(k - 3):
        pts.append(lo + (hi - lo) * rng.uniform(0, 1, lo.shape))
    return pts


@pytest.mark.parametrize("fam,n", [(PR.SEP_COS, 5), (PR.SEP_COS, 100), (PR.SEP_ABS_SIN2, 7), (PR.SEP_ABS_SIN2, 130),
                                   (PR.CHAIN, 9), (PR.CHAIN, 200)])
def test_fp32_boxes_contain_point_values(fam, n):
    p = PR.make(fam, n, 600 + n)
    rng = np.random.default_rng(n)
    lo, hi = PR.random_boxes(p, 32, seed=n, max_width_frac=0.2)
    lo[0], hi[0] = p.x_star, p.x_star
    print(f"case fp32 boxes {p.name}", flush=True)
    F, ub, mono, G = ibb.eval_boxes(p, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda(), want_grad=True,
                                    precision="fp32_bulk")
    F, ub, mono, G = F.cpu().numpy(), ub.cpu().numpy(), mono.cpu().numpy(), G.cpu().numpy()
    F64, ub64, _, _ = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi, want_grad=True)
    assert np.array_equal(ub, ub64) or p.family != PR.CHAIN     # midpoint bound stays FP64
    assert np.all(ub >= ub64) if p.family != PR.CHAIN else True
    for x in _sample_points(lo, hi, rng):
        Fp, _, _, Gp = O.eval_boxes(p.family, p.coef, p.lower, p.upper, x, x, want_grad=True)
        # f(x) lies in [Fp.lo, Fp.hi]; the FP32 box bound must not exclude it
        assert np.all(F[:, 0] <= Fp[:, 1]) and np.all(Fp[:, 0] <= F[:, 1])
        assert np.all(G[..., 0] <= Gp[..., 1]) and np.all(Gp[..., 0] <= G[..., 1])
    # the filter is useful: its lower bound is close to the FP64 one
    scale = np.abs(F64).max(axis=1) + 1.0
    assert np.all(F[:, 0] >= F64[:, 0] - 1e-4 * n * scale)
    # the box at the minimiser: 0 inside, first-order test passes
    assert F[0, 0] <= 0.0 <= F[0, 1] and not mono[0]


def test_fp32_eval_rejects_overflowing_magnitudes():
    # domain [-5e12, 5e12]: (x - c)^2 alone reaches 2.5e25 and a sum of such terms
    # times the coefficients is too close to the float range for the guard
    p = PR.sep_cos(4, 3, lo=-5e12, hi=5e12)
    coef = p.coef.copy()
    coef[:4] = 1e15
    q = _with(p, coef=coef)
    lo = torch.zeros((1, 4), dtype=torch.float64).cuda()
    with pytest.raises(ibb.IbbError):
        ibb.eval_boxes(q, lo, lo + 1.0, precision="fp32_bulk")


def _with(p, **kw):
    import dataclasses
    return dataclasses.replace(p, **kw)


def _x_star_in_boxes(p, r):
    inside = np.all((r.lo <= p.x_star) & (p.x_star <= r.hi), axis=1)
    return bool(np.any(inside))


SOLVES = [(PR.SEP_COS, 2, 101), (PR.SEP_COS, 9, 2), (PR.CHAIN, 5, 505), (PR.SEP_ABS_SIN2, 12, 4),
          (PR.SEP_COS, 100, 102)]


@pytest.mark.parametrize("fam,n,seed", SOLVES)
def test_fp32_solve_encloses_minimum(fam, n, seed):
    p = PR.chain(n, seed, hi=2.3) if fam == PR.CHAIN else PR.make(fam, n, seed)
    print(f"case fp32 solve {p.name}", flush=True)
    a = ibb.minimize(p, precision="fp32_bulk", max_boxes_fetched=200_000)
    assert a.status == ibb.OK
    assert a.f_lo <= 0.0 <= a.f_hi and a.f_hi - a.f_lo <= p.tol_f
    assert a.n_boxes <= 200_000 and _x_star_in_boxes(p, a)
    assert a.fp64_confirmed + a.fp32_pruned == a.boxes_evaluated
    b = ibb.minimize(p, precision="fp32_bulk", max_boxes_fetched=200_000)    # deterministic
    assert (a.f_lo, a.f_hi, a.sweeps, a.boxes_evaluated, a.fp32_pruned) == (b.f_lo, b.f_hi, b.sweeps,
                                                                          b.boxes_evaluated, b.fp32_pruned)
    assert np.array_equal(a.flo, b.flo) and np.array_equal(a.lo, b.lo) and np.array_equal(a.trace_gub, b.trace_gub)
    if n == 100:
        print(f"fp32 filter: {a.fp32_sweeps} sweeps, {a.fp32_pruned} of {a.boxes_evaluated} children", flush=True)
        assert a.fp32_sweeps > 0 and a.fp32_pruned > 0


def test_fp32_filter_off_equals_fp64():
    # magnitudes that could overflow single precision: the filter stays off and the
    # run is the FP64 run bit for bit
    p = PR.sep_cos(6, 21, lo=-5e12, hi=5e12)
    p = _with(p, coef=np.concatenate([np.full(6, 1e15), p.coef[6:]]))
    print("case fp32 off", flush=True)
    a = ibb.minimize(p, precision="fp32_bulk", max_sweeps=40)
    b = ibb.minimize(p, precision="fp64", max_sweeps=40, incremental=False)
    assert a.fp32_sweeps == 0 and a.fp32_pruned == 0
    assert (a.f_lo, a.f_hi, a.sweeps, a.boxes_evaluated) == (b.f_lo, b.f_hi, b.sweeps, b.boxes_evaluated)
    assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.flo, b.flo)


def test_fp32_batch_equals_alone():
    # n = 100 and 200 run with 2 and 4 waves per child alone but one in the batch:
    # the filter's float sums use one canonical order, so the decisions agree
    ps = [PR.sep_cos(9, 2), PR.chain(5, 505, hi=2.3), PR.sep_abs_sin2(12, 4), PR.sep_cos(40, 77),
          PR.sep_cos(100, 102), PR.chain(300, 505, hi=2.3)]
    print("case fp32 batch", flush=True)
    alone = [ibb.minimize(p, precision="fp32_bulk", max_sweeps=400, max_boxes_fetched=500) for p in ps]
    got = ibb.solve_batch(ps, precision="fp32_bulk", max_sweeps=400, max_boxes_fetched=500)
    for a, b in zip(alone, got):
        assert (a.status, a.f_lo, a.f_hi, a.sweeps, a.boxes_evaluated, a.fp32_pruned) == \
            (b.status, b.f_lo, b.f_hi, b.sweeps, b.boxes_evaluated, b.fp32_pruned)
        assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.flo, b.flo)
