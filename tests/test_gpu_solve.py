"""Whole iterations on the GPU (ibb_solve through the C ABI) against the oracle.

CHAIN: every bound is bit-identical, so the two iterations must agree sweep for
sweep (GUB after each sweep, children inserted, live count, selected box) and
end with the same boxes.  Separable families: the GPU's trig enclosures may be
a couple of doubles wider, so decisions can differ in rare ties; both runs must
enclose the known minimum 0 at the stated width and keep the minimiser, and
their traces must agree closely.  The workload sizes run on the GPU in full and
are compared with a prefix of the oracle's iteration.
"""
import numpy as np
import pytest

import oracle_runs as ORC
from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def inside_some_box(x, lo, hi):
    return bool(np.any(np.all((lo <= x) & (x <= hi), axis=1)))


def run_both(p, incremental, **kw):
    """The same iteration on the GPU and in the oracle, with full or incremental child bounds."""
    print(f"case {p.name} incremental={incremental} {kw}", flush=True)
    r = ibb.minimize(p, incremental=incremental, **kw)
    o = ORC.solve(p, max_sweeps=kw.get("max_sweeps", 100000), incremental=incremental)
    return r, o


MODES = [False, True]


# [-2, 2.3] keeps x* = 1 off the bisection points, so the runs take 40-50 sweeps;
# n = 13 on [-2, 2] does not converge quickly and stops on the sweep budget.
# n = 70 and 100 use two wavefronts per child, n = 200 four.
# n = 13 runs 300 sweeps: the row arrays grow past 256 rows on the way.
CHAIN_CASES = [(2, 2.0, 3000), (3, 2.3, 3000), (5, 2.3, 3000), (8, 2.3, 3000), (12, 2.3, 3000), (13, 2.0, 300),
               (70, 2.0, 3000), (100, 2.3, 30), (200, 2.3, 20)]
WORKLOAD_PREFIX = [(1, 6), (2, 12)]
# the slow oracle runs start on host threads as soon as this module is imported
for _inc in MODES:
    for _cfg, _prefix in WORKLOAD_PREFIX:
        ORC.prefetch(PR.config(_cfg), max_sweeps=_prefix, incremental=_inc)
    for _n, _hi, _budget in CHAIN_CASES:
        if _n >= 12:
            ORC.prefetch(PR.chain(_n, 505, hi=_hi), max_sweeps=_budget, incremental=_inc)


@pytest.mark.parametrize("n,hi,budget", CHAIN_CASES)
@pytest.mark.parametrize("incremental", MODES)
def test_chain_identical_iteration(n, hi, budget, incremental):
    p = PR.chain(n, 505, hi=hi)
    r, o = run_both(p, incremental, max_sweeps=budget)
    assert r.status == o.status
    assert r.sweeps == o.sweeps
    assert np.array_equal(r.trace_gub, o.trace_gub)
    assert np.array_equal(r.trace_nsurv, o.trace_nsurv)
    assert np.array_equal(r.trace_nlive, o.trace_nlive)
    assert np.array_equal(r.trace_sel, o.trace_sel)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
    assert np.array_equal(r.seq, o.seq) and np.array_equal(r.flo, o.flo)
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
    assert boxes_equal_count(r, o)


def boxes_equal_count(r, o):
    return r.n_boxes == len(o.flo)


@pytest.mark.parametrize("fam,n,seed", [(PR.SEP_COS, 1, 1), (PR.SEP_COS, 2, 101), (PR.SEP_COS, 9, 2),
                                        (PR.SEP_ABS_SIN2, 2, 3), (PR.SEP_ABS_SIN2, 12, 4)])
@pytest.mark.parametrize("incremental", MODES)
def test_separable_matches_oracle(fam, n, seed, incremental):
    p = PR.make(fam, n, seed)
    r, o = run_both(p, incremental, max_sweeps=20000)
    assert r.status == ibb.OK and o.status == O.ST_OK
    for res in (r, o):
        assert res.f_lo <= 0.0 <= res.f_hi and res.f_hi - res.f_lo <= 1e-6
        assert inside_some_box(p.x_star, res.lo, res.hi)
    # same path up to last-bit differences of the bounds
    assert abs(r.sweeps - o.sweeps) <= max(2, o.sweeps // 20)
    k = min(len(r.trace_gub), len(o.trace_gub), 10)
    assert np.allclose(r.trace_gub[:k], o.trace_gub[:k], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("incremental", MODES)
def test_budget_and_width_criterion(incremental):
    p = PR.sep_cos(6, 9)
    r = ibb.minimize(p, max_sweeps=4, incremental=incremental)
    assert r.status == ibb.NOT_CONVERGED and r.sweeps == 4 and r.stop_reason == 2
    assert r.f_lo <= 0.0 <= r.f_hi and inside_some_box(p.x_star, r.lo, r.hi)
    # a time limit stops on the host between chunks; the last children are still inserted
    r = ibb.minimize(p, time_limit_s=1e-9, incremental=incremental)
    assert r.status == ibb.NOT_CONVERGED and r.sweeps >= 1 and r.stop_reason == 5
    assert r.f_lo <= 0.0 <= r.f_hi and inside_some_box(p.x_star, r.lo, r.hi)
    assert r.trace_nsurv.sum() + 1 - r.sweeps >= r.n_boxes
    p.tol_x = 1e-4
    r = ibb.minimize(p, max_sweeps=20000, incremental=incremental)
    assert r.status == ibb.OK and np.all(r.hi - r.lo < 1e-4) and r.stop_reason == 1


@pytest.mark.parametrize("incremental", MODES)
def test_live_box_limit_identical_to_oracle(incremental):
    # the run stops at the first sweep that leaves more live boxes than the limit
    # (here the sixth), inside the persistent loop, exactly where the oracle stops
    p = PR.chain(12, 505, hi=2.3)
    free = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, tol_x=p.tol_x, max_sweeps=3000,
                   incremental=incremental)
    limit = int(free.trace_nlive[:5].max())
    print(f"case {p.name} live limit {limit} incremental={incremental}", flush=True)
    r = ibb.minimize(p, max_sweeps=3000, max_live_boxes=limit, incremental=incremental)
    o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, tol_x=p.tol_x, max_sweeps=3000,
                max_live_boxes=limit, incremental=incremental)
    assert o.status == O.ST_NOT_CONVERGED and o.sweeps == 6
    assert r.status == ibb.NOT_CONVERGED and r.sweeps == o.sweeps and r.stop_reason == 3
    assert np.array_equal(r.trace_nlive, o.trace_nlive) and np.array_equal(r.trace_gub, o.trace_gub)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
    assert np.array_equal(r.seq, o.seq) and np.array_equal(r.flo, o.flo)
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)

@pytest.mark.parametrize("incremental", MODES)
def test_width_criterion_identical_to_oracle(incremental):
    # with a box-width tolerance the run goes on until every listed box is narrower
    # as well (3 and 9 sweeps past the GUB - GLB criterion here), sweep for sweep as
    # in the oracle
    p = PR.chain(5, 505, hi=2.3)
    for tol_x in (1e-3, 1e-4):
        p.tol_x = tol_x
        r, o = run_both(p, incremental, max_sweeps=100000)
        assert o.status == O.ST_OK and r.status == ibb.OK and r.sweeps == o.sweeps
        assert np.array_equal(r.trace_gub, o.trace_gub) and np.array_equal(r.trace_nlive, o.trace_nlive)
        assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
        assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
        assert np.all(r.hi - r.lo < tol_x)

@pytest.mark.parametrize("incremental", MODES)
def test_one_ulp_coordinates_identical_to_oracle(incremental):
    # coordinates one ulp wide are never split (their split point is an endpoint)
    # and the children that would take their upper halves are not formed
    p = PR.chain(6, 505, hi=2.3)
    p.lower[2], p.upper[2] = 1.0, np.nextafter(1.0, 2.0)
    p.lower[4], p.upper[4] = 0.5, np.nextafter(0.5, 1.0)
    for m in (3, 6):
        print(f"case {p.name} one-ulp coordinates m={m} incremental={incremental}", flush=True)
        r = ibb.minimize(p, split_dims=m, max_sweeps=3000, incremental=incremental)
        o = O.solve(p.family, p.coef, p.lower, p.upper, tol_f=p.tol_f, split_dims=m, max_sweeps=3000,
                    incremental=incremental)
        assert o.status == O.ST_OK and r.status == ibb.OK and r.sweeps == o.sweeps
        assert r.boxes_evaluated == o.boxes_evaluated
        assert np.array_equal(r.trace_gub, o.trace_gub) and np.array_equal(r.trace_nsurv, o.trace_nsurv)
        assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
        assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
    q = PR.sep_cos(5, 7)
    q.lower[1], q.upper[1] = 0.25, np.nextafter(0.25, 1.0)
    r, o = run_both(q, incremental, max_sweeps=3000)
    assert o.status == O.ST_OK and r.status == ibb.OK
    assert r.f_lo <= o.f_hi and o.f_lo <= r.f_hi
    assert np.all(r.lo[:, 1] == q.lower[1]) and np.all(r.hi[:, 1] == q.upper[1])

@pytest.mark.parametrize("lo,hi,n", [(1.0, 2.3, 6), (-3.0, 1.0, 9)])
@pytest.mark.parametrize("incremental", MODES)
def test_minimiser_on_the_boundary_identical_to_oracle(lo, hi, n, incremental):
    # x* = (1, ..., 1) on a face of the domain: the boxes on that face survive the
    # first-order test, sweep for sweep as in the oracle
    p = PR.chain(n, 505, lo=lo, hi=hi)
    r, o = run_both(p, incremental, max_sweeps=3000)
    assert o.status == O.ST_OK and r.status == ibb.OK and r.sweeps == o.sweeps
    assert np.array_equal(r.trace_gub, o.trace_gub) and np.array_equal(r.trace_nlive, o.trace_nlive)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi and r.f_lo <= 0.0 <= r.f_hi
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
    assert inside_some_box(np.ones(n), r.lo, r.hi)

@pytest.mark.parametrize("incremental", MODES)
def test_zero_sweeps_identical_to_oracle(incremental):
    # a tolerance the root already meets, and a budget of no sweeps: the output is
    # the root box with its own bounds and empty traces
    p = PR.chain(4, 505, hi=2.3)
    for tol_f, budget, status in ((1e6, 100, ibb.OK), (1e-6, 0, ibb.NOT_CONVERGED)):
        p.tol_f = tol_f
        print(f"case {p.name} tol_f={tol_f} max_sweeps={budget} incremental={incremental}", flush=True)
        r, o = run_both(p, incremental, max_sweeps=budget)
        assert r.status == status and o.status == status and r.sweeps == o.sweeps == 0
        assert r.f_lo == o.f_lo and r.f_hi == o.f_hi and r.boxes_evaluated == 1
        assert r.n_boxes == 1 and np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
        assert r.trace_gub.size == 0 and r.trace_nlive.size == 0

@pytest.mark.parametrize("incremental", MODES)
def test_workload0_full_parity(incremental):
    p = PR.config(0)
    r, o = run_both(p, incremental)
    assert r.status == ibb.OK and r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6
    assert r.sweeps == o.sweeps


@pytest.mark.parametrize("cfg,prefix", WORKLOAD_PREFIX)
@pytest.mark.parametrize("incremental", MODES)
def test_workload_full_run_and_prefix(cfg, prefix, incremental):
    p = PR.config(cfg)
    print(f"case workload {cfg} full incremental={incremental}", flush=True)
    r = ibb.minimize(p, max_sweeps=200000, fetch_boxes=True, max_boxes_fetched=2000, incremental=incremental)
    assert r.status == ibb.OK, r.status
    assert r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6
    assert inside_some_box(p.x_star, r.lo, r.hi) or r.n_boxes > 2000
    print(f"case workload {cfg} oracle prefix {prefix}", flush=True)
    o = ORC.solve(p, max_sweeps=prefix, incremental=incremental)
    if p.family == PR.CHAIN:
        assert np.array_equal(r.trace_gub[:prefix], o.trace_gub)
        assert np.array_equal(r.trace_nsurv[:prefix], o.trace_nsurv)
        assert np.array_equal(r.trace_sel[:prefix], o.trace_sel)
    else:
        assert np.allclose(r.trace_gub[:prefix], o.trace_gub, rtol=1e-12)
        assert np.array_equal(r.trace_sel[:prefix], o.trace_sel)


@pytest.mark.parametrize("incremental,budget", [(False, 40), (True, 400)])
def test_workload3_capped_run(incremental, budget):
    # n = 10,000: the oracle needs about 30 s per sweep, so only invariants here
    # (the bounds themselves are compared on sampled boxes in test_gpu_eval)
    p = PR.config(3)
    print(f"case workload 3 capped incremental={incremental}", flush=True)
    r = ibb.minimize(p, max_sweeps=budget, fetch_boxes=False, incremental=incremental)
    assert r.status == ibb.NOT_CONVERGED and r.sweeps == budget
    assert r.f_lo <= 0.0 <= r.f_hi
    assert r.trace_sel[0] == 0 and np.all(np.diff(r.trace_gub) <= 0)


def _same_run(a, b):
    assert (a.status, a.f_lo, a.f_hi, a.sweeps, a.boxes_evaluated, a.n_boxes) == \
        (b.status, b.f_lo, b.f_hi, b.sweeps, b.boxes_evaluated, b.n_boxes)
    assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.trace_nsurv, b.trace_nsurv)
    assert np.array_equal(a.flo, b.flo) and np.array_equal(a.seq, b.seq)


@pytest.mark.parametrize("p,shapes", [(PR.sep_cos(100, 102), [0, 1, 2, 3]), (PR.chain(300, 505, hi=2.3), [0, 1, 2, 3, 4]),
                                      (PR.sep_abs_sin2(40, 9), [0, 2])])
def test_every_bound_shape_gives_the_same_run(p, shapes):
    # the autotuner may pick any shape: all must follow the same iteration bit for bit
    runs = []
    for s in shapes:
        print(f"case shape {s} {p.name}", flush=True)
        r = ibb.minimize(p, max_sweeps=60, bound_shape=s, fetch_boxes=False)
        assert r.bound_shape == s
        runs.append(r)
    auto = ibb.minimize(p, max_sweeps=60, fetch_boxes=False, incremental=False)
    assert auto.bound_shape in shapes
    for r in runs[1:] + [auto]:
        _same_run(runs[0], r)
    # and in FP32 mode (throughput shapes only) the filter's decisions agree too
    f32 = [ibb.minimize(p, max_sweeps=60, bound_shape=s, precision="fp32_bulk", fetch_boxes=False)
           for s in shapes if s >= 2]
    for r in f32[1:]:
        _same_run(f32[0], r)
        assert r.fp32_pruned == f32[0].fp32_pruned


def test_forced_shape_rejected_when_not_admissible():
    with pytest.raises(ibb.IbbError):
        ibb.minimize(PR.sep_cos(100, 102), max_sweeps=5, bound_shape=4)          # 4 waves, 2 tiles
    with pytest.raises(ibb.IbbError):
        ibb.minimize(PR.sep_cos(9, 2), max_sweeps=5, bound_shape=0, precision="fp32_bulk")


@pytest.mark.parametrize("p", [PR.sep_cos(100, 102), PR.chain(70, 505), PR.sep_abs_sin2(12, 4)])
@pytest.mark.parametrize("incremental", MODES)
def test_sweep_continues_the_same_run(p, incremental):
    # budget a, then ibb_sweep in pieces == one run with the summed budget, and a
    # run continued to convergence == the unbudgeted solve
    print(f"case ibb_sweep {p.name} incremental={incremental}", flush=True)
    whole = ibb.minimize(p, max_sweeps=38, fetch_boxes=False, incremental=incremental)   # 3 + 5 x 7
    with ibb.Run(p, max_sweeps=3, incremental=incremental) as r:
        assert r.result(fetch_boxes=False).sweeps == 3
        for _ in range(5):
            r.sweep(7)
        got = r.result(fetch_boxes=False)
        assert r.sweep(0) == got.status             # no sweep: the status as it was
    _same_run(whole, got)
    full = ibb.minimize(p, max_sweeps=5000, fetch_boxes=False, incremental=incremental)
    with ibb.Run(p, max_sweeps=10, incremental=incremental) as r:
        st = r.sweep(5000)
        got = r.result(fetch_boxes=False)
        assert st == full.status == got.status
        assert r.sweep(10) == got.status            # a converged run stays as it is
        again = r.result(fetch_boxes=False)
    _same_run(full, got)
    _same_run(full, again)
