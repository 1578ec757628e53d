"""K > 1 boxes per sweep on the GPU (ibb_solve through the C ABI) against the
oracle's select_k (the K smallest (lower bound, insertion number) per sweep,
children inserted in parent-rank then child-index order).

Chained family: every bound is bit-identical, so the runs must agree sweep for
sweep (GUB, children inserted, live count, rank-0 selection) and end with the
same boxes, in both bound modes.  The cases cover lists shorter than K (the
first sweeps), K = 1024 with four children per box (lists of thousands of keys,
the radix selection's boundary inside a bin, ties in the lower bound broken by
insertion order across many chunks of the list), and windows that wrap.
Separable families: the same path up to last-bit differences of the trig
enclosures.
"""
import numpy as np
import pytest

import oracle_runs as ORC
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402

MODES = [False, True]
# (n, upper bound of the domain, split width, K, sweep budget).  n = 13 on [-2, 2]
# keeps thousands of boxes whose lower bound is exactly 0 (ties broken by
# insertion order over many chunks); n = 16 with K = 1024 has lists of up to
# 54,000 keys (the radix selection's boundary inside a bin)
CHAIN_K = [(7, 2.3, 3, 2, 3000), (7, 2.3, 3, 5, 3000), (13, 2.0, 10, 4, 60), (12, 2.3, 10, 32, 40),
           (30, 2.3, 5, 64, 30), (100, 2.3, 10, 8, 6), (16, 2.3, 4, 1024, 30)]
SEP_K = [(PR.SEP_COS, 9, 2, 4, 10), (PR.SEP_ABS_SIN2, 12, 4, 16, 10), (PR.SEP_COS, 20, 7, 32, 5)]

for _inc in MODES:
    for _n, _hi, _m, _k, _budget in CHAIN_K:
        ORC.prefetch(PR.chain(_n, 505, hi=_hi), split_dims=_m, select_k=_k, max_sweeps=_budget, incremental=_inc)
    for _fam, _n, _seed, _k, _m in SEP_K:
        ORC.prefetch(PR.make(_fam, _n, _seed), split_dims=_m, select_k=_k, max_sweeps=20000, incremental=_inc)


def inside_some_box(x, lo, hi):
    return bool(np.any(np.all((lo <= x) & (x <= hi), axis=1)))


@pytest.mark.parametrize("n,hi,m,k,budget", CHAIN_K)
@pytest.mark.parametrize("incremental", MODES)
def test_chain_select_k_identical_iteration(n, hi, m, k, budget, incremental):
    p = PR.chain(n, 505, hi=hi)
    print(f"case chain n={n} m={m} K={k} budget={budget} incremental={incremental}", flush=True)
    r = ibb.minimize(p, split_dims=m, select_k=k, max_sweeps=budget, incremental=incremental,
                     max_boxes_fetched=400_000)
    o = ORC.solve(p, split_dims=m, select_k=k, max_sweeps=budget, incremental=incremental)
    assert r.status == o.status and r.sweeps == o.sweeps and r.boxes_evaluated == o.boxes_evaluated
    assert np.array_equal(r.trace_gub, o.trace_gub)
    assert np.array_equal(r.trace_nsurv, o.trace_nsurv)
    assert np.array_equal(r.trace_nlive, o.trace_nlive)
    assert np.array_equal(r.trace_sel, o.trace_sel)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
    assert r.n_boxes == len(o.flo)
    assert np.array_equal(r.seq, o.seq) and np.array_equal(r.flo, o.flo)
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)


@pytest.mark.parametrize("fam,n,seed,k,m", SEP_K)
@pytest.mark.parametrize("incremental", MODES)
def test_separable_select_k_matches_oracle(fam, n, seed, k, m, incremental):
    p = PR.make(fam, n, seed)
    print(f"case {p.name} m={m} K={k} incremental={incremental}", flush=True)
    r = ibb.minimize(p, split_dims=m, select_k=k, max_sweeps=20000, incremental=incremental)
    o = ORC.solve(p, split_dims=m, select_k=k, max_sweeps=20000, incremental=incremental)
    assert r.status == ibb.OK and o.status == 0
    for res in (r, o):
        assert res.f_lo <= 0.0 <= res.f_hi and res.f_hi - res.f_lo <= 1e-6
        assert inside_some_box(p.x_star, res.lo, res.hi)
    assert abs(r.sweeps - o.sweeps) <= max(2, o.sweeps // 20)
    q = min(len(r.trace_gub), len(o.trace_gub), 10)
    assert np.allclose(r.trace_gub[:q], o.trace_gub[:q], rtol=1e-12, atol=1e-12)
    assert np.array_equal(r.trace_sel[:3], o.trace_sel[:3])


@pytest.mark.parametrize("incremental", MODES)
def test_select_k_continues_the_same_run(incremental):
    # budget a, then ibb_sweep in pieces == one run with the summed budget
    p = PR.chain(12, 505, hi=2.3)
    print(f"case ibb_sweep K=8 incremental={incremental}", flush=True)
    whole = ibb.minimize(p, select_k=8, max_sweeps=23, fetch_boxes=False, incremental=incremental)
    with ibb.Run(p, select_k=8, max_sweeps=3, incremental=incremental) as run:
        for _ in range(4):
            run.sweep(5)
        got = run.result(fetch_boxes=False)
    assert (got.status, got.sweeps, got.f_lo, got.f_hi, got.n_boxes) == \
        (whole.status, whole.sweeps, whole.f_lo, whole.f_hi, whole.n_boxes)
    assert np.array_equal(got.trace_gub, whole.trace_gub) and np.array_equal(got.flo, whole.flo)
    assert np.array_equal(got.seq, whole.seq)


def test_select_k_every_bound_shape_and_fp32_filter():
    # the bound kernel's shapes give the same K > 1 run; the FP32 filter keeps the
    # enclosure rigorous
    p = PR.sep_cos(100, 102)
    runs = [ibb.minimize(p, select_k=16, max_sweeps=40, bound_shape=s, fetch_boxes=False) for s in (0, 1, 2, 3)]
    for r in runs[1:]:
        assert (r.sweeps, r.f_lo, r.f_hi, r.n_boxes) == (runs[0].sweeps, runs[0].f_lo, runs[0].f_hi, runs[0].n_boxes)
        assert np.array_equal(r.trace_gub, runs[0].trace_gub) and np.array_equal(r.flo, runs[0].flo)
    f32 = ibb.minimize(p, select_k=16, precision="fp32_bulk", max_sweeps=20000)
    assert f32.status == ibb.OK and f32.f_lo <= 0.0 <= f32.f_hi and f32.f_hi - f32.f_lo <= 1e-6
    assert inside_some_box(p.x_star, f32.lo, f32.hi)
