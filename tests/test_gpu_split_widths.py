"""Whole iterations with split widths other than the default 10, on the GPU
(ibb_solve through the C ABI) against the oracle.

Covers the narrow windows (fewer split coordinates than the prefix table's six
positions, a single split coordinate), windows that wrap past coordinate n - 1,
and wide ones (more than 1024 children per sweep, whose bounds are not cached
between the two passes of the incremental sweep), in both bound modes.  Chained
family: bit-identical sweep by sweep; separable cosine family: the same path up
to last-bit differences of the trig enclosures.
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

MODES = [False, True]


CHAIN_WIDTHS = [(20, 1, 400), (20, 3, 300), (13, 5, 200), (30, 7, 100), (14, 11, 30), (12, 12, 16), (24, 16, 2)]
SEP_WIDTHS = [(40, 3, 300), (14, 12, 40)]
for _inc in MODES:
    for _n, _m, _budget in CHAIN_WIDTHS:
        ORC.prefetch(PR.chain(_n, 505, hi=2.3), split_dims=_m, max_sweeps=_budget, incremental=_inc)
    for _n, _m, _budget in SEP_WIDTHS:
        ORC.prefetch(PR.sep_cos(_n, 7), split_dims=_m, max_sweeps=_budget, incremental=_inc)


@pytest.mark.parametrize("n,m,budget", CHAIN_WIDTHS)
@pytest.mark.parametrize("incremental", MODES)
def test_chain_split_width_identical_iteration(n, m, budget, incremental):
    p = PR.chain(n, 505, hi=2.3)
    print(f"case chain n={n} m={m} budget={budget} incremental={incremental}", flush=True)
    r = ibb.minimize(p, split_dims=m, max_sweeps=budget, incremental=incremental, max_boxes_fetched=200_000)
    o = ORC.solve(p, split_dims=m, max_sweeps=budget, incremental=incremental)
    assert r.status == o.status and r.sweeps == o.sweeps and r.boxes_evaluated == o.boxes_evaluated
    assert np.array_equal(r.trace_gub, o.trace_gub)
    assert np.array_equal(r.trace_nsurv, o.trace_nsurv)
    assert np.array_equal(r.trace_nlive, o.trace_nlive)
    assert np.array_equal(r.trace_sel, o.trace_sel)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
    assert r.n_boxes == len(o.flo)
    assert np.array_equal(r.seq, o.seq) and np.array_equal(r.flo, o.flo)
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)


@pytest.mark.parametrize("n,m,budget", SEP_WIDTHS)
@pytest.mark.parametrize("incremental", MODES)
def test_separable_split_width_matches_oracle(n, m, budget, incremental):
    p = PR.sep_cos(n, 7)
    print(f"case sep_cos n={n} m={m} budget={budget} incremental={incremental}", flush=True)
    r = ibb.minimize(p, split_dims=m, max_sweeps=budget, incremental=incremental, fetch_boxes=False)
    o = ORC.solve(p, split_dims=m, max_sweeps=budget, incremental=incremental)
    assert r.status == ibb.OK and o.status == O.ST_OK
    assert r.f_lo <= 0.0 <= r.f_hi and r.f_hi - r.f_lo <= 1e-6
    assert abs(r.sweeps - o.sweeps) <= max(2, o.sweeps // 20)
    k = min(len(r.trace_gub), len(o.trace_gub), 10)
    assert np.allclose(r.trace_gub[:k], o.trace_gub[:k], rtol=1e-12, atol=1e-12)
    assert np.array_equal(r.trace_sel[:3], o.trace_sel[:3])


def test_trace_past_its_first_block():
    # more sweeps than the first trace block holds (4096): the block is grown on
    # the way, and the run is the same as its first 300 sweeps alone
    p = PR.sep_cos(400, 7)   # one split coordinate per sweep: still running after 5000 sweeps
    print("case trace growth sep_cos n=400 m=1", flush=True)
    long = ibb.minimize(p, split_dims=1, max_sweeps=5000, fetch_boxes=False)
    short = ibb.minimize(p, split_dims=1, max_sweeps=300, fetch_boxes=False)
    assert long.status == ibb.NOT_CONVERGED and long.sweeps == 5000
    assert len(long.trace_gub) == len(long.trace_sel) == len(long.trace_nlive) == 5000
    assert np.array_equal(long.trace_gub[:300], short.trace_gub)
    assert np.array_equal(long.trace_sel[:300], short.trace_sel)
    assert np.array_equal(long.trace_nsurv[:300], short.trace_nsurv)
    assert np.all(np.diff(long.trace_gub) <= 0)
