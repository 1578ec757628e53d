"""The generic family (expression tapes: the benchmark functions of the paper's
SI Appendix A, Eqs. S1-S21, and Appendix D, Eq. S22) on the GPU, through the C
ABI, against the oracle.

  * Box bounds (ibb_eval_boxes): the GPU's exp, cos and sin enclosures hold the
    oracle's and the tape's operations and their order are the same, so by
    inclusion isotonicity the GPU's F and G hold the oracle's and its midpoint
    bound is at least the oracle's; the GPU discards a box by the first-order
    test only where the oracle does.  Rosenbrock uses only +, -, x and squares:
    bit for bit.
  * Whole runs: Rosenbrock identical to the oracle sweep by sweep; the other
    functions with the same sweeps, survivors and selections (GUB to 1e-12).
  * The paper's own experiments (Sec. 4: n = 50, 10 cycled coordinates cut into
    four pieces, 4^10 subregions per iteration, 10 diagonal samples, width
    1e-4): the iteration counts and the single output region of Tables S2-S10
    and Table 2.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR
from paper_2507_01770_amd import tapes as TP

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_schedule_results.txt")
NAMES = list(TP.PAPER_FUNCTIONS)
PAPER = dict(pieces=4, diag_samples=10)


def paper_rows():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.lstrip().startswith("#"):
                fn, n, it, reg, src = line.split()
                rows[(fn, int(n))] = (int(it), int(reg))
    return rows


def boxes(p, nb, seed):
    g = np.random.default_rng(seed)
    W = p.upper - p.lower
    w = W * np.exp(g.uniform(np.log(1e-9), np.log(0.3), (nb, p.n)))
    lo = p.lower + g.uniform(0, 1, (nb, p.n)) * (W - w)
    hi = np.minimum(lo + w, p.upper)
    lo[0], hi[0] = p.x_star, p.x_star
    return lo, hi


@pytest.mark.parametrize("name", NAMES)
def test_box_bounds_hold_the_oracle(name):
    p = TP.PAPER_FUNCTIONS[name](5)
    lo, hi = boxes(p, 96, seed=len(name))
    print(f"case eval {name} n=5", flush=True)
    F, ub, mono, G = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi, want_grad=True)
    gF, gub, gmono, gG = (t.cpu().numpy() for t in ibb.eval_boxes(p, torch.from_numpy(lo).cuda(),
                                                                   torch.from_numpy(hi).cuda(), want_grad=True))
    if name == "rosenbrock":
        assert np.array_equal(gF, F) and np.array_equal(gub, ub) and np.array_equal(gG, G)
        assert np.array_equal(gmono, mono.astype(bool))
        return
    assert np.all(gF[:, 0] <= F[:, 0]) and np.all(F[:, 1] <= gF[:, 1])
    assert np.all(gub >= ub)
    assert np.all(gG[..., 0] <= G[..., 0]) and np.all(G[..., 1] <= gG[..., 1])
    assert not np.any(gmono & ~mono.astype(bool))
    scale = 1.0 + np.abs(F).max(axis=1)
    assert np.all((gF[:, 1] - gF[:, 0]) - (F[:, 1] - F[:, 0]) <= 1e-9 * scale)


@pytest.mark.parametrize("name", NAMES)
def test_runs_follow_the_oracle(name):
    for n, m, sched in ((4, 2, PAPER), (3, 3, {})):
        p = TP.PAPER_FUNCTIONS[name](n)
        tol = dict(tol_f=1e300, tol_x=1e-4) if sched else dict(tol_f=1e-6, tol_x=0.0)
        print(f"case run {name} n={n} m={m} {'paper schedule' if sched else 'bisection'}", flush=True)
        r = ibb.minimize(p, split_dims=m, max_sweeps=5000, **tol, **sched)
        o = O.solve(p.family, p.coef, p.lower, p.upper, split_dims=m, max_sweeps=5000, **tol,
                    pieces=4 if sched else 2, samples=10 if sched else 0)
        assert r.status == o.status == ibb.OK and r.sweeps == o.sweeps
        assert np.array_equal(r.trace_nsurv, o.trace_nsurv) and np.array_equal(r.trace_sel, o.trace_sel)
        assert np.array_equal(r.trace_nlive, o.trace_nlive)
        if name == "rosenbrock":
            assert np.array_equal(r.trace_gub, o.trace_gub) and np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)
        else:
            assert np.allclose(r.trace_gub, o.trace_gub, rtol=1e-12, atol=1e-12)
        assert r.n_boxes == len(o.flo)
        assert r.f_lo <= p.f_star <= r.f_hi


@pytest.mark.parametrize("name", [n for n in NAMES if n != "rosenbrock"])
def test_paper_tables_at_n_50(name):
    # Sec. 4's schedule as the paper ran it: 4^10 subregions per iteration
    it, reg = paper_rows()[(name, 50)]
    p = TP.PAPER_FUNCTIONS[name](50)
    print(f"case paper table {name} n=50: {it} iterations, {reg} region", flush=True)
    r = ibb.minimize(p, split_dims=10, max_sweeps=5000, tol_f=1e300, tol_x=1e-4, max_boxes_fetched=1000, **PAPER)
    print(f"  {r.sweeps} iterations, {r.n_boxes} regions, {r.seconds:.2f} s, [{r.f_lo}, {r.f_hi}]", flush=True)
    assert r.status == ibb.OK and r.sweeps == it and r.n_boxes == reg
    assert np.all(r.hi - r.lo < 1e-4) and np.any(np.all((r.lo <= p.x_star) & (p.x_star <= r.hi), axis=1))
    assert r.f_lo <= p.f_star <= r.f_hi


def test_generic_family_refusals():
    p = TP.ackley(3)
    with pytest.raises(ibb.IbbError, match="select_k"):
        ibb.minimize(p, select_k=4)
    with pytest.raises(ibb.IbbError, match="FP64"):
        ibb.eval_boxes(p, torch.from_numpy(p.lower[None]).cuda(), torch.from_numpy(p.upper[None]).cuda(),
                       precision="fp32_bulk")
    with pytest.raises(ibb.IbbError):
        ibb.solve_batch([p])
    bad = TP.ackley(3)
    bad.coef = bad.coef.copy()
    bad.coef[0] = 2.0
    with pytest.raises(ibb.IbbError, match="tape"):
        ibb.minimize(bad)
