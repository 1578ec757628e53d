"""Incremental sweeps at n >= 1024 terms (more terms than one workgroup has
threads, so every thread walks several): GPU (C ABI) against the oracle, and the
same problems alone, in a batch and in the server's mix."""
import time

import numpy as np
import pytest

import oracle_runs as ORC
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def same(a, b):
    assert a.status == b.status and a.sweeps == b.sweeps
    assert a.f_lo == b.f_lo and a.f_hi == b.f_hi
    assert a.boxes_evaluated == b.boxes_evaluated and a.n_boxes == b.n_boxes
    assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.trace_nsurv, b.trace_nsurv)
    assert np.array_equal(a.trace_nlive, b.trace_nlive) and np.array_equal(a.trace_sel, b.trace_sel)
    assert np.array_equal(a.flo, b.flo) and np.array_equal(a.seq, b.seq)


CHAIN_LARGE = [(1024, 5), (2500, 3)]
SEP_LARGE = [(PR.SEP_ABS_SIN2, 2000, 4, 4), (PR.SEP_COS, 1500, 9, 4)]
for _n, _budget in CHAIN_LARGE:
    ORC.prefetch(PR.chain(_n, 505, hi=2.3), max_sweeps=_budget, incremental=True)
for _fam, _n, _seed, _budget in SEP_LARGE:
    ORC.prefetch(PR.make(_fam, _n, _seed), max_sweeps=_budget, incremental=True)


@pytest.mark.parametrize("n,budget", CHAIN_LARGE)
def test_chain_large_n_identical_to_oracle(n, budget):
    p = PR.chain(n, 505, hi=2.3)
    print(f"case chain n={n} budget={budget}", flush=True)
    r = ibb.minimize(p, max_sweeps=budget, max_boxes_fetched=200_000)
    o = ORC.solve(p, max_sweeps=budget, incremental=True)
    assert r.status == o.status and r.sweeps == o.sweeps
    assert np.array_equal(r.trace_gub, o.trace_gub)
    assert np.array_equal(r.trace_nsurv, o.trace_nsurv)
    assert np.array_equal(r.trace_nlive, o.trace_nlive)
    assert np.array_equal(r.trace_sel, o.trace_sel)
    assert r.f_lo == o.f_lo and r.f_hi == o.f_hi
    assert np.array_equal(r.seq, o.seq) and np.array_equal(r.flo, o.flo)
    assert np.array_equal(r.lo, o.lo) and np.array_equal(r.hi, o.hi)


@pytest.mark.parametrize("fam,n,seed,budget", SEP_LARGE)
def test_separable_large_n_matches_oracle(fam, n, seed, budget):
    p = PR.make(fam, n, seed)
    print(f"case {p.name} budget={budget}", flush=True)
    r = ibb.minimize(p, max_sweeps=budget, fetch_boxes=False)
    o = ORC.solve(p, max_sweeps=budget, incremental=True)
    assert r.sweeps == o.sweeps == budget
    assert np.allclose(r.trace_gub, o.trace_gub, rtol=1e-12, atol=1e-12)
    assert np.array_equal(r.trace_sel, o.trace_sel)
    assert r.f_lo <= 0.0 <= r.f_hi


def test_large_n_alone_batch_and_server():
    # alone: ibb_solve with the term cache; in the batch and the server: the same
    # iteration without it (each term evaluated from the box)
    big = [PR.chain(1100, 505, hi=2.3), PR.sep_abs_sin2(1500, 7)]
    budget = dict(max_sweeps=60)
    alone = []
    for p in big:
        print(f"case alone {p.name}", flush=True)
        alone.append(ibb.minimize(p, fetch_boxes=False, **budget))
    print("case batch of both", flush=True)
    got = ibb.solve_batch(big, fetch_boxes=False, **budget)   # persistent batched kernel
    for a, b in zip(alone, got):
        same(a, b)
    # next to a problem with full bounds the server runs the per-sweep batched
    # selection kernel for the incremental ones
    with ibb.Server(mem_budget_bytes=4 << 30, max_slots=4) as srv:
        print("case server mix", flush=True)
        tickets = [srv.submit(PR.sep_cos(20, 7), max_sweeps=60, incremental=False)]
        tickets += [srv.submit(p, **budget) for p in big]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in res:
                    r = srv.poll(t, fetch_boxes=False)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
    assert len(res) == len(tickets)
    for t, a in zip(tickets[1:], alone):
        same(a, res[t])


def test_term_cache_at_n_10000_whole_solve():
    # the non-smooth n = 10,000 workload to its enclosure: ibb_solve (term cache;
    # from n = 5120 on each sweep runs on several workgroups: the selection, the
    # row and base terms over blocks of coordinates, the slot sums, then the
    # children in one workgroup) and the batched engine (no cache, one workgroup
    # per sweep) run the same iteration bit for bit
    p = PR.config(3)
    budget = dict(max_sweeps=40000)
    print("case n=10000 alone (term cache)", flush=True)
    a = ibb.minimize(p, fetch_boxes=False, **budget)
    print(f"{a.sweeps} sweeps, largest live list {a.trace_nlive.max()}", flush=True)
    print("case n=10000 batch (no cache)", flush=True)
    b = ibb.solve_batch([p], fetch_boxes=False, **budget)[0]
    same(a, b)
    assert a.status == ibb.OK and a.f_lo <= 0.0 <= a.f_hi and a.f_hi - a.f_lo <= 1e-6


@pytest.mark.parametrize("make,sweeps", [(lambda: PR.chain(8300, 505, hi=2.3), 2000),
                                         (lambda: PR.sep_cos(5200, 9), 3000)],
                         ids=["chain_n8300", "sep_cos_n5200"])
def test_several_workgroup_sweeps_equal_the_batched_engine(make, sweeps):
    # n past 5120 and ragged against the coordinate blocks (256) and the slots
    # (64): the other two families through the several-workgroup sweep
    p = make()
    print(f"case {p.name} alone and batch, {sweeps} sweeps", flush=True)
    a = ibb.minimize(p, fetch_boxes=False, max_sweeps=sweeps)
    b = ibb.solve_batch([p], fetch_boxes=False, max_sweeps=sweeps)[0]
    same(a, b)
