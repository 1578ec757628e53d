"""Batched solves and the continuous-batching server (C ABI) on the GPU.

Each problem keeps its own list and GUB and follows exactly the iteration that
ibb_solve runs for it alone, so every result must be the same bit for bit alone,
in a batch, and in the server's mix (whatever else was admitted next to it and
whenever it arrived).
"""
import time

import numpy as np
import pytest

from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def mix():
    return [PR.sep_cos(2, 101), PR.sep_cos(9, 2), PR.chain(5, 505, hi=2.3), PR.sep_abs_sin2(12, 4),
            PR.chain(13, 505), PR.sep_cos(100, 102), PR.sep_abs_sin2(130, 7), PR.chain(70, 505),
            PR.chain(200, 505, hi=2.3)]


BUDGET = dict(max_sweeps=400)


def same(a, b):
    assert a.status == b.status and a.sweeps == b.sweeps
    assert a.f_lo == b.f_lo and a.f_hi == b.f_hi
    assert a.boxes_evaluated == b.boxes_evaluated and a.n_boxes == b.n_boxes
    assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.trace_nsurv, b.trace_nsurv)
    assert np.array_equal(a.trace_nlive, b.trace_nlive) and np.array_equal(a.trace_sel, b.trace_sel)
    assert np.array_equal(a.flo, b.flo) and np.array_equal(a.seq, b.seq)
    if a.lo is not None and b.lo is not None:
        assert np.array_equal(a.lo, b.lo) and np.array_equal(a.hi, b.hi)


@pytest.fixture(scope="module")
def alone():
    out = []
    for p in mix():
        print(f"case alone {p.name}", flush=True)
        out.append(ibb.minimize(p, max_boxes_fetched=500, **BUDGET))
    return out


def test_batch_equals_alone(alone):
    print("case batch of all", flush=True)
    got = ibb.solve_batch(mix(), max_boxes_fetched=500, **BUDGET)
    for a, b in zip(alone, got):
        same(a, b)


def test_batch_subsets_equal_alone(alone):
    ps = mix()
    for idx in ([0], [8, 1], [5, 6, 2]):
        print(f"case batch subset {idx}", flush=True)
        got = ibb.solve_batch([ps[i] for i in idx], max_boxes_fetched=500, **BUDGET)
        for i, b in zip(idx, got):
            same(alone[i], b)


def test_server_mix_equals_alone(alone):
    ps = mix()
    with ibb.Server(mem_budget_bytes=4 << 30, max_slots=4) as srv:
        tickets = []
        for p in ps:                      # staggered arrivals while others run
            print(f"case server submit {p.name}", flush=True)
            tickets.append(srv.submit(p, **BUDGET))
            time.sleep(0.002)
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in res:
                    r = srv.poll(t, fetch_boxes=True, max_boxes_fetched=500)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
        st = srv.stats()
    assert len(res) == len(tickets)
    for t, a in zip(tickets, alone):
        same(a, res[t])
    assert st["completed"] == len(ps) and 2 <= st["max_active"] <= 4


def test_server_respects_memory_budget():
    ps = [PR.sep_cos(100, 11 + i) for i in range(6)]
    # about 1.4 MB each at the start (a 1 MiB slab and the arrays larger than its
    # pieces): a 4 MiB budget admits at most three at once
    with ibb.Server(mem_budget_bytes=4 << 20, max_slots=8) as srv:
        pending = {srv.submit(p, max_sweeps=300) for p in ps}
        t0 = time.time()
        while pending and time.time() - t0 < 120:
            for t in list(pending):
                if srv.poll(t) is not None:
                    pending.discard(t)
            time.sleep(0.002)
        st = srv.stats()
    assert not pending and st["completed"] == len(ps)
    assert st["max_active"] <= 3


@pytest.mark.parametrize("incremental", [True, False])
def test_long_lists_batch_and_server_equal_alone(incremental):
    # lists past 2^18 keys are scanned on several workgroups per problem before
    # each selection, in the batched kernels as in ibb_solve
    ps = [PR.chain(64, 41), PR.chain(100, 42), PR.sep_cos(30, 43)]
    kw = dict(max_sweeps=400, incremental=incremental)
    print(f"case long lists alone incremental={incremental}", flush=True)
    alone = [ibb.minimize(p, max_boxes_fetched=500, **kw) for p in ps]
    assert max(int(a.trace_nlive.max()) for a in alone) > (1 << 18)
    print("case long lists batch", flush=True)
    for a, b in zip(alone, ibb.solve_batch(ps, max_boxes_fetched=500, **kw)):
        same(a, b)
    print("case long lists server", flush=True)
    with ibb.Server(mem_budget_bytes=8 << 30, max_slots=4) as srv:
        tickets = [srv.submit(p, **kw) for p in ps]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in res:
                    r = srv.poll(t, fetch_boxes=True, max_boxes_fetched=500)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
    assert len(res) == len(tickets)
    for t, a in zip(tickets, alone):
        same(a, res[t])


def test_server_ends_a_problem_at_the_memory_budget():
    # a problem whose list would have to grow past the budget ends at its next sweep,
    # not converged, with exactly the list, GUB and trace that ibb_solve reaches with
    # that many sweeps as its budget; a small problem in the same server goes on
    big, small = PR.sep_cos(100, 31), PR.sep_cos(2, 32)
    print("case server memory stop", flush=True)
    with ibb.Server(mem_budget_bytes=3 << 20, max_slots=4) as srv:
        tickets = [srv.submit(big), srv.submit(small)]
        res = {}
        t0 = time.time()
        while len(res) < 2 and time.time() - t0 < 120:
            for t in tickets:
                if t not in res:
                    r = srv.poll(t, fetch_boxes=True, max_boxes_fetched=500)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
    assert len(res) == 2
    rb, rs = res[tickets[0]], res[tickets[1]]
    assert rb.status == ibb.NOT_CONVERGED and rb.stop_reason == 8 and 0 <= rb.sweeps < 150
    assert rb.f_lo <= 0.0 <= rb.f_hi   # the family's minimum
    ref = ibb.minimize(big, max_sweeps=rb.sweeps, max_boxes_fetched=500)
    assert ref.stop_reason == 2
    same(ref, rb)
    assert rs.status == ibb.OK and rs.stop_reason == 1
    same(ibb.minimize(small, max_boxes_fetched=500), rs)


def test_server_rejects_invalid():
    with ibb.Server(mem_budget_bytes=1 << 30, max_slots=2) as srv:
        p = PR.sep_cos(3, 1)
        p.lower = p.lower.copy()
        p.lower[0] = p.upper[0]
        with pytest.raises(ibb.IbbError):
            srv.submit(p)
        with pytest.raises(ibb.IbbError):
            srv.poll(12345)


def test_server_on_the_null_stream(alone):
    # the legacy null stream cannot be captured: the engine then runs on a stream of its own
    ps = mix()[:3]
    with ibb.Server(mem_budget_bytes=1 << 30, max_slots=2, stream=torch.cuda.default_stream()) as srv:
        tickets = [srv.submit(p, **BUDGET) for p in ps]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 120:
            for t in tickets:
                if t not in res:
                    r = srv.poll(t, fetch_boxes=True, max_boxes_fetched=500)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
    assert len(res) == len(tickets)
    for t, a in zip(tickets, alone[:3]):
        same(a, res[t])


def test_batch_full_bounds_equals_alone():
    # children bounded over all n terms by the batched bound kernel (one wavefront each);
    # the solves alone run one after another in this process, so later ones get
    # recycled device memory from the caching allocator
    ps = mix()
    print("case batch full bounds", flush=True)
    alone = []
    for p in ps:
        print(f"case alone full bounds {p.name}", flush=True)
        alone.append(ibb.minimize(p, max_boxes_fetched=500, incremental=False, **BUDGET))
    got = ibb.solve_batch(ps, max_boxes_fetched=500, incremental=False, **BUDGET)
    for a, b in zip(alone, got):
        same(a, b)


def test_server_results_freed_while_it_runs():
    # the caller receives and frees results while the server thread keeps capturing
    # and replaying graphs of the remaining problems: frees must never land on the
    # stream being captured (regression test)
    reqs = PR.serving_trace(count=48, seed=105, rate=1.0)
    ps = [q for _, q in reqs]
    picks = [0, 7, 19, 31, 47]
    ref = {i: ibb.minimize(ps[i], max_sweeps=200, fetch_boxes=False) for i in picks}
    with ibb.Server(mem_budget_bytes=1 << 30, max_slots=8) as srv:
        tickets = []
        got = {}
        t0 = time.time()
        for i, q in enumerate(ps):
            tickets.append(srv.submit(q, max_sweeps=200))
            for j, t in enumerate(tickets):         # poll (and so free) while submitting
                if j not in got:
                    r = srv.poll(t)
                    if r is not None:
                        got[j] = r
        while len(got) < len(ps) and time.time() - t0 < 150:
            for j, t in enumerate(tickets):
                if j not in got:
                    r = srv.poll(t)
                    if r is not None:
                        got[j] = r
            time.sleep(0.0005)
        st = srv.stats()
    assert len(got) == len(ps) and st["completed"] == len(ps)
    for i in picks:
        a, b = ref[i], got[i]
        assert (a.status, a.f_lo, a.f_hi, a.sweeps, a.boxes_evaluated) == (b.status, b.f_lo, b.f_hi, b.sweeps,
                                                                             b.boxes_evaluated)
        assert np.array_equal(a.trace_gub, b.trace_gub) and np.array_equal(a.flo, b.flo)


def degenerate_mix():
    root_done = PR.chain(4, 505, hi=2.3)
    root_done.tol_f = 1e6                      # the root meets the tolerance: no sweep
    ulp = PR.chain(6, 505, hi=2.3)             # two coordinates one ulp wide: never split
    ulp.lower[2], ulp.upper[2] = 1.0, np.nextafter(1.0, 2.0)
    ulp.lower[4], ulp.upper[4] = 0.5, np.nextafter(0.5, 1.0)
    face = PR.chain(6, 505, lo=1.0, hi=2.3)    # minimiser on a face of the domain
    return [root_done, ulp, face, PR.sep_cos(9, 2)]


@pytest.mark.parametrize("incremental", [False, True])
def test_batch_with_degenerate_members_equals_alone(incremental):
    ps = degenerate_mix()
    alone = []
    for p in ps:
        print(f"case alone {p.name} incremental={incremental}", flush=True)
        alone.append(ibb.minimize(p, max_boxes_fetched=500, incremental=incremental, **BUDGET))
    assert alone[0].sweeps == 0 and alone[0].n_boxes == 1
    print(f"case batch of degenerate members incremental={incremental}", flush=True)
    got = ibb.solve_batch(ps, max_boxes_fetched=500, incremental=incremental, **BUDGET)
    for a, b in zip(alone, got):
        same(a, b)
