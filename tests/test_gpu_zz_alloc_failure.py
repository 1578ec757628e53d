"""An allocator that refuses (ibb_allocator.alloc returning NULL) ends a solve with
IBB_E_NOMEM at whichever request it refuses, with every block the library took
given back, and the library keeps working afterwards."""
import ctypes as C

import numpy as np
import pytest

from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402

NOMEM = -2


class CountingAllocator:
    """ibb_allocator over torch's caching allocator that refuses the fail_at-th
    request (1-based) and every one after it; records what is still held."""

    def __init__(self, fail_at=None):
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.bad_frees = 0
        dev = torch.cuda.current_device()

        def _alloc(ctx, nbytes, stream):
            self.calls += 1
            if self.fail_at is not None and self.calls >= self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            self.live[p] = int(nbytes)
            return p

        def _free(ctx, p, nbytes, stream):
            if self.live.pop(p, None) is None:
                self.bad_frees += 1
                return
            torch.cuda.caching_allocator_delete(p)

        self._a = ibb._ALLOC_FN(_alloc)
        self._f = ibb._FREE_FN(_free)
        self.struct = ibb._Allocator(None, self._a, self._f)


def solve_with(alloc, p, incremental):
    L = ibb.lib()
    k = ibb._prob_args(p)
    o = ibb._options(max_sweeps=300, incremental=incremental)
    h = C.c_void_p()
    rc = L.ibb_solve(C.byref(k.s), C.byref(o), C.byref(alloc.struct), ibb._stream_ptr(), C.byref(h))
    torch.cuda.synchronize()
    return rc, h


@pytest.mark.parametrize("incremental", [False, True])
def test_refused_allocation_gives_nomem_and_returns_everything(incremental):
    # chained n = 13 on [-2, 2] runs the 300 sweeps, so its row arrays grow on the way
    p = PR.chain(13, 505)
    L = ibb.lib()
    ref = ibb.minimize(p, max_sweeps=300, incremental=incremental, fetch_boxes=False)
    counts = []
    for _ in range(2):   # the second run is the one measured (shape tuning is cached by then)
        a = CountingAllocator()
        rc, h = solve_with(a, p, incremental)
        assert rc == ibb.NOT_CONVERGED and h.value
        L.ibb_result_free(h)
        assert not a.live and a.bad_frees == 0
        counts.append(a.calls)
    total = counts[-1]
    assert total >= 3
    for fail_at in sorted({1, 2, total // 2, total}):
        print(f"case refuse request {fail_at} of {total} incremental={incremental}", flush=True)
        a = CountingAllocator(fail_at)
        rc, h = solve_with(a, p, incremental)
        assert rc == NOMEM and not h.value, (fail_at, rc)
        assert "allocation" in L.ibb_last_error().decode()
        assert not a.live and a.bad_frees == 0, (fail_at, a.live)
    again = ibb.minimize(p, max_sweeps=300, incremental=incremental, fetch_boxes=False)
    assert (again.status, again.sweeps, again.f_lo, again.f_hi) == (ref.status, ref.sweeps, ref.f_lo, ref.f_hi)
    assert np.array_equal(again.trace_gub, ref.trace_gub)


@pytest.mark.parametrize("incremental", [False, True])
def test_refused_allocation_in_a_batch(incremental):
    # a refusal while problems are admitted fails those problems; one while the
    # batch runs (its row or key arrays growing) fails the call, and the results
    # of problems that finished before it are still handed over.  Either way,
    # once the caller frees the results every block has come back.
    ps = [PR.chain(13, 505), PR.sep_cos(9, 2), PR.chain(5, 505, hi=2.3)]
    L = ibb.lib()
    keeps = [ibb._prob_args(p) for p in ps]
    arr = (ibb._Problem * len(keeps))(*[k.s for k in keeps])
    o = ibb._options(max_sweeps=300, incremental=incremental)

    def run(alloc):
        outs = (C.c_void_p * len(ps))()
        sts = (C.c_int32 * len(ps))()
        rc = L.ibb_solve_batch(arr, len(ps), C.byref(o), C.byref(alloc.struct), ibb._stream_ptr(), outs, sts)
        torch.cuda.synchronize()
        got = [(sts[i], bool(outs[i])) for i in range(len(ps))]
        for i in range(len(ps)):
            if outs[i]:
                L.ibb_result_free(C.c_void_p(outs[i]))
        return rc, got

    counts = []
    for _ in range(2):
        a = CountingAllocator()
        rc, got = run(a)
        assert rc == ibb.OK and all(st in (ibb.OK, ibb.NOT_CONVERGED) and have for st, have in got)
        assert not a.live and a.bad_frees == 0
        counts.append(a.calls)
    total = counts[-1]
    outcomes = set()
    for fail_at in sorted({1, 2, max(1, total // 3), max(1, total // 2), total}):
        print(f"case batch refuse request {fail_at} of {total} incremental={incremental}", flush=True)
        a = CountingAllocator(fail_at)
        rc, got = run(a)
        assert rc in (ibb.OK, NOMEM), rc
        for st, have in got:
            assert have == (st in (ibb.OK, ibb.NOT_CONVERGED))
            assert st in (ibb.OK, ibb.NOT_CONVERGED, NOMEM, ibb.PENDING)
        assert not a.live and a.bad_frees == 0, (fail_at, a.live)
        outcomes.add(rc)
    assert NOMEM in outcomes
