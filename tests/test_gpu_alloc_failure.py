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
