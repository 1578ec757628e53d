"""Pin of the oracle's selection of K boxes per sweep (Sec. 3.1 selects the region
with the smallest lower bound; the sweep generalises it to the K smallest
(lower bound, insertion number), and the children of the K parents enter the
list in (parent rank, child index) order).

Read off the oracle's own output lists after t and t + 1 sweeps:
  * the boxes that leave the list in sweep t + 1 are exactly the K smallest
    (lower bound, insertion number) of the list after t sweeps, plus the boxes
    the new GUB cuts off (lower bound > GUB);
  * the trace's selected insertion number is that of the rank-0 parent;
  * every new box lies inside one of the K parents and is one of its children
    (each side is the parent's or one half of it), and the new insertion numbers
    increase with the parent's rank and, within a parent, with the child index
    (bit j: upper half of the j-th coordinate of the parent's split window).
A wrong rank order, a missing parent, a parent selected twice or children
appended parent-interleaved all break one of these.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR


def run(p, t, k, m):
    return O.solve(p.family, p.coef, p.lower, p.upper, tol_f=1e-30, split_dims=m, select_k=k, max_sweeps=t)


def child_index(par_lo, par_hi, lo, hi, n):
    """(window start, r) of a child box inside its parent, from the split sides."""
    split = np.nonzero((lo != par_lo) | (hi != par_hi))[0]
    upper = {int(d): bool(lo[d] != par_lo[d]) for d in split}
    return split, upper


@pytest.mark.parametrize("make,k,m,sweeps", [(lambda: PR.chain(7, 505, hi=2.3), 2, 3, 7),
                                             (lambda: PR.chain(7, 505, hi=2.3), 4, 3, 5),
                                             (lambda: PR.sep_cos(5, 7), 3, 2, 8),
                                             (lambda: PR.sep_abs_sin2(6, 4), 5, 2, 5)])
def test_k_smallest_selected_and_children_in_rank_order(make, k, m, sweeps):
    p = make()
    n = p.n
    prev = run(p, 0, k, m)
    for t in range(sweeps):
        nxt = run(p, t + 1, k, m)
        assert nxt.sweeps == t + 1
        gub = nxt.trace_gub[t]
        keys = sorted(range(len(prev.seq)), key=lambda i: (prev.flo[i], prev.seq[i]))
        sel = keys[:k]
        assert nxt.trace_sel[t] == prev.seq[sel[0]]
        old = set(prev.seq.tolist())
        kept = set(nxt.seq.tolist()) & old
        gone = old - kept
        cut = {int(prev.seq[i]) for i in range(len(prev.seq)) if prev.flo[i] > gub}
        assert gone == {int(prev.seq[i]) for i in sel} | cut
        # the new boxes: children of the selected parents, in (rank, child index) order
        new = [i for i in range(len(nxt.seq)) if int(nxt.seq[i]) not in old]
        assert all(nxt.seq[i] > max(old) for i in new)
        order = []
        for i in new:
            owners = [rk for rk, j in enumerate(sel)
                      if np.all(prev.lo[j] <= nxt.lo[i]) and np.all(nxt.hi[i] <= prev.hi[j])]
            assert len(owners) == 1
            rk = owners[0]
            j = sel[rk]
            split, upper = child_index(prev.lo[j], prev.hi[j], nxt.lo[i], nxt.hi[i], n)
            for d in split:   # each split side is one half of the parent's side
                mid = nxt.lo[i][d] if upper[int(d)] else nxt.hi[i][d]
                assert prev.lo[j][d] < mid < prev.hi[j][d]
            order.append((rk, split, upper, int(nxt.seq[i])))
        by_rank = {}
        for rk, split, upper, sq in order:
            by_rank.setdefault(rk, []).append((split, upper, sq))
        ranks = [rk for rk, *_ in sorted(order, key=lambda e: e[3])]
        assert ranks == sorted(ranks)             # parent-major order
        for rk, kids in by_rank.items():
            # the window of split coordinates is cyclic; its start is the split
            # coordinate whose predecessor (mod n) is not split in any child
            dims = set(int(d) for s, _, _ in kids for d in s)
            starts = [d for d in dims if (d - 1) % n not in dims] or [min(dims)]
            start = starts[0]
            rs = []
            for split, upper, sq in sorted(kids, key=lambda e: e[2]):
                r = sum((1 << ((d - start) % n)) for d in dims if upper.get(d, False))
                rs.append(r)
            assert rs == sorted(rs) and len(set(rs)) == len(rs)
        prev = nxt
