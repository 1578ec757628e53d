"""Pin of the canonical summation order that defines F (the paper fixes no order
of the additions in its natural interval extension, Sec. 2.1; the reading
adopted here: term i goes to slot i mod 64, each slot sums its terms left to
right, then slots are folded with strides 32, 16, 8, 4, 2, 1, slot s absorbing
slot s + h).

The boxes are points of the non-smooth separable family with s_i = 1, b_i = 0,
c_i = 0, so that term i is exactly |x_i| and only the order of the directed
additions decides the bits of F.  The expected endpoints are computed here with
exact rational arithmetic and a directed rounding to double written from its
definition (the neighbouring double on the required side), not with the
floating-point rounding modes the oracle switches.  The terms are chosen so that
every plausible other order (plain left to right, 32 slots, the folds taken
with increasing strides, slots summed right to left) gives other bits, which the
test checks first: a wrong slot, fold or direction in the oracle fails it.
"""
import math
from fractions import Fraction as Q

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR


def rnd(q: Q, up: bool) -> float:
    """q rounded to a double toward +inf (up) or -inf."""
    f = float(q)                      # nearest double (int / int division rounds correctly)
    if Q(f) == q:
        return f
    if up:
        return f if Q(f) > q else math.nextafter(f, math.inf)
    return f if Q(f) < q else math.nextafter(f, -math.inf)


def dadd(a: float, b: float, up: bool) -> float:
    return rnd(Q(a) + Q(b), up)


def slot_fold(ts, up, nslots=64, fold="halves", reverse_slots=False):
    """Slot sums of ts (term i in slot i mod nslots, in increasing i, or decreasing
    with reverse_slots), then a fold: "halves" adds slot s + h into slot s for
    s < h, h = nslots/2, ..., 1; "pairs" adds slot s + h into slot s for s a
    multiple of 2h, h = 1, 2, ..., nslots/2."""
    slot = [None] * nslots
    order = range(len(ts) - 1, -1, -1) if reverse_slots else range(len(ts))
    for i in order:
        s = i % nslots
        slot[s] = ts[i] if slot[s] is None else dadd(slot[s], ts[i], up)
    hs = [nslots >> k for k in range(1, nslots.bit_length())]
    if fold == "pairs":
        hs = hs[::-1]
    for h in hs:
        targets = range(h) if fold == "halves" else range(0, nslots, 2 * h)
        for s in targets:
            if slot[s + h] is not None:
                slot[s] = slot[s + h] if slot[s] is None else dadd(slot[s], slot[s + h], up)
    return slot[0] if slot[0] is not None else 0.0


def canonical(ts, up):
    return slot_fold(ts, up)


def alternatives(ts, up):
    """Other plausible orders, each of which differs from the canonical one for
    the terms used here (orders that coincide with it for n <= 64 are left out)."""
    seq = ts[0]
    for t in ts[1:]:
        seq = dadd(seq, t, up)
    alt = {"left to right": seq, "folds by pairs": slot_fold(ts, up, fold="pairs")}
    if len(ts) > 64:
        alt["32 slots"] = slot_fold(ts, up, nslots=32)
        alt["slots right to left"] = slot_fold(ts, up, reverse_slots=True)
    return alt


def designed_terms(n: int, seed: int) -> np.ndarray:
    """Terms of mixed magnitudes: large ones, tiny ones that vanish when added to a
    large sum one at a time but not when grouped first, and mid-sized ones."""
    rng = np.random.default_rng(seed)
    ts = np.empty(n)
    for i in range(n):
        kind = rng.integers(0, 4)
        if kind == 0:
            ts[i] = rng.uniform(0.5, 4.0)
        elif kind == 1:
            ts[i] = 2.0 ** -int(rng.integers(50, 56)) * (1 + int(rng.integers(0, 8)) / 8)
        elif kind == 2:
            ts[i] = rng.uniform(1e-9, 1e-6)
        else:
            ts[i] = 3.0 * 2.0 ** -int(rng.integers(20, 54))
    if n > 99:
        # slot 3: a large term, then tiny ones that the canonical order pairs with
        # each other (terms 35 and 99 meet in the fold of stride 32) but that
        # 32 slots, or left-to-right addition, add to the large sum one at a time
        ts[3], ts[35], ts[67], ts[99] = 1.0, 2.0 ** -53, 2.0 ** -70, 2.0 ** -53
    return ts


def point_problem(ts: np.ndarray):
    """Non-smooth separable family with s = 1, b = 0, k = 1, c = 0: term i at the
    point x_i = t_i is exactly t_i."""
    n = ts.shape[0]
    coef = np.concatenate([np.ones(n), np.zeros(n), np.ones(n), np.zeros(n)])
    return coef, -10.0 * np.ones(n), 10.0 * np.ones(n)


CASES = [(130, 49), (200, 4), (160, 5), (64, 3)]   # seeds whose terms tell every order above apart


@pytest.mark.parametrize("n,seed", CASES)
def test_terms_discriminate_the_order(n, seed):
    # every other order gives other bits in at least one endpoint, so the pin below
    # would catch an oracle that used it
    ts = [float(t) for t in designed_terms(n, seed)]
    lo, hi = canonical(ts, False), canonical(ts, True)
    alo, ahi = alternatives(ts, False), alternatives(ts, True)
    for name in alo:
        assert (alo[name], ahi[name]) != (lo, hi), name


@pytest.mark.parametrize("n,seed", CASES)
def test_oracle_sum_follows_the_canonical_order(n, seed):
    ts = designed_terms(n, seed)
    coef, lower, upper = point_problem(ts)
    x = ts.reshape(1, -1)
    F, ub, mono = O.eval_boxes(PR.SEP_ABS_SIN2, coef, lower, upper, x, x)
    tl = [float(t) for t in ts]
    assert F[0, 0] == canonical(tl, False)
    assert F[0, 1] == canonical(tl, True)
    # the midpoint upper bound is the same sum rounded up (the midpoint of a point is the point)
    assert ub[0] == canonical(tl, True)
