"""Box bounds on the GPU against the oracle (ibb_eval_boxes through the C ABI).

CHAIN uses only +, -, x and sqr: F, the midpoint upper bound, the first-order
flag and every gradient component must be bit-identical.  The separable
families also use cos(2 pi y) / sin(2 pi y), where the GPU enclosure contains
the oracle's and is at most two doubles wider: by inclusion isotonicity the GPU
F and G must contain the oracle's, the GPU midpoint bound must be >= the
oracle's, and the excess must stay tiny.  Sizes span several 64-wide tiles with
a ragged tail; the workload sizes (n = 100, 1000, 10000) are checked on a
sample of boxes.
"""
import dataclasses

import numpy as np
import pytest

import test_oracle_sum_order as SUM
from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def both(p, nb, seed, width=0.3, grad=True):
    lo, hi = PR.random_boxes(p, nb, seed=seed, max_width_frac=width)
    # include the point box at the minimiser and a box touching the domain edge
    lo[0], hi[0] = p.x_star, p.x_star
    lo[1] = p.lower
    print(f"case {p.name} nb={nb} seed={seed}", flush=True)
    ref = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi, want_grad=grad)
    got = ibb.eval_boxes(p, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda(), want_grad=grad)
    torch.cuda.synchronize()
    got = tuple(None if t is None else t.cpu().numpy() for t in got)
    return ref, got


@pytest.mark.parametrize("n", [2, 7, 64, 130, 1000])
def test_chain_bit_exact(n):
    p = PR.chain(n, 300 + n)
    (F, ub, mono, G), (gF, gub, gmono, gG) = both(p, 96 if n <= 130 else 24, seed=n)
    assert np.array_equal(gF, F)
    assert np.array_equal(gub, ub)
    assert np.array_equal(gmono, mono)
    assert np.array_equal(gG, G)
    assert F[0].tolist() == [0.0, 0.0] and ub[0] == 0.0


def _contains(outer, inner):
    return np.all(outer[..., 0] <= inner[..., 0]) and np.all(inner[..., 1] <= outer[..., 1])


@pytest.mark.parametrize("fam,n", [(PR.SEP_COS, 1), (PR.SEP_COS, 5), (PR.SEP_COS, 100), (PR.SEP_COS, 131),
                                   (PR.SEP_ABS_SIN2, 3), (PR.SEP_ABS_SIN2, 100), (PR.SEP_ABS_SIN2, 200)])
def test_separable_contains_oracle(fam, n):
    p = PR.make(fam, n, 400 + n)
    (F, ub, mono, G), (gF, gub, gmono, gG) = both(p, 64, seed=n)
    assert _contains(gF, F) and _contains(gG, G)
    assert np.all(gub >= ub)
    # GPU discards a box only when the oracle does (its G contains the oracle's)
    assert not np.any(gmono & ~mono)
    # the excess is a few units in the last place of each term
    scale = np.abs(F).max(axis=1) + 1.0
    assert np.all((F[:, 0] - gF[:, 0]) <= 1e-13 * n * scale) and np.all((gF[:, 1] - F[:, 1]) <= 1e-13 * n * scale)
    assert np.all(gub - ub <= 1e-13 * n * (np.abs(ub) + 1.0))
    assert gF[0].tolist() == [0.0, 0.0]


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_workload_sizes_sampled(cfg):
    p = PR.config(cfg)
    nb = 6 if cfg == 3 else 16
    (F, ub, mono), (gF, gub, gmono) = both(p, nb, seed=cfg, grad=False)
    if p.family == PR.CHAIN:
        assert np.array_equal(gF, F) and np.array_equal(gub, ub) and np.array_equal(gmono, mono)
    else:
        assert _contains(gF, F) and np.all(gub >= ub) and not np.any(gmono & ~mono)
        assert np.all(np.abs(gF - F) <= 1e-12 * p.n * (np.abs(F) + 1.0))


@pytest.mark.parametrize("precision", [ibb.FP64, ibb.FP32_BULK])
def test_empty_box_batch(precision):
    # no boxes: empty results, no launch
    p = PR.sep_cos(5, 3)
    print(f"case empty batch precision={precision}", flush=True)
    e = torch.empty((0, 5), dtype=torch.float64, device="cuda")
    F, ub, mono, G = ibb.eval_boxes(p, e, e.clone(), want_grad=True, precision=precision)
    torch.cuda.synchronize()
    assert F.shape == (0, 2) and ub.shape == (0,) and mono.shape == (0,) and G.shape == (0, 5, 2)


@pytest.mark.parametrize("n,seed", SUM.CASES)
def test_sum_order_bit_exact(n, seed):
    # point boxes whose terms are exactly t_i (the oracle pin of the canonical
    # order): the GPU's slot sums and wavefront fold must give the bits that the
    # exact-rational evaluation of that order gives, in both directions
    ts = SUM.designed_terms(n, seed)
    coef, lower, upper = SUM.point_problem(ts)
    p = dataclasses.replace(PR.sep_abs_sin2(n, 1), coef=coef, lower=lower, upper=upper, x_star=None)
    x = torch.from_numpy(ts.reshape(1, -1)).cuda()
    print(f"case sum order n={n} seed={seed}", flush=True)
    F, ub, mono = (t.cpu().numpy() for t in ibb.eval_boxes(p, x, x))
    tl = [float(t) for t in ts]
    assert F[0, 0] == SUM.canonical(tl, False) and F[0, 1] == SUM.canonical(tl, True)
    assert ub[0] == SUM.canonical(tl, True)
