"""ibb_eval_boxes_noalloc (no device allocation: the problem's tables live in a
fixed device array) against ibb_eval_boxes, both through the C ABI: the same F,
midpoint bound, first-order flag and gradient, bit for bit, on consecutive
calls where the second is smaller than the first (the array keeps the previous
call's contents), in both precisions, up to the largest problem the array
holds.  The chained family is also checked against the oracle (bit-exact there).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_01770_amd import problems as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2507_01770_amd as ibb  # noqa: E402


def run_both(p, nb, seed, precision, grad):
    lo, hi = PR.random_boxes(p, nb, seed=seed, max_width_frac=0.3)
    lo[0], hi[0] = p.x_star, p.x_star
    print(f"case {p.name} nb={nb} precision={precision} grad={grad}", flush=True)
    dlo, dhi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    want = ibb.eval_boxes(p, dlo, dhi, want_grad=grad, precision=precision)
    got = ibb.eval_boxes_noalloc(p, dlo, dhi, want_grad=grad, precision=precision)
    torch.cuda.synchronize()
    for a, b in zip(want, got):
        assert (a is None) == (b is None)
        if a is not None:
            assert torch.equal(a, b)
    return lo, hi, got


# (first call, second call): family, n, boxes, precision, gradient
SEQUENCES = [
    ((PR.SEP_COS, 300, 700, ibb.FP64, True), (PR.CHAIN, 37, 50, ibb.FP64, True)),
    ((PR.SEP_ABS_SIN2, 1000, 200, "fp32_bulk", True), (PR.SEP_COS, 5, 3, "fp32_bulk", False)),
    ((PR.CHAIN, 2000, 130, "fp32_bulk", False), (PR.CHAIN, 2, 1, ibb.FP64, True)),
    ((PR.SEP_COS, 100_000, 6, "fp32_bulk", False), (PR.SEP_ABS_SIN2, 64, 65, ibb.FP64, True)),
]


@pytest.mark.parametrize("first,second", SEQUENCES)
def test_noalloc_equals_eval_boxes_on_two_calls(first, second):
    for k, (fam, n, nb, prec, grad) in enumerate((first, second)):
        p = PR.make(fam, n, 900 + n)
        lo, hi, got = run_both(p, nb, seed=10 * k + n, precision=prec, grad=grad)
        if fam == PR.CHAIN and prec == ibb.FP64:
            F, ub, mono, G = O.eval_boxes(p.family, p.coef, p.lower, p.upper, lo, hi, want_grad=True)
            assert np.array_equal(got[0].cpu().numpy(), F) and np.array_equal(got[1].cpu().numpy(), ub)
            assert np.array_equal(got[2].cpu().numpy(), mono.astype(bool))
            if grad:
                assert np.array_equal(got[3].cpu().numpy(), G)


def test_noalloc_refuses_a_problem_beyond_the_array():
    p = PR.sep_cos(200_000, 7)
    lo, hi = PR.random_boxes(p, 2, seed=1)
    with pytest.raises(ibb.IbbError, match="fixed device array"):
        ibb.eval_boxes_noalloc(p, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda(), precision="fp32_bulk")
    # the array is untouched by the refusal: the next call is exact
    run_both(PR.chain(9, 3), 17, seed=3, precision=ibb.FP64, grad=True)
