"""The C ABI (include/ibb.h) without a GPU: every declared entry point is exported,
and argument validation rejects bad problems before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2507_01770_amd as ibb
from paper_2507_01770_amd import problems as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ibb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibb_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 11, names
    L = ibb.lib()
    for name in names:
        assert hasattr(L, name), name


def test_options_default_and_status_strings():
    L = ibb.lib()
    o = ibb._Options()
    assert L.ibb_options_default(C.byref(o)) == 0
    assert (o.precision, o.split_dims, o.select_k, o.deterministic) == (0, 10, 1, 1)
    for s in [0, 1, 2, -1, -2, -3, -4, -5]:
        assert L.ibb_status_string(s)


def _solve_rc(**kw):
    p = PR.sep_cos(3, 1)
    args = dict(family=p.family, coef=p.coef, lower=p.lower, upper=p.upper, tol_f=1e-6, tol_x=0.0)
    args.update(kw)
    k = ibb._ProblemKeep(args["family"], args["coef"], args["lower"], args["upper"], args["tol_f"], args["tol_x"])
    o = ibb._Options()
    ibb.lib().ibb_options_default(C.byref(o))
    for key in ("split_dims", "select_k", "precision", "pieces", "diag_samples", "incremental"):
        if key in kw:
            setattr(o, key, kw[key])
    h = C.c_void_p()
    rc = ibb.lib().ibb_solve(C.byref(k.s), C.byref(o), None, None, C.byref(h))
    return rc, ibb.lib().ibb_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(family=7), "unknown family"),
    (dict(coef=np.zeros(5)), "coef_len"),
    (dict(lower=np.array([0.0, 0.0, 1.0]), upper=np.array([1.0, 1.0, 1.0])), "lower < upper"),
    (dict(upper=np.array([1.0, np.inf, 1.0])), "finite"),
    (dict(tol_f=0.0), "tol_f"),
    (dict(coef=np.concatenate([np.ones(3), np.ones(3), [1.5, 1, 1], np.zeros(3)])), "positive integer"),
    (dict(split_dims=17), "split_dims"),
    (dict(select_k=0), "select_k"),
    (dict(select_k=1025), "select_k"),
    (dict(select_k=1024, split_dims=15), "2^24"),
    (dict(pieces=3), "pieces"),
    (dict(pieces=4, diag_samples=0), "pieces"),
    (dict(pieces=2, diag_samples=10), "pieces"),
    (dict(pieces=4, diag_samples=17), "pieces"),
    (dict(pieces=4, diag_samples=10, select_k=2), "four-piece"),
    (dict(pieces=4, diag_samples=10, incremental=0), "four-piece"),
    (dict(pieces=4, diag_samples=10, split_dims=13), "12 coordinates"),
])
def test_validation_rejects_before_touching_the_device(kw, msg):
    rc, err = _solve_rc(**kw)
    assert rc == -1 and msg in err, (rc, err)


def _problem_struct():
    p = PR.sep_cos(3, 1)
    return ibb._ProblemKeep(p.family, p.coef, p.lower, p.upper, 1e-6, 0.0)


def test_empty_inputs_are_accepted_without_device_work():
    # count 0 / nb 0 returns before any device call, with NULL arrays
    L = ibb.lib()
    k = _problem_struct()
    assert L.ibb_eval_boxes(C.byref(k.s), 0, 0, None, None, None, None, None, None, None) == 0
    assert L.ibb_eval_boxes_noalloc(C.byref(k.s), 0, 0, None, None, None, None, None, None, None) == 0
    assert L.ibb_interval_op(0, 0, None, None, None, None) == 0
    assert L.ibb_point_trig(0, 0, None, None, None) == 0
    assert L.ibb_interval_op32(0, 0, None, None, None, None) == 0
    assert L.ibb_point_trig32(1, 0, None, None, None) == 0


@pytest.mark.parametrize("call,msg", [
    (lambda L, k: L.ibb_eval_boxes(C.byref(k.s), 0, -1, None, None, None, None, None, None, None), "nb < 0"),
    (lambda L, k: L.ibb_eval_boxes(C.byref(k.s), 0, 4, None, None, None, None, None, None, None), "NULL"),
    (lambda L, k: L.ibb_eval_boxes(C.byref(k.s), 5, 4, None, None, None, None, None, None, None), "precision"),
    (lambda L, k: L.ibb_eval_boxes_noalloc(C.byref(k.s), 0, -1, None, None, None, None, None, None, None), "nb < 0"),
    (lambda L, k: L.ibb_eval_boxes_noalloc(C.byref(k.s), 0, 4, None, None, None, None, None, None, None), "NULL"),
    (lambda L, k: L.ibb_eval_boxes_noalloc(C.byref(k.s), 5, 4, None, None, None, None, None, None, None), "precision"),
    (lambda L, k: L.ibb_interval_op(14, 4, None, None, None, None), "unknown op"),
    (lambda L, k: L.ibb_interval_op(0, -1, None, None, None, None), "count < 0"),
    (lambda L, k: L.ibb_interval_op(0, 4, None, None, None, None), "NULL"),
    (lambda L, k: L.ibb_point_trig(2, 4, None, None, None), "fn must be"),
    (lambda L, k: L.ibb_point_trig(0, -3, None, None, None), "count < 0"),
    (lambda L, k: L.ibb_interval_op32(3, 4, None, None, None, None), "single precision"),
    (lambda L, k: L.ibb_point_trig32(0, 4, None, None, None), "NULL"),
])
def test_bad_kernel_arguments_rejected_before_the_device(call, msg):
    L = ibb.lib()
    rc = call(L, _problem_struct())
    assert rc == -1 and msg in L.ibb_last_error().decode()


@pytest.mark.parametrize("n,prec,fits", [(100_000, 1, True), (120_000, 1, False), (170_000, 0, True),
                                         (180_000, 0, False)])
def test_noalloc_array_limit_checked_before_the_device(n, prec, fits):
    # the fixed device array (16 MiB) holds the problem's tables, or the call is
    # refused with IBB_E_CAPACITY before any device work (nb = 0 returns after the check)
    p = PR.sep_cos(n, 7)
    k = ibb._ProblemKeep(p.family, p.coef, p.lower, p.upper, 1e-6, 0.0)
    L = ibb.lib()
    rc = L.ibb_eval_boxes_noalloc(C.byref(k.s), prec, 0, None, None, None, None, None, None, None)
    if fits:
        assert rc == 0
    else:
        assert rc == -4 and "fixed device array" in L.ibb_last_error().decode()


def test_batch_and_server_take_one_box_per_sweep():
    # K > 1 boxes per sweep runs in ibb_solve / ibb_sweep; the batched engine and
    # the server refuse it before any device work
    k = _problem_struct()
    o = ibb._Options()
    L = ibb.lib()
    L.ibb_options_default(C.byref(o))
    o.select_k = 4
    outs = (C.c_void_p * 1)()
    sts = (C.c_int32 * 1)()
    rc = L.ibb_solve_batch(C.byref(k.s), 1, C.byref(o), None, None, outs, sts)
    assert rc == -1 and "select_k" in L.ibb_last_error().decode()


def test_malformed_tapes_refused_before_the_device():
    # the generic family's tape is checked op by op before any device work
    from paper_2507_01770_amd import tapes as TP
    L = ibb.lib()
    good = TP.ackley(3)

    def solve(coef):
        k = ibb._ProblemKeep(TP.TAPE, coef, good.lower, good.upper, 1e-6, 0.0)
        o = ibb._Options()
        L.ibb_options_default(C.byref(o))
        h = C.c_void_p()
        return L.ibb_solve(C.byref(k.s), C.byref(o), None, None, C.byref(h))

    cases = []
    c = good.coef.copy(); c[0] = 2.0; cases.append(c)                      # unknown format
    c = good.coef.copy(); c[1] = 9.0; cases.append(c)                      # too many reductions
    c = good.coef.copy(); c[4 + 6 + 5 + 1] = 5.0; cases.append(c)          # operand not an earlier op
    c = good.coef.copy(); c[4 + 6] = 99.0; cases.append(c)                 # unknown op code
    cases.append(good.coef[:-1].copy())                                    # length does not match
    c = good.coef.copy(); c[4] = 1.0; c[4 + 6 + 5] = 2.0; cases.append(c)  # x_{i+1} in a product
    for c in cases:
        assert solve(c) == -1 and "tape" in L.ibb_last_error().decode()
