"""ctypes wrapper around the plain CPU oracle (``ibb_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the GPU library never imports it and it
imports nothing from the GPU package.

The oracle computes, with IEEE directed rounding switched per operation, the
interval extension of f and of its gradient on boxes, the midpoint upper
bound, and the whole best-first branch-and-bound iteration (Sec. 3.1-3.2 of
the paper).  See the header of ``ibb_oracle.c`` for what each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ibb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=gnu11", "-frounding-math", "-fno-fast-math", "-ffp-contract=off",
             "-fexcess-precision=standard", "-fPIC", "-shared"]

SEP_COS, CHAIN, SEP_ABS_SIN2 = 1, 2, 3
OP = dict(add=0, sub=1, mul=2, div=3, sqrt=4, sqr=5, abs=6, recip=7, cos2pi=8, sin2pi=9, dabs=10, exp=11, cos=12, sin=13)
ST_OK, ST_NOT_CONVERGED = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle.so`` next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [("family", C.c_int32), ("n", C.c_int32),
                ("coef", C.POINTER(C.c_double)), ("coef_len", C.c_int64),
                ("lower", C.POINTER(C.c_double)), ("upper", C.POINTER(C.c_double)),
                ("tol_f", C.c_double), ("tol_x", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("split_dims", C.c_int32), ("select_k", C.c_int32),
                ("max_sweeps", C.c_int64), ("max_live_boxes", C.c_int64),
                ("incremental", C.c_int32), ("reserved", C.c_int32),
                ("pieces", C.c_int32), ("samples", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("f_lo", C.c_double), ("f_hi", C.c_double), ("n_boxes", C.c_int64),
                ("sweeps", C.c_int64), ("boxes_evaluated", C.c_int64), ("status", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        dp, i64 = C.POINTER(C.c_double), C.c_int64
        L.orc_solve.restype = C.c_void_p
        L.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), i64]
        L.orc_info_get.argtypes = [C.c_void_p, C.POINTER(_Info)]
        L.orc_boxes.restype = i64
        L.orc_boxes.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(i64), i64]
        L.orc_trace.restype = i64
        L.orc_trace.argtypes = [C.c_void_p, dp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), i64]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_eval_boxes.argtypes = [C.POINTER(_Problem), i64, dp, dp, dp, dp, C.POINTER(C.c_uint8), dp]
        L.orc_iv_op.argtypes = [C.c_int, i64, dp, dp, dp]
        L.orc_point_trig.argtypes = [C.c_int, i64, dp, dp]
        L.orc_midpoint.restype = C.c_double
        L.orc_midpoint.argtypes = [C.c_double, C.c_double]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self, family, coef, lower, upper, tol_f, tol_x):
        self.coef, self.lower, self.upper = _f64(coef), _f64(lower), _f64(upper)
        n = self.lower.shape[0]
        self.p = _Problem(family, n, _dp(self.coef), self.coef.shape[0], _dp(self.lower),
                          _dp(self.upper), float(tol_f), float(tol_x))


def iv_op(op: str, a: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """Apply one interval operation elementwise.  a, b, result: [cnt, 2] (lo, hi)."""
    a = _f64(a).reshape(-1, 2)
    bb = None if b is None else _f64(b).reshape(-1, 2)
    out = np.empty_like(a)
    rc = lib().orc_iv_op(OP[op], a.shape[0], _dp(a), None if bb is None else _dp(bb), _dp(out))
    assert rc == 0
    return out


def point_trig(fn: str, y: np.ndarray) -> np.ndarray:
    """Enclosure [lo, hi] of cos(2 pi y) (fn='cos2pi') or sin(2 pi y) (fn='sin2pi')."""
    y = _f64(y).reshape(-1)
    out = np.empty((y.shape[0], 2))
    lib().orc_point_trig(0 if fn == "cos2pi" else 1, y.shape[0], _dp(y), _dp(out))
    return out


def midpoint(lo: float, hi: float) -> float:
    return lib().orc_midpoint(lo, hi)


def eval_boxes(family, coef, lower, upper, lo, hi, want_grad=False):
    """Bound nb boxes.  lo, hi: [nb, n].  Returns F [nb,2], ub [nb], mono [nb] (bool),
    and G [nb, n, 2] when want_grad."""
    k = _Keep(family, coef, lower, upper, 1e-6, 0.0)
    lo, hi = _f64(lo), _f64(hi)
    nb = lo.shape[0]
    n = k.lower.shape[0]
    F = np.empty((nb, 2))
    ub = np.empty(nb)
    mono = np.empty(nb, dtype=np.uint8)
    G = np.empty((nb, n, 2)) if want_grad else None
    lib().orc_eval_boxes(C.byref(k.p), nb, _dp(lo), _dp(hi), _dp(F), _dp(ub),
                         mono.ctypes.data_as(C.POINTER(C.c_uint8)), None if G is None else _dp(G))
    return (F, ub, mono.astype(bool), G) if want_grad else (F, ub, mono.astype(bool))


@dataclass
class SolveResult:
    f_lo: float
    f_hi: float
    status: int
    sweeps: int
    boxes_evaluated: int
    lo: np.ndarray          # [n_boxes, n], sorted by insertion sequence number
    hi: np.ndarray
    flo: np.ndarray         # lower bound of f per live box
    seq: np.ndarray         # insertion sequence number per live box
    trace_gub: np.ndarray   # GUB after each sweep
    trace_nsurv: np.ndarray  # children inserted by each sweep
    trace_nlive: np.ndarray  # live boxes after each sweep
    trace_sel: np.ndarray   # sequence number of the first selected parent of each sweep


def solve(family, coef, lower, upper, tol_f=1e-6, tol_x=0.0, split_dims=10, select_k=1,
          max_sweeps=100000, max_live_boxes=0, trace_cap=None, incremental=False, pieces=2,
          samples=0) -> SolveResult:
    """The iteration of Sec. 3.1-3.2.  incremental=True bounds each child from its
    parent's shared terms (same enclosures up to the order of the additions).
    pieces=4, samples=10 (with tol_x = 1e-4 and a tol_f that never binds) is the
    schedule of the paper's experiments (Sec. 4): four equal subintervals of each
    cycled coordinate (Eqs. (8)-(11)) and ten sample points on each subregion's
    diagonal; with it, incremental=True is the practical mode (4^m children)."""
    k = _Keep(family, coef, lower, upper, tol_f, tol_x)
    n = k.lower.shape[0]
    if trace_cap is None:
        trace_cap = max_sweeps
    opts = _Options(split_dims, select_k, max_sweeps, max_live_boxes, int(bool(incremental)), 0, pieces, samples)
    L = lib()
    h = L.orc_solve(C.byref(k.p), C.byref(opts), trace_cap)
    if not h:
        raise MemoryError("oracle solve failed to allocate")
    try:
        info = _Info()
        L.orc_info_get(h, C.byref(info))
        nb = info.n_boxes
        lo = np.empty((nb, n)); hi = np.empty((nb, n)); flo = np.empty(nb); seq = np.empty(nb, dtype=np.int64)
        L.orc_boxes(h, _dp(lo), _dp(hi), _dp(flo), seq.ctypes.data_as(C.POINTER(C.c_int64)), nb)
        tc = min(trace_cap, info.sweeps)
        tg = np.empty(tc); ts = np.empty(tc, dtype=np.int64); tl = np.empty(tc, dtype=np.int64)
        tsel = np.empty(tc, dtype=np.int64)
        P64 = C.POINTER(C.c_int64)
        got = L.orc_trace(h, _dp(tg), ts.ctypes.data_as(P64), tl.ctypes.data_as(P64),
                          tsel.ctypes.data_as(P64), tc)
        return SolveResult(info.f_lo, info.f_hi, info.status, info.sweeps, info.boxes_evaluated,
                           lo, hi, flo, seq, tg[:got], ts[:got], tl[:got], tsel[:got])
    finally:
        L.orc_free(h)
