"""Rigorous interval branch-and-bound minimisation on AMD MI355X (gfx950).

Thin binding over ``libibb.so`` (C ABI in ``include/ibb.h``): it marshals
arguments only.  Every step of the method runs in the HIP kernels of the
library; PyTorch provides device memory (its caching allocator) and streams.
There is no CPU fallback: when the library is missing, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import problems  # noqa: F401  (seeded inputs)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibb.so")

SEP_COS, CHAIN, SEP_ABS_SIN2 = 1, 2, 3
FP64, FP32_BULK = 0, 1
OK, NOT_CONVERGED, PENDING = 0, 1, 2
OPS = dict(add=0, sub=1, mul=2, div=3, sqrt=4, sqr=5, abs=6, recip=7, cos2pi=8, sin2pi=9, dabs=10, exp=11,
           cos=12, sin=13)


class IbbError(RuntimeError):
    pass


class _Problem(C.Structure):
    _fields_ = [("family", C.c_int32), ("n", C.c_int32),
                ("coef", C.POINTER(C.c_double)), ("coef_len", C.c_int64),
                ("lower", C.POINTER(C.c_double)), ("upper", C.POINTER(C.c_double)),
                ("tol_f", C.c_double), ("tol_x", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("split_dims", C.c_int32), ("select_k", C.c_int32),
                ("deterministic", C.c_int32), ("max_sweeps", C.c_int64), ("max_live_boxes", C.c_int64),
                ("time_limit_s", C.c_double), ("profile", C.c_int32), ("bound_shape", C.c_int32),
                ("incremental", C.c_int32), ("pieces", C.c_int32), ("diag_samples", C.c_int32),
                ("reserved", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


class _Info(C.Structure):
    _fields_ = [("f_lo", C.c_double), ("f_hi", C.c_double), ("n_boxes", C.c_int64), ("sweeps", C.c_int64),
                ("boxes_evaluated", C.c_int64), ("fp32_pruned", C.c_int64), ("fp64_confirmed", C.c_int64),
                ("seconds", C.c_double), ("status", C.c_int32), ("fp32_sweeps", C.c_int32),
                ("ub_evaluated", C.c_int64), ("t_bound_ms", C.c_double), ("t_select_ms", C.c_double),
                ("n_bound_launches", C.c_int64), ("n_select_launches", C.c_int64),
                ("bound_shape", C.c_int32), ("stop_reason", C.c_int32), ("n_persistent_launches", C.c_int64),
                ("t_persistent_ms", C.c_double), ("n_persistent_sweeps", C.c_int64)]


_lib = None


def lib():
    """Load libibb.so (built by ``__graft_entry__.build()``); raise when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise IbbError(f"{LIB_PATH} is missing: build it with `python paper_2507_01770_amd/build.py`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one the library
    # binds to, so device memory and streams from torch are valid in the library
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.ibb_options_default.argtypes = [C.POINTER(_Options)]
    L.ibb_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(_Allocator), vp, C.POINTER(vp)]
    L.ibb_result_info.argtypes = [vp, C.POINTER(_Info)]
    L.ibb_result_boxes.argtypes = [vp, dp, dp, dp, C.POINTER(i64), i64, C.POINTER(i64)]
    L.ibb_result_trace.argtypes = [vp, dp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), i64, C.POINTER(i64)]
    L.ibb_result_free.argtypes = [vp]
    L.ibb_sweep.argtypes = [vp, i64, vp]
    L.ibb_result_free.restype = None
    L.ibb_eval_boxes.argtypes = [C.POINTER(_Problem), i32, i64, vp, vp, vp, vp, vp, vp, vp]
    L.ibb_eval_boxes_noalloc.argtypes = [C.POINTER(_Problem), i32, i64, vp, vp, vp, vp, vp, vp, vp]
    L.ibb_interval_op.argtypes = [i32, i64, vp, vp, vp, vp]
    L.ibb_point_trig.argtypes = [i32, i64, vp, vp, vp]
    L.ibb_interval_op32.argtypes = [i32, i64, vp, vp, vp, vp]
    L.ibb_point_trig32.argtypes = [i32, i64, vp, vp, vp]
    L.ibb_status_string.restype = C.c_char_p
    L.ibb_status_string.argtypes = [C.c_int]
    L.ibb_last_error.restype = C.c_char_p
    L.ibb_solve_batch.argtypes = [C.POINTER(_Problem), i32, C.POINTER(_Options), C.POINTER(_Allocator), vp,
                                  C.POINTER(vp), C.POINTER(i32)]
    L.ibb_server_create.argtypes = [C.c_size_t, i32, C.POINTER(_Allocator), vp, C.POINTER(vp)]
    L.ibb_server_submit.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Options), C.POINTER(C.c_uint64)]
    L.ibb_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    L.ibb_server_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.ibb_server_destroy.argtypes = [vp]
    for f in ["ibb_options_default", "ibb_solve", "ibb_sweep", "ibb_result_info", "ibb_result_boxes", "ibb_result_trace",
              "ibb_eval_boxes", "ibb_eval_boxes_noalloc", "ibb_interval_op", "ibb_point_trig", "ibb_interval_op32", "ibb_point_trig32",
              "ibb_solve_batch", "ibb_server_create",
              "ibb_server_submit", "ibb_server_poll", "ibb_server_stats", "ibb_server_destroy"]:
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _prec(p) -> int:
    """precision as FP64 / FP32_BULK or the names 'fp64' / 'fp32_bulk'."""
    if isinstance(p, str):
        return {"fp64": FP64, "fp32_bulk": FP32_BULK}[p]
    return int(p)


def _check(rc: int, ok=(OK,)):
    if rc not in ok:
        L = lib()
        raise IbbError(f"{L.ibb_status_string(rc).decode()}: {L.ibb_last_error().decode()}")
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise IbbError("no GPU visible: libibb runs on the device only")
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class _TorchAllocator:
    """ibb_allocator backed by PyTorch's caching allocator."""

    def __init__(self):
        torch = _torch()
        self.torch = torch
        self.device = torch.cuda.current_device()

        def _alloc(ctx, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream)
            except Exception:  # out of memory -> NULL -> IBB_E_NOMEM
                return None

        def _free(ctx, p, nbytes, stream):
            torch.cuda.caching_allocator_delete(p)

        self._a = _ALLOC_FN(_alloc)
        self._f = _FREE_FN(_free)
        self.struct = _Allocator(None, self._a, self._f)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _ProblemKeep:
    def __init__(self, family, coef, lower, upper, tol_f, tol_x):
        self.coef, self.lower, self.upper = _f64(coef), _f64(lower), _f64(upper)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        self.s = _Problem(int(family), int(self.lower.shape[0]), dp(self.coef), int(self.coef.shape[0]),
                          dp(self.lower), dp(self.upper), float(tol_f), float(tol_x))


def _prob_args(problem=None, family=None, coef=None, lower=None, upper=None, tol_f=None, tol_x=None):
    if problem is not None:
        family = problem.family if family is None else family
        coef = problem.coef if coef is None else coef
        lower = problem.lower if lower is None else lower
        upper = problem.upper if upper is None else upper
        tol_f = problem.tol_f if tol_f is None else tol_f
        tol_x = problem.tol_x if tol_x is None else tol_x
    return _ProblemKeep(family, coef, lower, upper, 1e-6 if tol_f is None else tol_f, 0.0 if tol_x is None else tol_x)


# ---------------------------------------------------------------------------
# kernel-level entry points
# ---------------------------------------------------------------------------

def interval_op(op: str, a, b=None, stream=None):
    """Elementwise interval op on device tensors a, b of shape [count, 2] (lo, hi)."""
    torch = _torch()
    a = a.to(device="cuda", dtype=torch.float64).contiguous()
    bb = None if b is None else b.to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty_like(a)
    _check(lib().ibb_interval_op(OPS[op], a.shape[0], C.c_void_p(a.data_ptr()),
                                 None if bb is None else C.c_void_p(bb.data_ptr()), C.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream)))
    return out


def point_trig(fn: str, y, stream=None):
    """[lo, hi] around cos(2 pi y) (fn='cos2pi') or sin(2 pi y) (fn='sin2pi') for a device tensor y."""
    torch = _torch()
    y = y.to(device="cuda", dtype=torch.float64).contiguous().reshape(-1)
    out = torch.empty((y.shape[0], 2), dtype=torch.float64, device="cuda")
    _check(lib().ibb_point_trig(0 if fn == "cos2pi" else 1, y.shape[0], C.c_void_p(y.data_ptr()),
                                C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def interval_op32(op: str, a, b=None, stream=None):
    """Single-precision interval op on device float tensors [count, 2] (lo, hi)."""
    torch = _torch()
    a = a.to(device="cuda", dtype=torch.float32).contiguous()
    bb = None if b is None else b.to(device="cuda", dtype=torch.float32).contiguous()
    out = torch.empty_like(a)
    _check(lib().ibb_interval_op32(OPS[op], a.shape[0], C.c_void_p(a.data_ptr()),
                                   None if bb is None else C.c_void_p(bb.data_ptr()), C.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream)))
    return out


def point_trig32(fn: str, y, stream=None):
    """Float [lo, hi] around cos(2 pi y) or sin(2 pi y) for a device float tensor y."""
    torch = _torch()
    y = y.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1)
    out = torch.empty((y.shape[0], 2), dtype=torch.float32, device="cuda")
    _check(lib().ibb_point_trig32(0 if fn == "cos2pi" else 1, y.shape[0], C.c_void_p(y.data_ptr()),
                                  C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def eval_boxes(problem, lo, hi, want_grad=False, precision=FP64, stream=None):
    """Bound boxes lo, hi ([nb, n] device tensors).  Returns F [nb,2], ub [nb], mono [nb] (bool)
    and, when want_grad, G [nb, n, 2].  precision='fp32_bulk' gives the FP32 filter's F, test and G."""
    return _eval(lib().ibb_eval_boxes, problem, lo, hi, want_grad, precision, stream)


def eval_boxes_noalloc(problem, lo, hi, want_grad=False, precision=FP64, stream=None):
    """eval_boxes through ibb_eval_boxes_noalloc: the library allocates no device memory (its
    problem tables go into a fixed device array); the outputs here are allocated by torch."""
    return _eval(lib().ibb_eval_boxes_noalloc, problem, lo, hi, want_grad, precision, stream)


def _eval(fn, problem, lo, hi, want_grad, precision, stream):
    torch = _torch()
    k = _prob_args(problem)
    lo = lo.to(device="cuda", dtype=torch.float64).contiguous()
    hi = hi.to(device="cuda", dtype=torch.float64).contiguous()
    nb = lo.shape[0]
    F = torch.empty((nb, 2), dtype=torch.float64, device="cuda")
    ub = torch.empty(nb, dtype=torch.float64, device="cuda")
    mono = torch.empty(nb, dtype=torch.uint8, device="cuda")
    G = torch.empty((nb, lo.shape[1], 2), dtype=torch.float64, device="cuda") if want_grad else None
    vp = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    _check(fn(C.byref(k.s), _prec(precision), nb, vp(lo), vp(hi), vp(F), vp(ub), vp(mono),
              None if G is None else vp(G), _stream_ptr(stream)))
    return (F, ub, mono.bool(), G) if want_grad else (F, ub, mono.bool())


# ---------------------------------------------------------------------------
# whole solve
# ---------------------------------------------------------------------------

@dataclass
class Result:
    f_lo: float
    f_hi: float
    status: int
    sweeps: int
    boxes_evaluated: int
    n_boxes: int
    seconds: float
    lo: np.ndarray | None      # [n_boxes, n] live boxes in insertion order (None if not fetched)
    hi: np.ndarray | None
    flo: np.ndarray            # lower bound of f per live box
    seq: np.ndarray            # insertion number per live box
    trace_gub: np.ndarray
    trace_nsurv: np.ndarray
    trace_nlive: np.ndarray
    trace_sel: np.ndarray
    ub_evaluated: int = 0
    t_bound_ms: float = 0.0        # summed k_bound time (profile=True)
    t_select_ms: float = 0.0
    n_bound_launches: int = 0
    n_select_launches: int = 0
    fp32_pruned: int = 0           # children discarded by the FP32 filter
    fp64_confirmed: int = 0        # boxes bounded in FP64
    fp32_sweeps: int = 0           # sweeps in which the FP32 filter ran
    bound_shape: int = -1          # shape of the bound kernel (0..4), picked by the autotuner unless forced
    n_persistent_launches: int = 0   # launches of the persistent sweep kernel (profile=True)
    t_persistent_ms: float = 0.0     # their summed time
    n_persistent_sweeps: int = 0     # the sweeps they ran
    stop_reason: int = 0             # 1 converged, 2 max_sweeps, 3 max_live_boxes, 5 time limit, 8 server memory


def minimize(problem=None, *, family=None, coef=None, lower=None, upper=None, tol_f=None, tol_x=None,
             precision=FP64, split_dims=10, select_k=1, max_sweeps=1_000_000, max_live_boxes=1 << 26,
             time_limit_s=0.0, fetch_boxes=True, max_boxes_fetched=100_000, use_torch_allocator=True,
             profile=False, bound_shape=None, incremental=None, pieces=2, diag_samples=0, stream=None) -> Result:
    """Enclose min f over [lower, upper]; returns [f_lo, f_hi] and the surviving boxes."""
    k = _prob_args(problem, family, coef, lower, upper, tol_f, tol_x)
    L = lib()
    opts = _options(precision, split_dims, select_k, max_sweeps, max_live_boxes, time_limit_s, profile, bound_shape,
                    incremental, pieces, diag_samples)
    alloc = _TorchAllocator() if use_torch_allocator else None
    h = C.c_void_p()
    rc = L.ibb_solve(C.byref(k.s), C.byref(opts), C.byref(alloc.struct) if alloc else None, _stream_ptr(stream),
                     C.byref(h))
    _check(rc, ok=(OK, NOT_CONVERGED))
    return _take_result(h, k.lower.shape[0], fetch_boxes, max_boxes_fetched)


def _take_result(h, n, fetch_boxes=True, max_boxes_fetched=100_000) -> Result:
    """Copy a result out of the library and free it."""
    try:
        return _read_result(h, n, fetch_boxes, max_boxes_fetched)
    finally:
        lib().ibb_result_free(h)


def _read_result(h, n, fetch_boxes=True, max_boxes_fetched=100_000) -> Result:
    """Copy a result out of the library (the handle stays valid)."""
    L = lib()
    info = _Info()
    _check(L.ibb_result_info(h, C.byref(info)))
    nb = info.n_boxes
    nf = min(nb, max_boxes_fetched) if fetch_boxes else 0
    flo = np.empty(nb)
    seq = np.empty(nb, dtype=np.int64)
    lo = np.empty((nf, n)) if fetch_boxes else None
    hi = np.empty((nf, n)) if fetch_boxes else None
    w = C.c_int64()
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))  # noqa: E731
    _check(L.ibb_result_boxes(h, None, None, dp(flo), ip(seq), nb, C.byref(w)))
    if fetch_boxes and nf:
        _check(L.ibb_result_boxes(h, dp(lo), dp(hi), None, None, nf, C.byref(w)))
    ts = info.sweeps
    tg, tn, tl, tsel = np.empty(ts), np.empty(ts, np.int64), np.empty(ts, np.int64), np.empty(ts, np.int64)
    _check(L.ibb_result_trace(h, dp(tg), ip(tn), ip(tl), ip(tsel), ts, C.byref(w)))
    got = w.value
    return Result(info.f_lo, info.f_hi, info.status, info.sweeps, info.boxes_evaluated, nb, info.seconds,
                  lo, hi, flo, seq, tg[:got], tn[:got], tl[:got], tsel[:got], info.ub_evaluated,
                  info.t_bound_ms, info.t_select_ms, info.n_bound_launches, info.n_select_launches,
                  info.fp32_pruned, info.fp64_confirmed, info.fp32_sweeps, info.bound_shape,
                  info.n_persistent_launches, info.t_persistent_ms, info.n_persistent_sweeps, info.stop_reason)


class Run:
    """A run kept on the device: ``Run(problem, max_sweeps=a)`` solves with budget a,
    ``sweep(b)`` continues it for up to b more sweeps (ibb_sweep), ``result()`` reads
    it, ``close()`` frees it."""

    def __init__(self, problem, *, stream=None, **opts):
        self._k = _prob_args(problem)
        self._stream = stream
        o = _options(**opts)
        self._alloc = _TorchAllocator()   # outlives the result: its blocks go back through it
        self._h = C.c_void_p()
        _check(lib().ibb_solve(C.byref(self._k.s), C.byref(o), C.byref(self._alloc.struct), _stream_ptr(stream),
                               C.byref(self._h)), ok=(OK, NOT_CONVERGED))

    def sweep(self, n_sweeps: int) -> int:
        return _check(lib().ibb_sweep(self._h, int(n_sweeps), _stream_ptr(self._stream)), ok=(OK, NOT_CONVERGED))

    def result(self, fetch_boxes=True, max_boxes_fetched=100_000) -> Result:
        return _read_result(self._h, self._k.lower.shape[0], fetch_boxes, max_boxes_fetched)

    def close(self):
        if self._h:
            lib().ibb_result_free(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _options(precision=FP64, split_dims=10, select_k=1, max_sweeps=1_000_000, max_live_boxes=1 << 26,
             time_limit_s=0.0, profile=False, bound_shape=None, incremental=None, pieces=2, diag_samples=0):
    """incremental=None: incremental child bounds unless the FP32 filter or a bound shape
    (both about full bounds) is asked for.  pieces=4, diag_samples=10: the paper's schedule."""
    prec = _prec(precision)
    if incremental is None:
        incremental = prec == FP64 and bound_shape is None
    return _Options(prec, split_dims, select_k, 1, max_sweeps, max_live_boxes, time_limit_s, int(profile),
                    0 if bound_shape is None else int(bound_shape) + 1, int(bool(incremental)), int(pieces),
                    int(diag_samples), 0)


def solve_batch(problems, *, fetch_boxes=True, max_boxes_fetched=100_000, stream=None, **opts) -> list:
    """Solve several problems together (their sweeps share kernel launches).  Returns a
    list of Result (or an IbbError instance for a problem that failed)."""
    L = lib()
    keeps = [_prob_args(p) for p in problems]
    arr = (_Problem * len(keeps))(*[k.s for k in keeps])
    o = _options(**opts)
    outs = (C.c_void_p * len(keeps))()
    sts = (C.c_int32 * len(keeps))()
    alloc = _TorchAllocator()   # kept until every result below has been freed
    rc = L.ibb_solve_batch(arr, len(keeps), C.byref(o), C.byref(alloc.struct), _stream_ptr(stream), outs, sts)
    if rc != OK:   # results of problems that finished before the error are still ours to free
        for i in range(len(keeps)):
            if outs[i]:
                L.ibb_result_free(C.c_void_p(outs[i]))
        _check(rc)
    res = []
    for i, k in enumerate(keeps):
        if sts[i] in (OK, NOT_CONVERGED) and outs[i]:
            res.append(_take_result(C.c_void_p(outs[i]), k.lower.shape[0], fetch_boxes, max_boxes_fetched))
        else:
            res.append(IbbError(f"problem {i}: {L.ibb_status_string(sts[i]).decode()}"))
    return res


class Server:
    """Continuous-batching server (C++ thread inside libibb).  submit() returns a
    ticket; poll() returns None while the problem is pending, else its Result."""

    def __init__(self, mem_budget_bytes=8 << 30, max_slots=64, stream=None):
        torch = _torch()
        self._stream = stream if stream is not None else torch.cuda.Stream()
        # device memory through torch's caching allocator; the callbacks run on the
        # server's own thread (ctypes takes the GIL for them), and the allocator
        # outlives the server and every result it hands over
        self._alloc = _TorchAllocator()
        self._h = C.c_void_p()
        _check(lib().ibb_server_create(int(mem_budget_bytes), int(max_slots), C.byref(self._alloc.struct),
                                       C.c_void_p(self._stream.cuda_stream), C.byref(self._h)))
        self._n = {}

    def submit(self, problem, **opts) -> int:
        k = _prob_args(problem)
        o = _options(**opts)
        t = C.c_uint64()
        _check(lib().ibb_server_submit(self._h, C.byref(k.s), C.byref(o), C.byref(t)))
        self._n[t.value] = k.lower.shape[0]
        return t.value

    def poll(self, ticket, fetch_boxes=False, max_boxes_fetched=100_000):
        out = C.c_void_p()
        rc = lib().ibb_server_poll(self._h, C.c_uint64(ticket), C.byref(out))
        if rc == PENDING:
            return None
        _check(rc, ok=(OK, NOT_CONVERGED))
        return _take_result(out, self._n.pop(ticket), fetch_boxes, max_boxes_fetched)

    def stats(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        _check(lib().ibb_server_stats(self._h, *[C.byref(x) for x in v]))
        return dict(admitted=v[0].value, completed=v[1].value, max_active=v[2].value, queued=v[3].value)

    def close(self):
        if self._h:
            _check(lib().ibb_server_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
