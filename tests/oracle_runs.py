"""Oracle iterations for the GPU parity tests, computed on host threads.

A GPU test module lists the oracle runs its cases need when it is imported
(`prefetch`), and the runs start at once on a pool of daemon threads; a test
then takes its result with `solve`, which waits for the prefetched run or, for
a run nobody prefetched, computes it in place.  The GPU work of earlier tests
overlaps the oracle's CPU work of later ones.

This is sound because the oracle is plain C called through ctypes (the GIL is
released for the whole call), keeps no global state, and switches its rounding
mode with fesetround, which acts on the calling thread only.  The threads are
daemons: a run that stops early (pytest -x) does not wait for queued work.
"""
from __future__ import annotations

import hashlib
import os
import queue
import threading

import numpy as np

from oracle import oracle as O

_WORKERS = max(1, min(16, (os.cpu_count() or 1) - 1))
_jobs: "queue.Queue" = queue.Queue()
_lock = threading.Lock()
_runs: dict = {}
_started = False


class _Run:
    def __init__(self, args, kw):
        self.args, self.kw = args, kw
        self.done = threading.Event()
        self.value = None
        self.error = None
        self._claimed = False

    def claim(self):
        """True for the one caller that gets to compute this run."""
        with _lock:
            if self._claimed:
                return False
            self._claimed = True
            return True

    def compute(self):
        try:
            self.value = O.solve(*self.args, **self.kw)
        except BaseException as e:  # handed to the test that asks for it
            self.error = e
        finally:
            self.done.set()


def _worker():
    while True:
        run = _jobs.get()
        if run.claim():
            run.compute()


def _start():
    global _started
    if not _started:
        _started = True
        for _ in range(_WORKERS):
            threading.Thread(target=_worker, daemon=True).start()


def _key(p, kw):
    h = hashlib.sha256()
    for a in (p.coef, p.lower, p.upper):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return (p.family, h.hexdigest(), float(p.tol_f), float(p.tol_x), tuple(sorted(kw.items())))


def _args(p, kw):
    kw = dict(kw)
    kw.setdefault("tol_f", p.tol_f)
    kw.setdefault("tol_x", p.tol_x)
    return (p.family, p.coef, p.lower, p.upper), kw


def prefetch(p, **kw):
    """Start the oracle run of problem p with options kw (those of oracle.solve)."""
    k = _key(p, kw)
    with _lock:
        if k in _runs:
            return
        args, akw = _args(p, kw)
        run = _Run(args, akw)
        _runs[k] = run
        _start()
    _jobs.put(run)


def solve(p, **kw):
    """The oracle run of problem p with options kw: the prefetched one, or a new one."""
    k = _key(p, kw)
    with _lock:
        run = _runs.get(k)
        if run is None:
            args, akw = _args(p, kw)
            run = _runs[k] = _Run(args, akw)
    if run.claim():      # not started by a worker yet: compute it here
        run.compute()
    else:
        run.done.wait()
    with _lock:
        _runs.pop(k, None)   # each result is taken once: the memory goes with it
    if run.error is not None:
        raise run.error
    return run.value
