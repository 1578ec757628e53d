"""Seeded synthetic objectives (inputs only: no interval arithmetic lives here).

Three closed-form families with a known global minimum 0, standing in for the
paper's scalable benchmark functions (SI Appendix A and D): a separable
multimodal family (like Rastrigin), a chained non-separable family (like
Rosenbrock) and a non-smooth separable family used at n = 10,000 (the scale of
the paper's Levy runs).  Coefficients are drawn with ``numpy.random.default_rng``
in the order listed for each family; the domain is fixed per family.

Coefficient layouts (all float64, length ``coef_len``):
  SEP_COS       a[n], b[n], k[n], c[n]        f = sum a(x-c)^2 + b(1 - cos(2 pi k (x-c)))
  CHAIN         alpha[n-1], beta[n-1]          f = sum alpha(x_{i+1} - x_i^2)^2 + beta(x_i - 1)^2
  SEP_ABS_SIN2  s[n], b[n], k[n], c[n]        f = sum s|x-c| + b sin^2(pi k (x-c))
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEP_COS, CHAIN, SEP_ABS_SIN2, TAPE = 1, 2, 3, 4
FAMILY_NAMES = {SEP_COS: "sep_cos", CHAIN: "chain", SEP_ABS_SIN2: "sep_abs_sin2", TAPE: "tape"}


@dataclass
class Problem:
    family: int
    n: int
    coef: np.ndarray
    lower: np.ndarray
    upper: np.ndarray
    tol_f: float = 1e-6
    tol_x: float = 0.0
    x_star: np.ndarray = field(default=None)  # a known global minimiser (f = 0 there)

    @property
    def name(self) -> str:
        return f"{FAMILY_NAMES[self.family]}_n{self.n}"


def sep_cos(n: int, seed: int, lo: float = -5.0, hi: float = 5.0) -> Problem:
    g = np.random.default_rng(seed)
    a = g.uniform(0.5, 2.0, n)
    b = g.uniform(1.0, 10.0, n)
    k = g.integers(1, 6, n).astype(np.float64)
    c = g.uniform(-1.0, 1.0, n)
    coef = np.concatenate([a, b, k, c])
    return Problem(SEP_COS, n, coef, np.full(n, lo), np.full(n, hi), x_star=c.copy())


def chain(n: int, seed: int, lo: float = -2.0, hi: float = 2.0) -> Problem:
    if n < 2:
        raise ValueError("the chained family needs n >= 2")
    g = np.random.default_rng(seed)
    alpha = g.uniform(10.0, 100.0, n - 1)
    beta = g.uniform(0.5, 2.0, n - 1)
    coef = np.concatenate([alpha, beta])
    return Problem(CHAIN, n, coef, np.full(n, lo), np.full(n, hi), x_star=np.ones(n))


def sep_abs_sin2(n: int, seed: int, lo: float = -10.0, hi: float = 10.0) -> Problem:
    g = np.random.default_rng(seed)
    s = g.uniform(0.1, 1.0, n)
    b = g.uniform(1.0, 5.0, n)
    k = g.integers(1, 9, n).astype(np.float64)
    c = g.uniform(-1.0, 1.0, n)
    coef = np.concatenate([s, b, k, c])
    return Problem(SEP_ABS_SIN2, n, coef, np.full(n, lo), np.full(n, hi), x_star=c.copy())


def make(family: int, n: int, seed: int) -> Problem:
    return {SEP_COS: sep_cos, CHAIN: chain, SEP_ABS_SIN2: sep_abs_sin2}[family](n, seed)


# The five workloads: index -> (description, constructor)
def config(i: int) -> Problem:
    """Workloads 0-3 (workload 4 is the serving trace, see ``serving_trace``)."""
    if i == 0:
        return sep_cos(2, 101)
    if i == 1:
        return sep_cos(100, 102)
    if i == 2:
        return chain(1000, 103)
    if i == 3:
        return sep_abs_sin2(10000, 104)
    raise ValueError(i)


def serving_trace(count: int = 4096, seed: int = 105, rate: float = 1.0):
    """Requests for the serving workload: n log-uniform in [2, 2000], family uniform
    over the three, Poisson arrivals of the given rate (requests per second).
    Returns a list of (arrival_time_s, Problem)."""
    g = np.random.default_rng(seed)
    ns = np.round(np.exp(g.uniform(np.log(2.0), np.log(2000.0), count))).astype(int)
    fams = g.integers(0, 3, count) + 1
    gaps = g.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    out = []
    for j in range(count):
        fam, n = int(fams[j]), int(ns[j])
        if fam == CHAIN and n < 2:
            n = 2
        out.append((float(t[j]), make(fam, n, 1_000_000 + j)))
    return out


def random_boxes(p: Problem, nb: int, seed: int, max_width_frac: float = 1.0):
    """nb random sub-boxes of p's domain: per coordinate a random width (log-uniform
    down to 1e-12 of the domain) at a random position.  Returns lo, hi [nb, n]."""
    g = np.random.default_rng(seed)
    W = p.upper - p.lower
    frac = np.exp(g.uniform(np.log(1e-12), np.log(max_width_frac), (nb, p.n)))
    w = frac * W
    lo = p.lower + g.uniform(0.0, 1.0, (nb, p.n)) * (W - w)
    hi = lo + w
    hi = np.minimum(hi, p.upper)
    lo = np.minimum(lo, hi)
    return lo, hi
