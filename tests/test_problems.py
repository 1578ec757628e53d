"""The seeded input generators: the recipe of each workload (sizes, domains,
coefficient ranges, the serving mix) and its determinism."""
import numpy as np

from paper_2507_01770_amd import problems as PR


def f_numpy(p, x):
    """the closed forms of the three families at a point (float64)"""
    n = p.n
    if p.family == PR.CHAIN:
        al, be = p.coef[: n - 1], p.coef[n - 1:]
        return float(np.sum(al * (x[1:] - x[:-1] ** 2) ** 2 + be * (x[:-1] - 1.0) ** 2))
    a, b, k, c = p.coef.reshape(4, n)
    if p.family == PR.SEP_COS:
        return float(np.sum(a * (x - c) ** 2 + b * (1.0 - np.cos(2 * np.pi * k * (x - c)))))
    return float(np.sum(a * np.abs(x - c) + b * np.sin(np.pi * k * (x - c)) ** 2))


def test_workloads_have_their_sizes_and_domains():
    want = {0: (PR.SEP_COS, 2, 5.0), 1: (PR.SEP_COS, 100, 5.0), 2: (PR.CHAIN, 1000, 2.0),
            3: (PR.SEP_ABS_SIN2, 10000, 10.0)}
    for i, (fam, n, half) in want.items():
        p = PR.config(i)
        assert (p.family, p.n) == (fam, n)
        assert np.all(p.lower == -half) and np.all(p.upper == half)
        assert p.coef.size == (2 * (n - 1) if fam == PR.CHAIN else 4 * n)
        assert p.tol_f == 1e-6 and np.all(p.lower <= p.x_star) and np.all(p.x_star <= p.upper)


def test_known_minimiser_gives_zero_and_terms_are_nonnegative():
    g = np.random.default_rng(0)
    for p in (PR.sep_cos(7, 1), PR.chain(7, 2), PR.sep_abs_sin2(7, 3)):
        assert abs(f_numpy(p, p.x_star)) < 1e-12
        for _ in range(50):
            x = g.uniform(p.lower, p.upper)
            assert f_numpy(p, x) >= 0.0


def test_coefficient_ranges():
    p = PR.sep_cos(2000, 5)
    a, b, k, c = p.coef.reshape(4, -1)
    assert a.min() >= 0.5 and a.max() <= 2.0 and b.min() >= 1.0 and b.max() <= 10.0
    assert set(np.unique(k)) <= {1, 2, 3, 4, 5} and np.all(np.abs(c) <= 1.0)
    q = PR.sep_abs_sin2(2000, 6)
    s, b, k, c = q.coef.reshape(4, -1)
    assert s.min() >= 0.1 and s.max() <= 1.0 and b.min() >= 1.0 and b.max() <= 5.0
    assert set(np.unique(k)) <= set(range(1, 9))
    r = PR.chain(2000, 7)
    assert r.coef[:1999].min() >= 10.0 and r.coef[:1999].max() <= 100.0
    assert r.coef[1999:].min() >= 0.5 and r.coef[1999:].max() <= 2.0


def test_serving_trace_recipe_and_determinism():
    a = PR.serving_trace(count=600, seed=105)
    b = PR.serving_trace(count=600, seed=105)
    t = np.array([x for x, _ in a])
    ns = np.array([p.n for _, p in a])
    fams = np.array([p.family for _, p in a])
    assert np.all(np.diff(t) > 0)
    assert ns.min() >= 2 and ns.max() <= 2000
    # log-uniform sizes on [2, 2000]: P(n <= 20) = log(10) / log(1000) = 1/3
    frac_small = np.mean(ns <= 20)
    assert 0.25 < frac_small < 0.42
    assert set(fams) == {PR.SEP_COS, PR.CHAIN, PR.SEP_ABS_SIN2}
    for (ta, pa), (tb, pb) in zip(a, b):
        assert ta == tb and pa.family == pb.family and np.array_equal(pa.coef, pb.coef)


def test_random_boxes_lie_in_the_domain():
    p = PR.sep_cos(9, 2)
    lo, hi = PR.random_boxes(p, 500, seed=3, max_width_frac=0.3)
    assert np.all(p.lower <= lo) and np.all(lo <= hi) and np.all(hi <= p.upper)
    assert np.all(hi - lo <= 0.3 * (p.upper - p.lower) * (1 + 1e-12))
