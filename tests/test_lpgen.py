"""The seeded input generators (lpgen) keep the contracts the tests and the
benchmark rely on (CPU only): canonical CSR, the stated sizes and bounds,
planted points that are feasible, bounded LPs (HiGHS finds an optimum),
infeasible and unbounded variants whose planted rays pass the oracle's
Farkas tests (and HiGHS agrees on the status), the batched size law, the
serving trace's arrival process and mix, and determinism in the seed."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import lpgen
import oracle


def _csr(lp):
    return sp.csr_matrix((lp.val, lp.col, lp.rowptr), shape=(lp.m, lp.n))


def _canonical(lp):
    rp, col = lp.rowptr, lp.col
    assert rp[0] == 0 and rp[-1] == len(col) == len(lp.val)
    assert np.all(np.diff(rp) >= 0)
    assert np.all((col >= 0) & (col < lp.n))
    for i in range(lp.m):
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0), i
    assert np.all(np.isfinite(lp.val)) and np.all(np.isfinite(lp.c)) and np.all(np.isfinite(lp.rhs))
    assert np.all(lp.lb <= lp.ub)


def _highs(lp):
    K = _csr(lp)
    return linprog(lp.c, A_ub=-K[lp.m_eq:], b_ub=-lp.rhs[lp.m_eq:], A_eq=K[:lp.m_eq], b_eq=lp.rhs[:lp.m_eq],
                   bounds=list(zip(np.where(np.isfinite(lp.lb), lp.lb, None),
                                   np.where(np.isfinite(lp.ub), lp.ub, None))),
                   method="highs")


def test_tiny_shape_box_and_planted_point():
    lp = lpgen.tiny()
    _canonical(lp)
    assert (lp.m_eq, lp.m_ineq, lp.n) == (40, 20, 120)
    assert np.all(lp.lb == 0.0) and np.all(lp.ub == 10.0)
    xs = lp.meta["x_plant"]
    kx = _csr(lp) @ xs
    assert np.allclose(kx[:lp.m_eq], lp.rhs[:lp.m_eq], rtol=0, atol=1e-12)
    slack = kx[lp.m_eq:] - lp.rhs[lp.m_eq:]
    assert np.all(slack >= 0.0) and np.all(slack <= 1.0)
    K = _csr(lp)
    assert np.all(np.diff(K.indptr) > 0) and np.all(np.bincount(K.indices, minlength=lp.n) > 0)


@pytest.mark.parametrize("seed,m,n", [(3, 200, 800), (4, 500, 1500)])
def test_powerlaw_feasible_bounded_and_scaled(seed, m, n):
    lp = lpgen.scaled_powerlaw(seed, m, n)
    _canonical(lp)
    assert lp.m_eq == (3 * m) // 4 and lp.m == m and lp.n == n
    free = ~np.isfinite(lp.lb)
    assert np.all(~np.isfinite(lp.ub[free])) and np.all(lp.lb[~free] == 0.0)
    assert 0.1 < free.mean() < 0.3
    xs = lp.meta["x_plant"]
    assert np.all(xs >= lp.lb) and np.all(xs <= lp.ub)
    kx = _csr(lp) @ xs
    scale = lp.meta["rowscale"]
    assert np.all(np.abs(kx[:lp.m_eq] - lp.rhs[:lp.m_eq]) <= 1e-9 * (1 + np.abs(kx[:lp.m_eq])))
    slack = kx[lp.m_eq:] - lp.rhs[lp.m_eq:]
    assert np.all(slack >= -1e-9 * (1 + np.abs(kx[lp.m_eq:]))) and np.all(slack <= scale[lp.m_eq:] * (1 + 1e-9))
    # rows scaled over six decades, mean row length near 8 n / m
    assert scale.min() >= 1e-3 and scale.max() <= 1e3
    assert 0.5 * 8 * n < lp.nnz < 2.0 * 8 * n
    res = _highs(lp)
    assert res.status == 0, res.message           # feasible and bounded


def test_contradictory_rows_are_certified_infeasible():
    base = lpgen.scaled_powerlaw(5, 120, 360)
    lp = lpgen.add_contradictory_rows(base, seed=9, rel_gap=0.1)
    _canonical(lp)
    i, j = lp.meta["infeasible_rows"]
    y = np.zeros(lp.m)
    y[i], y[j] = -1.0, 1.0
    ok, info = oracle.primal_ray_check(lp, y)
    assert ok, info
    assert _highs(lp).status == 2                 # infeasible


def test_unbounded_column_is_a_ray():
    base = lpgen.scaled_powerlaw(6, 120, 360)
    lp = lpgen.add_unbounded_column(base, seed=11)
    _canonical(lp)
    d = np.zeros(lp.n)
    d[lp.meta["ray_column"]] = 1.0
    ok, info = oracle.dual_ray_check(lp, d)
    assert ok, info
    assert _highs(lp).status == 3                 # unbounded


def test_batch_size_law():
    m, n, inf = lpgen.batch_sizes(lpgen.BASE_SEED + 3, 512)
    assert m.min() >= 500 and m.max() <= 20000
    assert np.all((n >= 2 * m - 1) & (n <= 5 * m + 1))
    assert 0.05 < inf.mean() < 0.15
    # log-uniform: the median near the geometric mean of the range
    assert 0.6 < np.median(m) / np.sqrt(500 * 20000) < 1.6


def test_serving_trace_arrivals_and_mix():
    tr = lpgen.serving_trace(count=6000)
    t = np.array([r.t_arrival for r in tr])
    assert np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1.0 / 200.0) < 0.1 / 200.0         # Poisson at 200 LP/s
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1            # exponential gaps
    kinds = np.array([r.kind for r in tr])
    for kind, frac in (("large", 0.02), ("infeasible", 0.05), ("unbounded", 0.02)):
        assert abs((kinds == kind).mean() - frac) < 0.01, kind


def test_generators_are_deterministic_in_the_seed():
    a, b = lpgen.scaled_powerlaw(7, 300, 900), lpgen.scaled_powerlaw(7, 300, 900)
    for f in ("rowptr", "col", "val", "c", "rhs", "lb", "ub"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = lpgen.scaled_powerlaw(8, 300, 900)
    assert not np.array_equal(a.val[:10], c.val[:10])
    r1 = lpgen.request_instance(lpgen.serving_trace(count=50)[17])
    r2 = lpgen.request_instance(lpgen.serving_trace(count=50)[17])
    assert np.array_equal(r1.col, r2.col) and np.array_equal(r1.rhs, r2.rhs)
