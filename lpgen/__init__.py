"""Seeded synthetic LP generators.

This module is shared by the CPU oracle and by the HIP solver's tests and
benchmark.  It only *draws* instances -- sparsity patterns, values, bounds,
right-hand sides and arrival traces -- and holds none of the solver's
arithmetic (no scaling, no PDHG step, no norms, no KKT evaluation).

Every instance is an LP of the form

    min c^T x   s.t.   A x = b,  G x >= h,  lb <= x <= ub

stored as one CSR matrix K = [A; G] (equality rows first) with right-hand
side rhs = [b; h].  Bounds may be +-inf.

The workloads imitate the paper's benchmark set (LP relaxations of MIPLIB
2017 instances, split by nnz into 100K-1M / 1M-10M / >10M classes, Section 7,
Table 1): that dataset is not available here, so power-law row lengths and
six decades of row scaling stand in for its skew and bad scaling.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 2407_16144


@dataclass
class LP:
    """One LP in CSR form (host arrays).  rowptr/col are int32, the rest f64."""
    n: int
    m_eq: int
    m_ineq: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    c: np.ndarray
    rhs: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.m_eq + self.m_ineq

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


# --------------------------------------------------------------------------
# sparsity helpers (pattern construction only)
# --------------------------------------------------------------------------

def _csr_from_coo(m, n, rows, cols, vals):
    """Sort (row, col) pairs, drop duplicate positions (keep the first draw)."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    keep = np.ones(key.shape[0], dtype=bool)
    keep[1:] = key[1:] != key[:-1]
    order = order[keep]
    r = rows[order].astype(np.int64)
    cidx = cols[order].astype(np.int32)
    v = vals[order]
    counts = np.bincount(r, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr.astype(np.int32), cidx, v


def _matvec(rowptr, col, val, x):
    """Plain CSR product used only to plant right-hand sides."""
    m = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    return np.bincount(rows, weights=val * x[col], minlength=m)


def _rmatvec(rowptr, col, val, y, n):
    m = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    return np.bincount(col, weights=val * y[rows], minlength=n)


def _ensure_nonempty(rng, m, n, rows, cols, vals_fn):
    """Give every empty row and every empty column one random entry."""
    rc = np.bincount(rows, minlength=m)
    cc = np.bincount(cols, minlength=n)
    er = np.nonzero(rc == 0)[0]
    ec = np.nonzero(cc == 0)[0]
    add_r = [er, rng.integers(0, m, size=ec.shape[0])]
    add_c = [rng.integers(0, n, size=er.shape[0]), ec]
    rows = np.concatenate([rows] + add_r)
    cols = np.concatenate([cols] + add_c)
    extra = er.shape[0] + ec.shape[0]
    return rows, cols, extra


# --------------------------------------------------------------------------
# tiny dense-ish instances (oracle finishes in well under a second)
# --------------------------------------------------------------------------

def tiny(seed: int = BASE_SEED, m_eq: int = 40, m_ineq: int = 20, n: int = 120,
         density: float = 0.10) -> LP:
    """Bernoulli(density) pattern with N(0,1) values, every variable boxed in
    [0, 10]; x* ~ U(1, 9); b = A x*; h = G x* - U(0, 1); c ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    m = m_eq + m_ineq
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    rows, cols, _ = _ensure_nonempty(rng, m, n, rows, cols, None)
    vals = rng.standard_normal(rows.shape[0])
    rowptr, col, val = _csr_from_coo(m, n, rows, cols, vals)
    xs = rng.uniform(1.0, 9.0, n)
    kx = _matvec(rowptr, col, val, xs)
    rhs = kx.copy()
    rhs[m_eq:] -= rng.uniform(0.0, 1.0, m_ineq)
    c = rng.standard_normal(n)
    return LP(n, m_eq, m_ineq, rowptr, col, val, c, rhs,
              np.zeros(n), np.full(n, 10.0), {"kind": "tiny", "x_plant": xs, "seed": seed})


def tiny_copy(seed: int = BASE_SEED) -> LP:
    """The 4-row / 6-variable copy of `tiny` used for brute-force vertex checks."""
    return tiny(seed, m_eq=3, m_ineq=1, n=6, density=0.5)


# --------------------------------------------------------------------------
# power-law instances (single large LP, batched and serving workloads)
# --------------------------------------------------------------------------

def _powerlaw_lengths_discrete(rng, m, lmin, lmax, alpha):
    support = np.arange(lmin, lmax + 1, dtype=np.float64)
    p = support ** (-alpha)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(m)
    return (np.searchsorted(cdf, u, side="left") + lmin).astype(np.int64)


def _powerlaw_lengths_continuous(rng, m, a, b, alpha=2.0):
    """Truncated continuous Pareto(alpha=2) on [a, b], rounded to integers."""
    u = rng.random(m)
    # inverse CDF of density ~ L^-2 on [a, b]
    inv = 1.0 / a - u * (1.0 / a - 1.0 / b)
    L = np.rint(1.0 / inv).astype(np.int64)
    return np.clip(L, 1, int(b))


def solve_lmin_for_mean(mean: float, b: float) -> float:
    """Lower end a of a truncated L^-2 law on [a, b] whose mean is `mean`."""
    if mean >= b:
        return b
    lo, hi = 1e-6, b
    for _ in range(200):
        a = 0.5 * (lo + hi)
        mu = math.log(b / a) / (1.0 / a - 1.0 / b)
        if mu < mean:
            lo = a
        else:
            hi = a
    return 0.5 * (lo + hi)


def powerlaw(seed: int, m_eq: int, m_ineq: int, n: int, *, lmin: float | None = None,
             mean_len: float | None = None, lmax: int = 5000, alpha: float = 2.0,
             free_frac: float = 0.2, discrete: bool = True) -> LP:
    """Power-law row lengths P(L) ~ L^-alpha on [lmin, min(lmax, n)], columns
    uniform without replacement per row, values N(0,1) * 10^U(-3,3) per row,
    80% of variables boxed [0, U(1,100)] and 20% free.  Feasible by a planted
    x*; bounded by a planted dual (y*_eq ~ N(0,1), y*_ineq = |N(0,1)|,
    lambda_j ~ N(0,1) on boxed variables) with c = K^T y* + lambda."""
    rng = np.random.default_rng(seed)
    m = m_eq + m_ineq
    b = min(lmax, n)
    if discrete:
        L = _powerlaw_lengths_discrete(rng, m, int(lmin), b, alpha)
    else:
        a = solve_lmin_for_mean(mean_len, b) if lmin is None else lmin
        L = _powerlaw_lengths_continuous(rng, m, a, b, alpha)
    rows = np.repeat(np.arange(m, dtype=np.int64), L)
    cols = rng.integers(0, n, size=rows.shape[0], dtype=np.int64)
    rows, cols, _ = _ensure_nonempty(rng, m, n, rows, cols, None)
    rowscale = 10.0 ** rng.uniform(-3.0, 3.0, m)
    vals = rng.standard_normal(rows.shape[0]) * rowscale[rows]
    rowptr, col, val = _csr_from_coo(m, n, rows, cols, vals)

    free = rng.random(n) < free_frac
    ub = rng.uniform(1.0, 100.0, n)
    lb = np.zeros(n)
    lb[free] = -np.inf
    ub[free] = np.inf
    xs = rng.uniform(0.0, 1.0, n) * np.where(free, 0.0, ub)
    xs[free] = rng.uniform(-50.0, 50.0, int(free.sum()))
    kx = _matvec(rowptr, col, val, xs)
    rhs = kx.copy()
    rhs[m_eq:] -= rowscale[m_eq:] * rng.uniform(0.0, 1.0, m_ineq)
    ys = rng.standard_normal(m)
    ys[m_eq:] = np.abs(ys[m_eq:])
    lam = rng.standard_normal(n)
    lam[free] = 0.0
    c = _rmatvec(rowptr, col, val, ys, n) + lam
    return LP(n, m_eq, m_ineq, rowptr, col, val, c, rhs, lb, ub,
              {"kind": "powerlaw", "seed": seed, "x_plant": xs, "rowscale": rowscale})


def large_single(seed: int = BASE_SEED + 1) -> LP:
    """Single large LP: 150k equality + 50k inequality rows, 1M variables,
    ~10M nnz (power law on [8, 5000])."""
    return powerlaw(seed, 150_000, 50_000, 1_000_000, lmin=8)


def large_mixed(seed: int = BASE_SEED + 2) -> LP:
    """The same generator at 375k + 125k rows, 2M variables, ~30M nnz."""
    return powerlaw(seed, 375_000, 125_000, 2_000_000, lmin=10)


def scaled_powerlaw(seed: int, m: int, n: int, nnz_per_col: float = 8.0) -> LP:
    """Power-law instance sized like the batched workload: 3/4 equality rows,
    row-length law solved so that nnz ~ nnz_per_col * n."""
    m_eq = (3 * m) // 4
    return powerlaw(seed, m_eq, m - m_eq, n, mean_len=nnz_per_col * n / m, discrete=False)


# --------------------------------------------------------------------------
# infeasible / unbounded variants (certificates known in closed form)
# --------------------------------------------------------------------------

def add_contradictory_rows(lp: LP, seed: int, k: int = 8, gap: float = 1.0,
                           rel_gap: float | None = None) -> LP:
    """Append two equality rows g^T x = beta and g^T x = beta + gap (g with k
    nonzeros) at the end of the equality block: primal infeasible, with the
    Farkas ray y = (-1, +1) on those two rows.  With rel_gap the gap is
    rel_gap * (1 + ||rhs||), so that the infeasibility stays visible to a
    relative KKT test on badly scaled instances."""
    if rel_gap is not None:
        gap = rel_gap * (1.0 + float(np.linalg.norm(lp.rhs)))
    rng = np.random.default_rng(seed)
    n = lp.n
    gcols = np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int32)
    gvals = rng.standard_normal(gcols.shape[0])
    xs = lp.meta.get("x_plant")
    beta = float(gvals @ xs[gcols]) if xs is not None else 0.0
    m_eq = lp.m_eq
    rp = lp.rowptr.astype(np.int64)
    split = rp[m_eq]
    col = np.concatenate([lp.col[:split], gcols, gcols, lp.col[split:]])
    val = np.concatenate([lp.val[:split], gvals, gvals, lp.val[split:]])
    kk = gcols.shape[0]
    rowptr = np.concatenate([rp[:m_eq + 1], [split + kk, split + 2 * kk], rp[m_eq + 1:] + 2 * kk])
    rhs = np.concatenate([lp.rhs[:m_eq], [beta, beta + gap], lp.rhs[m_eq:]])
    meta = dict(lp.meta)
    meta.update(kind=lp.meta.get("kind", "") + "+infeasible", infeasible_rows=(m_eq, m_eq + 1))
    return LP(n, m_eq + 2, lp.m_ineq, rowptr.astype(np.int32), col, val, lp.c.copy(), rhs,
              lp.lb.copy(), lp.ub.copy(), meta)


def add_unbounded_column(lp: LP, seed: int, k: int = 8) -> LP:
    """Append one column j with lb_j = 0, ub_j = inf, c_j = -1 and positive
    entries on k inequality rows only: x_j can grow forever, so d = e_j is an
    unbounded ray (dual infeasible).  x*_j = 0 keeps the planted point feasible."""
    rng = np.random.default_rng(seed)
    if lp.m_ineq == 0:
        raise ValueError("needs inequality rows")
    m_eq, m = lp.m_eq, lp.m
    rsel = np.sort(rng.choice(lp.m_ineq, size=min(k, lp.m_ineq), replace=False)) + m_eq
    scale = lp.meta.get("rowscale")
    v = np.abs(rng.standard_normal(rsel.shape[0])) + 0.1
    if scale is not None:
        v = v * scale[rsel]
    j = lp.n
    rp = lp.rowptr.astype(np.int64)
    rows = np.repeat(np.arange(m), np.diff(rp))
    rows = np.concatenate([rows, rsel])
    cols = np.concatenate([lp.col.astype(np.int64), np.full(rsel.shape[0], j)])
    vals = np.concatenate([lp.val, v])
    rowptr, col, val = _csr_from_coo(m, lp.n + 1, rows, cols, vals)
    meta = dict(lp.meta)
    xs = meta.get("x_plant")
    if xs is not None:
        meta["x_plant"] = np.concatenate([xs, [0.0]])
    meta.update(kind=lp.meta.get("kind", "") + "+unbounded", ray_column=j)
    return LP(lp.n + 1, m_eq, lp.m_ineq, rowptr, col, val,
              np.concatenate([lp.c, [-1.0]]), lp.rhs.copy(),
              np.concatenate([lp.lb, [0.0]]), np.concatenate([lp.ub, [np.inf]]), meta)


# --------------------------------------------------------------------------
# instances with a known optimum / special structure (oracle pins)
# --------------------------------------------------------------------------

def planted_opt(seed: int, m_eq: int = 12, m_ineq: int = 8, n: int = 30,
                density: float = 0.3) -> LP:
    """An LP whose optimal primal-dual pair (x*, y*) is planted exactly:
    x* has coordinates at the lower bound, at the upper bound and strictly
    inside; reduced costs lambda are complementary to x*; half the inequality
    rows are tight with y*_i > 0, the rest slack with y*_i = 0."""
    rng = np.random.default_rng(seed)
    m = m_eq + m_ineq
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    rows, cols, _ = _ensure_nonempty(rng, m, n, rows, cols, None)
    vals = rng.standard_normal(rows.shape[0])
    rowptr, col, val = _csr_from_coo(m, n, rows, cols, vals)
    lb = np.full(n, -1.0)
    ub = rng.uniform(1.0, 3.0, n)
    kind = rng.integers(0, 3, n)            # 0 at lb, 1 at ub, 2 interior
    xs = np.where(kind == 0, lb, np.where(kind == 1, ub, rng.uniform(-0.5, 0.5, n)))
    lam = np.where(kind == 0, rng.uniform(0.5, 2.0, n),
                   np.where(kind == 1, -rng.uniform(0.5, 2.0, n), 0.0))
    ys = rng.standard_normal(m)
    tight = np.arange(m_ineq) % 2 == 0
    ys[m_eq:] = np.where(tight, rng.uniform(0.5, 2.0, m_ineq), 0.0)
    kx = _matvec(rowptr, col, val, xs)
    rhs = kx.copy()
    rhs[m_eq:] = np.where(tight, kx[m_eq:], kx[m_eq:] - rng.uniform(0.5, 1.5, m_ineq))
    c = _rmatvec(rowptr, col, val, ys, n) + lam
    return LP(n, m_eq, m_ineq, rowptr, col, val, c, rhs, lb, ub,
              {"kind": "planted_opt", "seed": seed, "x_opt": xs, "y_opt": ys,
               "obj_opt": float(c @ xs)})


def affine(seed: int, m: int = 10, n: int = 16, density: float = 0.4) -> LP:
    """Equality rows only and all variables free: the projections vanish and
    the PDHG map is affine (the unconstrained bilinear case)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    rows, cols, _ = _ensure_nonempty(rng, m, n, rows, cols, None)
    vals = rng.standard_normal(rows.shape[0])
    rowptr, col, val = _csr_from_coo(m, n, rows, cols, vals)
    return LP(n, m, 0, rowptr, col, val, rng.standard_normal(n), rng.standard_normal(m),
              np.full(n, -np.inf), np.full(n, np.inf), {"kind": "affine", "seed": seed})


def bilinear_1d() -> LP:
    """min_{x>=0} max_y (x - 1) y as an LP: min 0 s.t. x = 1, x >= 0.
    Its unique primal-dual solution is (x, y) = (1, 0)."""
    return LP(1, 1, 0, np.array([0, 1], np.int32), np.array([0], np.int32),
              np.array([1.0]), np.array([0.0]), np.array([1.0]),
              np.array([0.0]), np.array([np.inf]), {"kind": "bilinear_1d"})


# --------------------------------------------------------------------------
# batched and serving workloads
# --------------------------------------------------------------------------

def batch_sizes(seed: int, count: int = 512, m_lo: int = 500, m_hi: int = 20000):
    """Per-instance (m_i, n_i, infeasible_i): m ~ logU[m_lo, m_hi], n = m*U(2,5),
    10% marked primal-infeasible."""
    rng = np.random.default_rng(seed)
    m = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))).astype(np.int64)
    n = np.rint(m * rng.uniform(2.0, 5.0, count)).astype(np.int64)
    infeas = rng.random(count) < 0.10
    return m, n, infeas


def batch_instance(seed: int, m: int, n: int, infeasible: bool) -> LP:
    lp = scaled_powerlaw(seed, int(m), int(n))
    if infeasible:
        lp = add_contradictory_rows(lp, seed + 7_000_000, rel_gap=0.1)
    return lp


def batch(count: int = 512, size_seed: int = BASE_SEED + 3, seed0: int = BASE_SEED + 3000,
          m_lo: int = 500, m_hi: int = 20000):
    """The batched workload: `count` power-law LPs of uneven size; instance i
    is drawn with seed seed0 + i."""
    m, n, inf = batch_sizes(size_seed, count, m_lo, m_hi)
    return [batch_instance(seed0 + i, m[i], n[i], bool(inf[i])) for i in range(count)]


@dataclass
class Request:
    t_arrival: float
    kind: str          # "small", "large", "infeasible", "unbounded"
    seed: int
    m: int
    n: int


def serving_trace(seed: int = BASE_SEED + 4, count: int = 6000, rate: float = 200.0,
                  p_large: float = 0.02, p_infeas: float = 0.05, p_unbnd: float = 0.02,
                  m_lo: int = 500, m_hi: int = 20000, large_m: int = 100_000,
                  large_n: int = 400_000):
    """Poisson arrivals at `rate` LP/s.  Kinds: 2% large (100k x 400k, ~4M nnz),
    5% primal infeasible, 2% dual infeasible, the rest batched-workload sizes."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    u = rng.random(count)
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))).astype(np.int64)
    ns = np.rint(ms * rng.uniform(2.0, 5.0, count)).astype(np.int64)
    out = []
    for i in range(count):
        if u[i] < p_large:
            kind, m, n = "large", large_m, large_n
        elif u[i] < p_large + p_infeas:
            kind, m, n = "infeasible", int(ms[i]), int(ns[i])
        elif u[i] < p_large + p_infeas + p_unbnd:
            kind, m, n = "unbounded", int(ms[i]), int(ns[i])
        else:
            kind, m, n = "small", int(ms[i]), int(ns[i])
        out.append(Request(float(t[i]), kind, seed * 1000 + i, m, n))
    return out


def request_instance(r: Request) -> LP:
    if r.kind == "large":
        return scaled_powerlaw(r.seed, r.m, r.n, nnz_per_col=10.0)
    lp = scaled_powerlaw(r.seed, r.m, r.n)
    if r.kind == "infeasible":
        lp = add_contradictory_rows(lp, r.seed + 7, rel_gap=0.1)
    elif r.kind == "unbounded":
        lp = add_unbounded_column(lp, r.seed + 7)
    return lp
