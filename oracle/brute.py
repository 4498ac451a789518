"""Brute-force vertex enumeration for tiny LPs with every variable boxed.

With all bounds finite the feasible set is a polytope, so if it is nonempty
the minimum of c^T x is attained at a vertex.  A vertex is a feasible point at
which n linearly independent constraints are active, all equalities among
them.  Enumerate every choice of (n - m_eq) active constraints from the
inequality rows and the 2n bounds, solve the square system, keep the
feasible solutions and return the best objective.
"""
import itertools

import numpy as np


def vertex_enumeration(lp, feas_tol=1e-9):
    """Returns (best_obj, best_x) or (None, None) if infeasible."""
    if not (np.all(np.isfinite(lp.lb)) and np.all(np.isfinite(lp.ub))):
        raise ValueError("vertex enumeration needs a bounded box")
    n, m_eq = lp.n, lp.m_eq
    Kd = np.zeros((lp.m, n))
    for i in range(lp.m):
        for p in range(lp.rowptr[i], lp.rowptr[i + 1]):
            Kd[i, lp.col[p]] += lp.val[p]
    A, b = Kd[:m_eq], lp.rhs[:m_eq]
    G, h = Kd[m_eq:], lp.rhs[m_eq:]
    I = np.eye(n)
    # inequality constraints written as (row, rhs) with the active form row.x = rhs
    ineq_rows = [G[i] for i in range(G.shape[0])] + [I[j] for j in range(n)] + [I[j] for j in range(n)]
    ineq_rhs = list(h) + list(lp.lb) + list(lp.ub)
    need = n - m_eq
    best, best_x = None, None
    for S in itertools.combinations(range(len(ineq_rows)), need):
        M = np.vstack([A] + [ineq_rows[s][None, :] for s in S]) if need > 0 else A
        r = np.concatenate([b, [ineq_rhs[s] for s in S]])
        if np.linalg.matrix_rank(M) < n:
            continue
        x = np.linalg.solve(M, r)
        scale = 1.0 + np.max(np.abs(x))
        if np.max(np.abs(A @ x - b), initial=0.0) > feas_tol * scale:
            continue
        if np.min(G @ x - h, initial=0.0) < -feas_tol * scale:
            continue
        if np.any(x < lp.lb - feas_tol * scale) or np.any(x > lp.ub + feas_tol * scale):
            continue
        obj = float(lp.c @ x)
        if best is None or obj < best:
            best, best_x = obj, x
    return best, best_x
