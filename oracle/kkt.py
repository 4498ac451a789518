"""Relative KKT error and Farkas-ray checks, on the ORIGINAL (unscaled) LP.

LP:  min c^T x  s.t.  A x = b,  G x >= h,  l <= x <= u,   K = [A; G], q = [b; h].
Dual sign: y_i >= 0 on inequality rows (the saddle function is
c^T x - y^T K x + q^T y).

The paper terminates on a relative KKT error no greater than the tolerance,
the same criterion as cuPDLP.jl (Section 7, "Termination criteria"), but does
not print it.  This module writes out the usual PDLP definition with l2 norms:

  r_p  = [A x - b ; min(G x - h, 0) ; x - clamp(x, l, u)]
  lam  = projection of (c - K^T y) onto Lambda, where Lambda_j is R+ if only
         l_j is finite, R- if only u_j is finite, R if both are, {0} if none
  r_d  = [(c - K^T y) - lam ; min(y_ineq, 0)]
  pobj = c^T x
  dobj = q^T y + sum_{l_j finite} l_j lam_j^+ - sum_{u_j finite} u_j lam_j^-
  relKKT = max(|r_p|/(1+|q|), |r_d|/(1+|c|), |pobj-dobj|/(1+|pobj|+|dobj|))

The bound and cone terms of r_p and r_d vanish identically at points produced
by one PDHG step, which is where the solver evaluates the error.

Infeasibility certificates follow the infimal-displacement facts of Section 5
(the primal part of v certifies dual infeasibility, the dual part certifies
primal infeasibility).  The acceptance tests are the Farkas conditions with a
relative tolerance eps:

  primal infeasible, ray y (clamped to y_ineq >= 0), g = K^T y:
      s    = sum_j (g_j > 0 ? u_j g_j : l_j g_j) over finite bounds
      viol = || (g_j)+ where u_j = inf ; (-g_j)+ where l_j = -inf ||
      accept iff q^T y - s > 0 and viol <= eps (q^T y - s)
  dual infeasible, ray d (projected onto the recession cone of the box):
      accept iff c^T d < 0 and ||A d|| + ||min(G d, 0)|| <= eps |c^T d|
"""
import numpy as np


def _csr(lp):
    import scipy.sparse as sp
    return sp.csr_matrix((lp.val, lp.col, lp.rowptr), shape=(lp.m, lp.n))


def reduced_cost_projection(r, lb, ub):
    lf = np.isfinite(lb)
    uf = np.isfinite(ub)
    lam = np.where(lf & uf, r,
          np.where(lf & ~uf, np.maximum(r, 0.0),
          np.where(~lf & uf, np.minimum(r, 0.0), 0.0)))
    return lam


def rel_kkt(lp, x, y, K=None):
    """Relative KKT error of (x, y) for `lp`.  Returns (relkkt, parts) where
    parts = dict(primal, dual, gap, pobj, dobj, rp, rd)."""
    K = _csr(lp) if K is None else K
    m_eq = lp.m_eq
    q = lp.rhs
    c = lp.c
    kx = K @ x
    rp = np.concatenate([kx[:m_eq] - q[:m_eq],
                         np.minimum(kx[m_eq:] - q[m_eq:], 0.0),
                         x - np.clip(x, lp.lb, lp.ub)])
    r = c - K.T @ y
    lam = reduced_cost_projection(r, lp.lb, lp.ub)
    rd = np.concatenate([r - lam, np.minimum(y[m_eq:], 0.0)])
    pobj = float(c @ x)
    lf = np.isfinite(lp.lb)
    uf = np.isfinite(lp.ub)
    dobj = float(q @ y
                 + np.sum(np.where(lf, lp.lb, 0.0) * np.maximum(lam, 0.0) * lf)
                 - np.sum(np.where(uf, lp.ub, 0.0) * np.maximum(-lam, 0.0) * uf))
    nrp = float(np.linalg.norm(rp))
    nrd = float(np.linalg.norm(rd))
    primal = nrp / (1.0 + float(np.linalg.norm(q)))
    dual = nrd / (1.0 + float(np.linalg.norm(c)))
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return max(primal, dual, gap), dict(primal=primal, dual=dual, gap=gap,
                                        pobj=pobj, dobj=dobj, rp=nrp, rd=nrd)


def clamp_dual_ray(lp, y):
    y = np.array(y, dtype=np.float64, copy=True)
    y[lp.m_eq:] = np.maximum(y[lp.m_eq:], 0.0)
    return y


def project_recession(lp, d):
    """Projection onto the recession cone of the box: 0 where both bounds are
    finite, >= 0 where only l is, <= 0 where only u is, free otherwise."""
    lf = np.isfinite(lp.lb)
    uf = np.isfinite(lp.ub)
    return np.where(lf & uf, 0.0,
           np.where(lf, np.maximum(d, 0.0),
           np.where(uf, np.minimum(d, 0.0), d)))


def primal_ray_check(lp, y, eps=1e-8, K=None):
    """Farkas test for primal infeasibility on the clamped ray y.
    Returns (ok, info)."""
    K = _csr(lp) if K is None else K
    y = clamp_dual_ray(lp, y)
    g = K.T @ y
    lf = np.isfinite(lp.lb)
    uf = np.isfinite(lp.ub)
    pos = g > 0
    s = float(np.sum(np.where(pos & uf, np.where(uf, lp.ub, 0.0) * g, 0.0))
              + np.sum(np.where(~pos & lf, np.where(lf, lp.lb, 0.0) * g, 0.0)))
    viol_v = np.where(pos & ~uf, g, 0.0) + np.where((g < 0) & ~lf, -g, 0.0)
    viol = float(np.linalg.norm(viol_v))
    qy = float(lp.rhs @ y)
    margin = qy - s
    ok = bool(margin > 0.0 and viol <= eps * margin)
    return ok, dict(qy=qy, s=s, margin=margin, viol=viol, ray=y)


def dual_ray_check(lp, d, eps=1e-8, K=None):
    """Test for dual infeasibility (an unbounded primal ray) on the projected
    ray d.  Returns (ok, info)."""
    K = _csr(lp) if K is None else K
    d = project_recession(lp, np.asarray(d, dtype=np.float64))
    kd = K @ d
    cd = float(lp.c @ d)
    res = float(np.linalg.norm(kd[:lp.m_eq]) + np.linalg.norm(np.minimum(kd[lp.m_eq:], 0.0)))
    ok = bool(cd < 0.0 and res <= eps * abs(cd))
    return ok, dict(cd=cd, res=res, ray=d)
