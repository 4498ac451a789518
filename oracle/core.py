"""Restarted Halpern PDHG (rHPDHG) and its reflected variant (r2HPDHG), FP64.

Paper: H. Lu and J. Yang, "Restarted Halpern PDHG for Linear Programming",
arXiv 2407.16144.  Where the paper fixes a step it is cited; where it defers
to cuPDLP or is silent, the reading used here is stated in the docstring.

Problem (generalising the standard form of Section 2, eq. (lp)/(minmax)):

    min_{x in X} max_{y in Y}  c^T x - y^T K x + q^T y
    X = {l <= x <= u},  Y = {y : y_i >= 0 on inequality rows},  K = [A; G].

With G empty, l = 0 and u = inf this is the paper's saddle problem with
y = -y_paper; the sign flip makes y_ineq >= 0 and keeps the usual PDLP
convention.  Everything below runs on the diagonally rescaled problem
K~ = D_r K D_c, c~ = D_c c, q~ = D_r q, l~ = l / D_c, u~ = u / D_c; solutions
are mapped back with x = D_c x~, y = D_r y~.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

from .kkt import rel_kkt, primal_ray_check, dual_ray_check
from .rng import uniform_pm1

OPTIMAL, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, ITER_LIMIT, TIME_LIMIT, NUMERICAL = 1, 2, 3, 4, 5, 6
STATUS_NAMES = {0: "UNSOLVED", 1: "OPTIMAL", 2: "PRIMAL_INFEASIBLE", 3: "DUAL_INFEASIBLE",
                4: "ITER_LIMIT", 5: "TIME_LIMIT", 6: "NUMERICAL"}


def to_csr(lp) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(lp.val, np.float64), np.asarray(lp.col),
                          np.asarray(lp.rowptr)), shape=(lp.m, lp.n))


# --------------------------------------------------------------------------
# preprocessing: Ruiz equilibration + Pock-Chambolle scaling
# --------------------------------------------------------------------------

def _row_ids(K):
    return np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))


def scale(K: sp.csr_matrix, ruiz_iters: int = 10, pc_alpha: float | None = 1.0):
    """Diagonal preconditioning "as cuPDLP" (Section 7, algorithmic
    enhancements; the paper prints no details).  Reading: `ruiz_iters` passes
    of Ruiz infinity-norm equilibration, r_i = sqrt(max_j |K_ij|),
    c_j = sqrt(max_i |K_ij|), followed by one Pock-Chambolle pass with
    r_i = sqrt(sum_j |K_ij|^(2-alpha)), c_j = sqrt(sum_i |K_ij|^alpha).  Each
    pass divides entry (i, j) by r_i and then by c_j.  An empty row or column
    gets the factor 1.  Returns (K~, D_r, D_c) with K~ = D_r K D_c."""
    Kt = sp.csr_matrix(K, dtype=np.float64, copy=True)
    Kt.sort_indices()
    m, n = Kt.shape
    rows = _row_ids(Kt)
    Dr = np.ones(m)
    Dc = np.ones(n)

    def apply(r, cfac):
        nonlocal Dr, Dc
        r = np.where(r > 0.0, r, 1.0)
        cfac = np.where(cfac > 0.0, cfac, 1.0)
        Kt.data = Kt.data / r[rows] / cfac[Kt.indices]
        Dr = Dr / r
        Dc = Dc / cfac

    for _ in range(ruiz_iters):
        a = np.abs(Kt.data)
        rmax = np.zeros(m)
        np.maximum.at(rmax, rows, a)
        cmax = np.zeros(n)
        np.maximum.at(cmax, Kt.indices, a)
        apply(np.sqrt(rmax), np.sqrt(cmax))
    if pc_alpha is not None:
        a = np.abs(Kt.data)
        rs = np.bincount(rows, weights=a ** (2.0 - pc_alpha), minlength=m)
        cs = np.bincount(Kt.indices, weights=a ** pc_alpha, minlength=n)
        apply(np.sqrt(rs), np.sqrt(cs))
    return Kt, Dr, Dc


def power_iteration(K: sp.csr_matrix, seed: int, max_iters: int = 1000, min_iters: int = 20,
                    rtol: float = 1e-4):
    """Estimate ||K||_2 by power iteration on K^T K.  The paper's theory takes a
    constant step eta <= 1/(2||A||_2) (Section 1.2 notation); the estimate
    sigma_t = sqrt(||K^T K v_{t-1}||) with unit v is what the constant step is
    built from.  Start: SplitMix64 uniform vector, normalised.  Stop at the
    first t >= min_iters with |sigma_t - sigma_{t-1}| <= rtol * sigma_t, or at
    max_iters.  Returns (sigma_hat, iterations)."""
    n = K.shape[1]
    v = uniform_pm1(seed, n)
    v = v / np.linalg.norm(v)
    KT = K.T.tocsr()
    prev = None
    s = 0.0
    for t in range(1, max_iters + 1):
        w = KT @ (K @ v)
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return 0.0, t
        s = math.sqrt(nw)
        v = w / nw
        if prev is not None and t >= min_iters and abs(s - prev) <= rtol * s:
            return s, t
        prev = s
    return s, max_iters


@dataclass
class ScaledLP:
    K: sp.csr_matrix          # K~
    KT: sp.csr_matrix         # (K~)^T, explicit
    c: np.ndarray
    q: np.ndarray
    l: np.ndarray
    u: np.ndarray
    Dr: np.ndarray
    Dc: np.ndarray
    m_eq: int


def scaled_problem(lp, ruiz_iters=10, pc_alpha=1.0) -> ScaledLP:
    K = to_csr(lp)
    Kt, Dr, Dc = scale(K, ruiz_iters, pc_alpha)
    return ScaledLP(Kt, Kt.T.tocsr(), Dc * lp.c, Dr * lp.rhs, lp.lb / Dc, lp.ub / Dc,
                    Dr, Dc, lp.m_eq)


# --------------------------------------------------------------------------
# the PDHG operator, its norm, and the Halpern step
# --------------------------------------------------------------------------

def proj_Y(P: ScaledLP, v):
    out = np.array(v, dtype=np.float64, copy=True)
    out[P.m_eq:] = np.maximum(out[P.m_eq:], 0.0)
    return out


def pdhg_T(P: ScaledLP, x, y, tau, sigma):
    """One PDHG step z -> T(z) (Section 2, eq. (pdhg), in the sign above):
        x+ = proj_X(x - tau (c - K^T y))
        y+ = proj_Y(y + sigma (q - K (2 x+ - x)))"""
    xp = np.clip(x - tau * (P.c - P.KT @ y), P.l, P.u)
    yp = proj_Y(P, y + sigma * (P.q - P.K @ (2.0 * xp - x)))
    return xp, yp


def m_norm(P: ScaledLP, dx, dy, tau, sigma):
    """||(dx, dy)||_M with M = [[I/tau, K^T], [K, I/sigma]]: the PDHG norm of
    Section 1.2 with the square root restored, tau = eta/omega and
    sigma = eta*omega, and the off-diagonal sign that goes with y = -y_paper."""
    with np.errstate(all="ignore"):   # IEEE results (inf, nan) instead of exceptions
        v = (np.float64(dx @ dx) / np.float64(tau) + np.float64(dy @ dy) / np.float64(sigma)
             + 2.0 * np.float64(dy @ (P.K @ dx)))
        return float(np.sqrt(np.maximum(v, 0.0))) if not np.isnan(v) else float("nan")


class _Activity:
    """Two-stage diagnostics (Section 4: identification, then local
    convergence): at each check, the activity of T(z) = (x+, y+) -- each x+_j
    at its lower bound (1), at its upper bound (2) or inside (0), each
    inequality row's y+_i at zero (1) or not (0) -- compared with the
    previous check's.  The first check only records."""

    def __init__(self):
        self.prev = None
        self.changes = 0
        self.ident = 0

    def update(self, P, m_eq, xp, yp, t):
        ax = np.where(np.isfinite(P.l) & (xp == P.l), 1, np.where(np.isfinite(P.u) & (xp == P.u), 2, 0))
        ay = np.zeros(yp.shape[0], dtype=np.int64)
        ay[m_eq:] = (yp[m_eq:] == 0.0)
        if self.prev is not None:
            self.changes = int(np.count_nonzero(ax != self.prev[0]) + np.count_nonzero(ay != self.prev[1]))
            if self.changes > 0:
                self.ident = t
        self.prev = (ax, ay)
        return self.changes


def halpern_point(xp, yp, x, y, x0, y0, k, reflect):
    """Halpern step (eq. (hpdhg)) or reflected Halpern step (eq. (hrpdhg)):
    z^{k+1} = (k+1)/(k+2) * That + 1/(k+2) * z^0, with That = T(z^k) or
    2 T(z^k) - z^k."""
    w = (k + 1.0) / (k + 2.0)
    if reflect:
        xh, yh = 2.0 * xp - x, 2.0 * yp - y
    else:
        xh, yh = xp, yp
    return w * xh + (1.0 - w) * x0, w * yh + (1.0 - w) * y0


# --------------------------------------------------------------------------
# the restarted solver
# --------------------------------------------------------------------------

@dataclass
class Options:
    method: str = "r2hpdhg"          # "rhpdhg" (Algorithm 1), "r2hpdhg" (Algorithm 2) or "rapdhg"
    tol: float = 1e-8                # relative KKT tolerance
    max_iter: int = 1_000_000        # enforced at check points: stop at the first check with t >= max_iter
    ruiz_iters: int = 10
    pc_alpha: float | None = 1.0
    check_every: int = 64            # C: restart/termination checks at k % C == 0, k > 0
    restart: str = "adaptive"        # "adaptive" (eq. (adaptive-restart)), "fixed", "none"
    fixed_restart_len: int = 0       # k* for restart == "fixed" (eq. (fixed-restart))
    restart_beta: float = math.exp(-1.0)
    avg_beta_sufficient: float = 0.2  # rapdhg: KKT-based restart thresholds (cuPDLP's values)
    avg_beta_necessary: float = 0.8
    artificial_restart: float = 0.36  # also restart when k >= this * t (0 disables)
    step_safety: float = 0.9
    power_max_iters: int = 1000
    power_min_iters: int = 20
    power_rtol: float = 1e-4
    eps_infeas: float = 1e-8
    primal_weight: bool = True
    seed: int = 0
    eta: float | None = None         # fixes the step size (skips the power iteration)
    omega0: float | None = None      # fixes the initial primal weight
    callback: object = None          # called every iteration with a dict of the state


@dataclass
class Result:
    status: int
    x: np.ndarray
    y: np.ndarray
    iters: int
    restarts: int
    kkt: float
    pobj: float
    dobj: float
    kkt_parts: dict
    omega: float
    eta: float
    sigma_hat: float
    power_iters: int
    ray: np.ndarray | None = None
    log: list = field(default_factory=list)
    scaled: ScaledLP | None = None
    active_changes: int = 0   # activity changes between the last two checks
    ident_iters: int = 0      # iterations at the last check with an activity change


def solve(lp, opts: Options | None = None) -> Result:
    """Restarted (reflected) Halpern PDHG, Algorithms 1 and 2 with the adaptive
    restart rule eq. (adaptive-restart).

    Readings where the paper defers to cuPDLP or is silent:
      * start z^{0,0} = (proj_X(0), 0); one iteration = one evaluation of T;
      * step eta = step_safety / sigma_hat with sigma_hat from power_iteration;
      * primal weight omega: omega_0 = ||c~||/||q~|| (1 if either is <= 1e-10);
        at each restart omega <- exp(0.5 ln(dy/dx) + 0.5 ln omega) with dx, dy
        the l2 distances between consecutive restart points (skipped if either
        is <= 1e-10); tau = eta/omega, sigma = eta*omega; omega is constant
        within an epoch;
      * r0 = ||z^{n,0} - T(z^{n,0})||_M is taken at the first step of each
        epoch with that epoch's tau and sigma;
      * restart, termination and infeasibility are evaluated only when k > 0
        and k % C == 0, at the candidate T(z^{n,k}); the first epoch restarts
        at its first check (tau^0 = C - 1); for n >= 1 the restart test is
        ||z - T(z)||_M <= beta * r0 with beta = 1/e;
      * cuPDLP's "artificial" restart is kept as well: restart when the epoch
        has run k >= 0.36 t of the t evaluations so far.  On an infeasible LP
        both sides of the residual test tend to the norm of the infimal
        displacement vector, so without it restarts stop and the ray
        candidates converge only sublinearly (Section 5);
      * the restart point is T(z^{n,k}) for both methods (Algorithms 1, 2);
      * order at a check: optimal (relative KKT at the candidate, unscaled),
        primal infeasible (rays T(z)-z, then z-z^{n,0}), dual infeasible
        (same rays), iteration limit, restart.
    """
    opts = opts or Options()
    reflect = opts.method == "r2hpdhg"
    K0 = to_csr(lp)
    P = scaled_problem(lp, opts.ruiz_iters, opts.pc_alpha)
    if opts.eta is not None:
        eta, sigma_hat, piters = float(opts.eta), float("nan"), 0
    else:
        sigma_hat, piters = power_iteration(P.K, opts.seed, opts.power_max_iters,
                                            opts.power_min_iters, opts.power_rtol)
        eta = opts.step_safety / sigma_hat if sigma_hat > 0.0 else opts.step_safety
    if opts.omega0 is not None:
        omega = float(opts.omega0)
    elif opts.primal_weight:
        nc, nq = float(np.linalg.norm(P.c)), float(np.linalg.norm(P.q))
        omega = nc / nq if (nc > 1e-10 and nq > 1e-10) else 1.0
    else:
        omega = 1.0
    tau, sigma = eta / omega, eta * omega

    m, n = lp.m, lp.n
    x = np.clip(np.zeros(n), P.l, P.u)
    y = np.zeros(m)
    x0, y0 = x.copy(), y.copy()
    nrest, k, t = 0, 0, 0
    r0 = float("nan")
    C = opts.check_every
    log = []

    act = _Activity()

    def finish(status, xp, yp, ray=None):
        xu, yu = P.Dc * xp, P.Dr * yp
        kkt, parts = rel_kkt(lp, xu, yu, K0)
        return Result(status, xu, yu, t, nrest, kkt, parts["pobj"], parts["dobj"], parts,
                      omega, eta, sigma_hat, piters, ray, log, P, act.changes, act.ident)

    if opts.method == "rapdhg":
        return _solve_average(lp, opts, P, K0, eta, sigma_hat, piters, omega, x, y)

    while True:
        xp, yp = pdhg_T(P, x, y, tau, sigma)
        t += 1
        if k == 0:
            r0 = m_norm(P, x - xp, y - yp, tau, sigma)
        if opts.callback is not None:
            opts.callback(dict(t=t, n=nrest, k=k, x=x, y=y, xp=xp, yp=yp, x0=x0, y0=y0,
                               tau=tau, sigma=sigma, P=P))
        if k > 0 and k % C == 0:
            res = m_norm(P, x - xp, y - yp, tau, sigma)
            xu, yu = P.Dc * xp, P.Dr * yp
            kkt, parts = rel_kkt(lp, xu, yu, K0)
            entry = dict(t=t, n=nrest, k=k, kkt=kkt, resid=res, r0=r0, restart=False,
                         margin=abs(res - opts.restart_beta * r0) / r0 if r0 > 0 else float("inf"),
                         active_changes=act.update(P, lp.m_eq, xp, yp, t))
            log.append(entry)
            if not all(np.isfinite(v) for v in (kkt, res, parts["primal"], parts["dual"], parts["gap"])):
                return finish(NUMERICAL, xp, yp)
            if kkt <= opts.tol:
                return finish(OPTIMAL, xp, yp)
            cands = [(xp - x, yp - y), (x - x0, y - y0)]
            for _, dy in cands:
                ok, info = primal_ray_check(lp, P.Dr * dy, opts.eps_infeas, K0)
                if ok:
                    return finish(PRIMAL_INFEASIBLE, xp, yp, info["ray"])
            for dx, _ in cands:
                ok, info = dual_ray_check(lp, P.Dc * dx, opts.eps_infeas, K0)
                if ok:
                    return finish(DUAL_INFEASIBLE, xp, yp, info["ray"])
            if t >= opts.max_iter:
                return finish(ITER_LIMIT, xp, yp)
            if opts.restart == "adaptive":
                do_restart = ((nrest == 0) or (res <= opts.restart_beta * r0)
                              or (opts.artificial_restart > 0 and k >= opts.artificial_restart * t))
            elif opts.restart == "fixed":
                do_restart = k >= opts.fixed_restart_len
            else:
                do_restart = False
            if do_restart:
                entry["restart"] = True
                dxn = float(np.linalg.norm(xp - x0))
                dyn = float(np.linalg.norm(yp - y0))
                if (opts.primal_weight and dxn > 1e-10 and dyn > 1e-10
                        and math.isfinite(dxn) and math.isfinite(dyn)):
                    omega = math.exp(0.5 * math.log(dyn / dxn) + 0.5 * math.log(omega))
                tau, sigma = eta / omega, eta * omega
                x0, y0 = xp.copy(), yp.copy()
                x, y = xp, yp
                nrest += 1
                k = 0
                continue
        x, y = halpern_point(xp, yp, x, y, x0, y0, k, reflect)
        k += 1


def _solve_average(lp, opts, P, K0, eta, sigma_hat, piters, omega, x, y) -> Result:
    """Restarted average PDHG (raPDHG, the base algorithm of PDLP/cuPDLP that
    the paper compares with, Section 2 and Section 7).  The paper describes it
    only as: run vanilla PDHG (eq. (pdhg)) within an epoch and restart at the
    average of the epoch's iterates, with cuPDLP's KKT-based adaptive restart.
    Readings:
      * average (as in Proposition 1): zbar^{n,k} = (1/(k+1)) sum_{i=0}^{k}
        z^{n,i}, the epoch's start included; at the check after the T
        evaluation of inner step k the candidate is zbar^{n,k+1};
      * checks at k > 0, k % C == 0 as for rHPDHG; termination and the
        iteration limit are tested at the candidate, the infeasibility tests on
        the same rays as rHPDHG (T(z) - z and z - z^{n,0}, z the current
        vanilla iterate);
      * restart metric: the relative KKT error at the candidate.  The first
        epoch restarts at its first check; later epochs restart when
        KKT(cand) <= 0.2 KKT(z^{n,0}), or KKT(cand) <= 0.8 KKT(z^{n,0}) and
        KKT(cand) > KKT at the epoch's previous check, or k >= 0.36 t
        (cuPDLP's sufficient / necessary + no-progress / artificial rules);
        restart_mode "fixed" and "none" as for rHPDHG;
      * restart point: the candidate (the average); primal weight update as
        for rHPDHG with the distance between consecutive restart points."""
    tau, sigma = eta / omega, eta * omega
    x0, y0 = x.copy(), y.copy()
    sx, sy = x.copy(), y.copy()      # sums of the epoch's iterates z^{n,0..k}
    cnt = 1
    nrest, k, t = 0, 0, 0
    kkt_anchor, kkt_prev = float("nan"), float("inf")
    C = opts.check_every
    log = []

    act = _Activity()

    def finish(status, xc, yc, ray=None):
        xu, yu = P.Dc * xc, P.Dr * yc
        kkt, parts = rel_kkt(lp, xu, yu, K0)
        return Result(status, xu, yu, t, nrest, kkt, parts["pobj"], parts["dobj"], parts,
                      omega, eta, sigma_hat, piters, ray, log, P, act.changes, act.ident)

    while True:
        xp, yp = pdhg_T(P, x, y, tau, sigma)
        t += 1
        sx = sx + xp
        sy = sy + yp
        cnt += 1
        if opts.callback is not None:
            opts.callback(dict(t=t, n=nrest, k=k, x=x, y=y, xp=xp, yp=yp, x0=x0, y0=y0,
                               xa=sx / cnt, ya=sy / cnt, tau=tau, sigma=sigma, P=P))
        if k > 0 and k % C == 0:
            xa, ya = sx / cnt, sy / cnt
            kkt, parts = rel_kkt(lp, P.Dc * xa, P.Dr * ya, K0)
            thr = [b * kkt_anchor for b in (opts.avg_beta_sufficient, opts.avg_beta_necessary)] + [kkt_prev]
            thr = [v for v in thr if math.isfinite(v) and v > 0.0]
            entry = dict(t=t, n=nrest, k=k, kkt=kkt, kkt_anchor=kkt_anchor, kkt_prev=kkt_prev,
                         restart=False,
                         margin=min((abs(kkt - v) / v for v in thr), default=float("inf")),
                         active_changes=act.update(P, lp.m_eq, xp, yp, t))
            log.append(entry)
            if not all(np.isfinite(v) for v in (kkt, parts["primal"], parts["dual"], parts["gap"])):
                return finish(NUMERICAL, xa, ya)
            if kkt <= opts.tol:
                return finish(OPTIMAL, xa, ya)
            cands = [(xp - x, yp - y), (x - x0, y - y0)]
            for _, dy in cands:
                ok, info = primal_ray_check(lp, P.Dr * dy, opts.eps_infeas, K0)
                if ok:
                    return finish(PRIMAL_INFEASIBLE, xa, ya, info["ray"])
            for dx, _ in cands:
                ok, info = dual_ray_check(lp, P.Dc * dx, opts.eps_infeas, K0)
                if ok:
                    return finish(DUAL_INFEASIBLE, xa, ya, info["ray"])
            if t >= opts.max_iter:
                return finish(ITER_LIMIT, xa, ya)
            if opts.restart == "adaptive":
                do_restart = ((nrest == 0) or (kkt <= opts.avg_beta_sufficient * kkt_anchor)
                              or (kkt <= opts.avg_beta_necessary * kkt_anchor and kkt > kkt_prev)
                              or (opts.artificial_restart > 0 and k >= opts.artificial_restart * t))
            elif opts.restart == "fixed":
                do_restart = k >= opts.fixed_restart_len
            else:
                do_restart = False
            kkt_prev = kkt
            if do_restart:
                entry["restart"] = True
                dxn = float(np.linalg.norm(xa - x0))
                dyn = float(np.linalg.norm(ya - y0))
                if (opts.primal_weight and dxn > 1e-10 and dyn > 1e-10
                        and math.isfinite(dxn) and math.isfinite(dyn)):
                    omega = math.exp(0.5 * math.log(dyn / dxn) + 0.5 * math.log(omega))
                tau, sigma = eta / omega, eta * omega
                x0, y0 = xa.copy(), ya.copy()
                x, y = xa, ya
                sx, sy = xa.copy(), ya.copy()
                cnt = 1
                kkt_anchor, kkt_prev = kkt, float("inf")
                nrest += 1
                k = 0
                continue
        x, y = xp, yp
        k += 1
