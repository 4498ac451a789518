"""Pins for the CPU oracle: each test checks it against something other than
itself -- a value fixed by the paper or by mathematics, a library routine
(SVD, HiGHS), brute force, or a hand-derived fixture under tests/golden/."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import lpgen
import oracle
from oracle import core

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lp_from_dict(d):
    f = lambda a: np.array([float(v) for v in a])
    return lpgen.LP(d["n"], d["m_eq"], d["m_ineq"], np.array(d["rowptr"], np.int32),
                    np.array(d["col"], np.int32), f(d["val"]), f(d["c"]), f(d["rhs"]),
                    f(d["lb"]), f(d["ub"]))


def _dense(lp):
    return oracle.to_csr(lp).toarray()


def _highs(lp):
    K = _dense(lp)
    me = lp.m_eq
    kw = {}
    if me:
        kw.update(A_eq=K[:me], b_eq=lp.rhs[:me])
    if lp.m_ineq:
        kw.update(A_ub=-K[me:], b_ub=-lp.rhs[me:])
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
              for a, b in zip(lp.lb, lp.ub)]
    return linprog(lp.c, bounds=bounds, method="highs", **kw)


# ---------------------------------------------------------------- generator of the start vector

def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    a = g["cases"][0]
    assert [int(v) for v in oracle.splitmix64(a["seed"], 3)] == [int(h, 16) for h in a["outputs"]]
    b = g["cases"][1]
    assert [int(v) for v in oracle.splitmix64(b["seed"], 3)] == b["outputs_decimal"]
    u = oracle.uniform_pm1(7, 10000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.03


# ---------------------------------------------------------------- relative KKT evaluator

@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "kkt_cases.json")))["cases"],
                         ids=lambda c: c["name"])
def test_rel_kkt_hand_derived(case):
    lp = _lp_from_dict(case["lp"])
    kkt, parts = oracle.rel_kkt(lp, np.array(case["x"], float), np.array(case["y"], float))
    for key, val in case["expect"].items():
        assert parts[key] == pytest.approx(val, abs=1e-15), key
    assert kkt == pytest.approx(max(case["expect"]["primal"], case["expect"]["dual"],
                                    case["expect"]["gap"]), abs=1e-15)


def test_rel_kkt_vanishes_at_highs_solution():
    """HiGHS' primal solution and marginals (y_eq = eqlin marginals,
    y_ineq = -ineqlin marginals for G x >= h written as -G x <= -h) satisfy the
    KKT system, so the evaluator must report ~0 there."""
    lp = lpgen.tiny(11)
    res = _highs(lp)
    assert res.status == 0
    y = np.concatenate([res.eqlin.marginals, -res.ineqlin.marginals])
    kkt, parts = oracle.rel_kkt(lp, res.x, y)
    assert kkt < 1e-7, parts
    # a perturbed point is not optimal
    kkt2, _ = oracle.rel_kkt(lp, res.x, 1.1 * y)
    assert kkt2 > 1e-4


# ---------------------------------------------------------------- scaling and step size

def test_ruiz_equilibrates_scaled_permutation_in_one_pass():
    rng = np.random.default_rng(0)
    n = 9
    perm = rng.permutation(n)
    a = 10.0 ** rng.uniform(-3, 3, n)
    b = 10.0 ** rng.uniform(-3, 3, n)
    sign = rng.choice([-1.0, 1.0], n)
    K = sp.csr_matrix((a * b[perm] * sign, (np.arange(n), perm)), shape=(n, n))
    Kt, Dr, Dc = oracle.scale(K, ruiz_iters=1, pc_alpha=None)
    assert np.allclose(np.abs(Kt.data), 1.0, rtol=1e-14)
    # scaling vectors reproduce the scaled matrix: K~ = D_r K D_c
    assert np.allclose((sp.diags(Dr) @ K @ sp.diags(Dc)).toarray(), Kt.toarray(), rtol=1e-14)


def test_ruiz_converges_to_unit_row_and_column_maxima():
    lp = lpgen.powerlaw(3, 30, 10, 80, lmin=2, lmax=40)
    Kt, _, _ = oracle.scale(oracle.to_csr(lp), ruiz_iters=40, pc_alpha=None)
    A = np.abs(Kt.toarray())
    assert np.allclose(A.max(axis=1), 1.0, atol=1e-6)
    assert np.allclose(A.max(axis=0), 1.0, atol=1e-6)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pock_chambolle_bounds_spectral_norm(seed):
    """Pock-Chambolle with alpha = 1 gives ||K~||_2 <= 1 (Schur test)."""
    lp = lpgen.powerlaw(seed, 40, 20, 100, lmin=2, lmax=60)
    Kt, Dr, Dc = oracle.scale(oracle.to_csr(lp))
    s = np.linalg.svd(Kt.toarray(), compute_uv=False)[0]
    assert s <= 1.0 + 1e-12
    assert np.allclose((sp.diags(Dr) @ oracle.to_csr(lp) @ sp.diags(Dc)).toarray(), Kt.toarray(),
                       rtol=1e-12, atol=0)


def test_power_iteration_matches_svd():
    K = sp.csr_matrix(np.diag([3.0, 2.0, 1.0, 0.5]))
    s, it = oracle.power_iteration(K, seed=5, rtol=1e-10, max_iters=2000)
    assert s == pytest.approx(3.0, rel=1e-8)
    lp = lpgen.tiny(4)
    P = core.scaled_problem(lp)
    s, it = oracle.power_iteration(P.K, seed=0)
    smax = np.linalg.svd(P.K.toarray(), compute_uv=False)[0]
    assert 20 <= it <= 1000
    assert s <= smax * (1 + 1e-12) and s >= smax * (1 - 1e-3)


# ---------------------------------------------------------------- the PDHG operator

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_T_fixes_planted_optimum(seed):
    """Fixed points of T are exactly the saddle points (Section 3, used in the
    proof of Proposition 2): T(z*) = z* for a planted optimal pair."""
    lp = lpgen.planted_opt(seed)
    P = core.scaled_problem(lp)
    xs = lp.meta["x_opt"] / P.Dc
    ys = lp.meta["y_opt"] / P.Dr
    for tau, sigma in [(0.3, 0.7), (1.1, 0.2)]:
        xp, yp = oracle.pdhg_T(P, xs, ys, tau, sigma)
        assert np.allclose(xp, xs, rtol=0, atol=1e-12 * (1 + np.abs(xs).max()))
        assert np.allclose(yp, ys, rtol=0, atol=1e-12 * (1 + np.abs(ys).max()))
    # the planted pair is optimal: HiGHS agrees on the objective
    res = _highs(lp)
    assert res.fun == pytest.approx(lp.meta["obj_opt"], rel=1e-9, abs=1e-9)


def test_T_residual_is_subgradient_at_T():
    """M (z - T z) lies in F(T z) (proof of Proposition 2):
    x-part = c - K^T y+ on coordinates strictly inside the box, <= at l, >= at u;
    y-part = K x+ - q on equality rows and on inequality rows with y+ > 0, and
    <= there when y+ = 0."""
    lp = lpgen.planted_opt(5, m_eq=10, m_ineq=10, n=25)
    P = core.scaled_problem(lp)
    rng = np.random.default_rng(1)
    tau, sigma = 0.4, 0.9
    for _ in range(5):
        x = rng.normal(size=lp.n) * 2
        y = rng.normal(size=lp.m) * 2
        xp, yp = oracle.pdhg_T(P, x, y, tau, sigma)
        dx, dy = x - xp, y - yp
        gx = dx / tau + P.KT @ dy
        gy = P.K @ dx + dy / sigma
        fx = P.c - P.KT @ yp
        fy = P.K @ xp - P.q
        inside = (xp > P.l) & (xp < P.u)
        atl = xp == P.l
        atu = xp == P.u
        tol = 1e-12 * (1 + np.abs(gx).max() + np.abs(fx).max())
        assert np.all(np.abs(gx - fx)[inside] <= tol)
        assert np.all((gx - fx)[atl & ~atu] <= tol)
        assert np.all((gx - fx)[atu & ~atl] >= -tol)
        me = lp.m_eq
        toly = 1e-12 * (1 + np.abs(gy).max() + np.abs(fy).max())
        act = np.ones(lp.m, bool)
        act[me:] = yp[me:] > 0
        assert np.all(np.abs(gy - fy)[act] <= toly)
        assert np.all((gy - fy)[~act] <= toly)


def _mdot(P, a, b, tau, sigma):
    (ax, ay), (bx, by) = a, b
    return ax @ bx / tau + ay @ by / sigma + ay @ (P.K @ bx) + by @ (P.K @ ax)


def test_T_firmly_nonexpansive_and_reflection_nonexpansive():
    """T is firmly nonexpansive in the PDHG norm and 2T - I is nonexpansive
    (Section 6, the reflected-operator proposition)."""
    lp = lpgen.tiny(9)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    eta = 0.9 / s
    rng = np.random.default_rng(2)
    for omega in [1.0, 3.0, 0.2]:
        tau, sigma = eta / omega, eta * omega
        for _ in range(10):
            z1 = (rng.normal(size=lp.n) * 5, rng.normal(size=lp.m) * 5)
            z2 = (rng.normal(size=lp.n) * 5, rng.normal(size=lp.m) * 5)
            t1 = oracle.pdhg_T(P, *z1, tau, sigma)
            t2 = oracle.pdhg_T(P, *z2, tau, sigma)
            dT = (t1[0] - t2[0], t1[1] - t2[1])
            dz = (z1[0] - z2[0], z1[1] - z2[1])
            lhs = _mdot(P, dT, dT, tau, sigma)
            rhs = _mdot(P, dT, dz, tau, sigma)
            assert lhs <= rhs * (1 + 1e-10) + 1e-10
            dR = (2 * dT[0] - dz[0], 2 * dT[1] - dz[1])
            assert _mdot(P, dR, dR, tau, sigma) <= _mdot(P, dz, dz, tau, sigma) * (1 + 1e-10)


# ---------------------------------------------------------------- Halpern weights

@pytest.mark.parametrize("reflect", [False, True])
def test_halpern_equals_average_on_affine_problem(reflect):
    """Proposition 1: on the unconstrained bilinear problem the Halpern
    iterates equal the running average of the plain iterates of the same
    (affine) map -- T for Halpern PDHG, 2T - I for the reflected variant."""
    lp = lpgen.affine(3)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    tau = sigma = 0.8 / s
    z0 = (np.random.default_rng(0).normal(size=lp.n), np.random.default_rng(1).normal(size=lp.m))

    def S(x, y):
        xp, yp = oracle.pdhg_T(P, x, y, tau, sigma)
        return (2 * xp - x, 2 * yp - y) if reflect else (xp, yp)

    x, y = z0
    plain = z0
    sx, sy = z0[0].copy(), z0[1].copy()
    for k in range(200):
        xp, yp = oracle.pdhg_T(P, x, y, tau, sigma)
        x, y = oracle.halpern_point(xp, yp, x, y, z0[0], z0[1], k, reflect)
        plain = S(*plain)
        sx += plain[0]
        sy += plain[1]
        ax, ay = sx / (k + 2), sy / (k + 2)
        scale = 1 + np.abs(ax).max() + np.abs(ay).max()
        assert np.abs(x - ax).max() <= 1e-12 * scale
        assert np.abs(y - ay).max() <= 1e-12 * scale


def test_reflected_first_step_is_T():
    """eq. (hrpdhg) with k = 0: (1/2)(2T(z) - z) + (1/2) z = T(z)."""
    lp = lpgen.tiny(2)
    P = core.scaled_problem(lp)
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=lp.n), rng.normal(size=lp.m)
    xp, yp = oracle.pdhg_T(P, x, y, 0.5, 0.5)
    x1, y1 = oracle.halpern_point(xp, yp, x, y, x, y, 0, True)
    assert np.allclose(x1, xp, rtol=0, atol=1e-14 * (1 + np.abs(xp).max()))
    assert np.allclose(y1, yp, rtol=0, atol=1e-14 * (1 + np.abs(yp).max()))


@pytest.mark.parametrize("method,const", [("rhpdhg", 2.0), ("r2hpdhg", 1.0)])
def test_lieder_residual_bounds(method, const):
    """Halpern: ||z^k - T z^k|| <= (2/k)||z^k - z^0|| and <= 2/(k+1) dist(z^0, Z*)
    (Lemma sublinear-feas); reflected: the same with constant 1
    (Corollary sublinear-feas-reflected).  Checked every iteration of one
    epoch, in the PDHG norm, against the planted optimum."""
    lp = lpgen.planted_opt(7, m_eq=15, m_ineq=10, n=40)
    ratios = []

    def cb(s):
        k = s["k"]
        P = s["P"]
        if k == 0 or s["n"] > 0:
            return
        res = oracle.m_norm(P, s["x"] - s["xp"], s["y"] - s["yp"], s["tau"], s["sigma"])
        d0 = oracle.m_norm(P, s["x"] - s["x0"], s["y"] - s["y0"], s["tau"], s["sigma"])
        xs, ys = lp.meta["x_opt"] / P.Dc, lp.meta["y_opt"] / P.Dr
        dstar = oracle.m_norm(P, s["x0"] - xs, s["y0"] - ys, s["tau"], s["sigma"])
        assert res <= (const / k) * d0 * (1 + 1e-10) + 1e-13
        assert res <= (const / (k + 1)) * dstar * (1 + 1e-10) + 1e-13
        ratios.append(res / ((const / k) * d0))

    oracle.solve(lp, oracle.Options(method=method, restart="none", max_iter=600, tol=0.0,
                                    callback=cb))
    assert len(ratios) > 500
    assert max(ratios) > 0.5   # the bound is nearly tight: a wrong constant would show


def test_fejer_monotone_restart_points():
    """Lemma iterates-feas (i): with a fixed norm (no primal-weight updates),
    ||z^{n,k} - z*|| <= ||z^{n,0} - z*|| and the restart points approach z*
    monotonically."""
    lp = lpgen.planted_opt(8, m_eq=12, m_ineq=8, n=30)
    anchors = []
    inner_ok = []

    def cb(s):
        P = s["P"]
        xs, ys = lp.meta["x_opt"] / P.Dc, lp.meta["y_opt"] / P.Dr
        dk = oracle.m_norm(P, s["x"] - xs, s["y"] - ys, s["tau"], s["sigma"])
        d0 = oracle.m_norm(P, s["x0"] - xs, s["y0"] - ys, s["tau"], s["sigma"])
        if s["k"] == 0:
            anchors.append(d0)
        inner_ok.append(dk <= d0 * (1 + 1e-10) + 1e-13)

    for method in ["rhpdhg", "r2hpdhg"]:
        anchors.clear()
        inner_ok.clear()
        r = oracle.solve(lp, oracle.Options(method=method, primal_weight=False, tol=1e-10,
                                            callback=cb))
        assert r.status == core.OPTIMAL
        assert all(inner_ok)
        assert len(anchors) >= 3
        assert all(b <= a * (1 + 1e-10) + 1e-13 for a, b in zip(anchors, anchors[1:]))



@pytest.mark.parametrize("kstar", [64, 150])
def test_fixed_frequency_restarts(kstar):
    """eq. (fixed-restart): with checks every 64 steps, every epoch ends at
    the first check with k >= k*; Lemma iterates-feas holds for this rule
    too: with a fixed norm the restart points approach z* monotonically."""
    lp = lpgen.planted_opt(8, m_eq=12, m_ineq=8, n=30)
    anchors = []

    def cb(s):
        if s["k"] == 0:
            P = s["P"]
            xs, ys = lp.meta["x_opt"] / P.Dc, lp.meta["y_opt"] / P.Dr
            anchors.append(oracle.m_norm(P, s["x0"] - xs, s["y0"] - ys, s["tau"], s["sigma"]))

    r = oracle.solve(lp, oracle.Options(restart="fixed", fixed_restart_len=kstar, primal_weight=False,
                                        tol=1e-9, callback=cb))
    assert r.status == core.OPTIMAL
    ks = [e["k"] for e in r.log if e["restart"]]
    first_check = -(-kstar // 64) * 64
    assert len(ks) >= 2 and all(k == first_check for k in ks)
    assert all(b <= a * (1 + 1e-10) + 1e-13 for a, b in zip(anchors, anchors[1:]))


def test_no_restarts():
    lp = lpgen.tiny()
    r = oracle.solve(lp, oracle.Options(restart="none", tol=0.0, max_iter=2000))
    assert r.restarts == 0 and not any(e["restart"] for e in r.log)


def test_average_pdhg_average_is_halpern_iterate_on_affine_problem():
    """Proposition 1 for the raPDHG oracle itself: on the unconstrained
    bilinear problem, with one step size and no restarts, its running average
    zbar^{k+1} (epoch start included) is the rHPDHG iterate z^{k+1}."""
    lp = lpgen.affine(3)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    opt = dict(eta=0.8 / s, primal_weight=False, restart="none", tol=0.0, max_iter=200)
    ra, hal = {}, {}
    oracle.solve(lp, oracle.Options(method="rapdhg", callback=lambda d: ra.__setitem__(d["t"], (d["xa"], d["ya"])),
                                    **opt))
    oracle.solve(lp, oracle.Options(method="rhpdhg", callback=lambda d: hal.__setitem__(d["t"], (d["x"], d["y"])),
                                    **opt))
    assert len(ra) >= 200
    for t in range(1, 200):
        (ax, ay), (hx, hy) = ra[t], hal[t + 1]
        scale = 1 + np.abs(ax).max() + np.abs(ay).max()
        assert np.abs(ax - hx).max() <= 1e-12 * scale
        assert np.abs(ay - hy).max() <= 1e-12 * scale


def test_average_pdhg_restart_rule():
    """raPDHG restarts only at checks, at the first check of the first epoch,
    and afterwards only when the KKT-based rule holds for the logged values;
    every epoch without a restart at a check fails all three tests."""
    lp = lpgen.scaled_powerlaw(23, 300, 1000)
    r = oracle.solve(lp, oracle.Options(method="rapdhg", tol=1e-6, max_iter=200_000))
    assert r.status == core.OPTIMAL and r.restarts >= 3
    first = True
    for e in r.log[:-1]:           # the last check ended the solve before any restart test
        if e["n"] == 0:
            assert e["restart"] == first
            first = False
            continue
        rule = (e["kkt"] <= 0.2 * e["kkt_anchor"]
                or (e["kkt"] <= 0.8 * e["kkt_anchor"] and e["kkt"] > e["kkt_prev"])
                or e["k"] >= 0.36 * e["t"])
        assert e["restart"] == rule


@pytest.mark.parametrize("method", ["rhpdhg", "r2hpdhg", "rapdhg"])
def test_activity_settles_before_convergence(method):
    """Section 4's two-stage picture: the active set of T(z) (x+ at a bound,
    inequality duals at zero) stops changing in finite time, well before the
    iterates converge (finite-time identification), and then stays fixed.
    The count is checked against a direct recount from the logged states."""
    lp = lpgen.tiny(0)
    states = []

    def cb(d):
        states.append((d["t"], d["xp"].copy(), d["yp"].copy(), d["P"]))

    r = oracle.solve(lp, oracle.Options(method=method, tol=1e-10, callback=cb))
    assert r.status == core.OPTIMAL
    assert 0 < r.ident_iters < 0.8 * r.iters
    assert r.active_changes == 0
    checks = [e for e in r.log]
    assert all(e["active_changes"] == 0 for e in checks if e["t"] > r.ident_iters)
    # recount from the T outputs at the check iterations
    by_t = {t: (xp, yp, P) for t, xp, yp, P in states}
    prev = None
    for e in checks:
        xp, yp, P = by_t[e["t"]]
        ax = [(1 if np.isfinite(lo) and v == lo else 2 if np.isfinite(hi) and v == hi else 0)
              for v, lo, hi in zip(xp, P.l, P.u)]
        ay = [int(v == 0.0) for v in yp[lp.m_eq:]]
        if prev is not None:
            want = sum(a != b for a, b in zip(ax, prev[0])) + sum(a != b for a, b in zip(ay, prev[1]))
            assert e["active_changes"] == want
        prev = (ax, ay)

# ---------------------------------------------------------------- whole solves

def test_one_dimensional_example_limit():
    """Figure 1's problem min_{x>=0} max_y (x-1) y has the unique saddle point (1, 0)."""
    lp = lpgen.bilinear_1d()
    for method in ["rhpdhg", "r2hpdhg"]:
        r = oracle.solve(lp, oracle.Options(method=method, tol=1e-12, ruiz_iters=0, pc_alpha=None))
        assert r.status == core.OPTIMAL
        assert r.x[0] == pytest.approx(1.0, abs=1e-10)
        assert r.y[0] == pytest.approx(0.0, abs=1e-10)


@pytest.mark.parametrize("seed", [lpgen.BASE_SEED, 1, 2])
def test_tiny_copy_matches_brute_force(seed):
    lp = lpgen.tiny_copy(seed)
    best, _ = oracle.vertex_enumeration(lp)
    res = _highs(lp)
    if best is None:
        assert res.status == 2
        return
    assert res.fun == pytest.approx(best, rel=1e-9, abs=1e-9)
    for method in ["rhpdhg", "r2hpdhg", "rapdhg"]:
        r = oracle.solve(lp, oracle.Options(method=method, tol=1e-9))
        assert r.status == core.OPTIMAL
        assert r.kkt <= 1e-9
        assert abs(r.pobj - best) <= 1e-7 * (1 + abs(best))


@pytest.mark.parametrize("method", ["rhpdhg", "r2hpdhg", "rapdhg"])
def test_tiny_matches_highs(method):
    lp = lpgen.tiny()
    res = _highs(lp)
    r = oracle.solve(lp, oracle.Options(method=method, tol=1e-8))
    assert r.status == core.OPTIMAL and r.kkt <= 1e-8
    assert abs(r.pobj - res.fun) <= 1e-7 * (1 + abs(res.fun))
    assert abs(r.dobj - res.fun) <= 1e-7 * (1 + abs(res.fun))
    assert np.all(r.x >= lp.lb - 1e-12) and np.all(r.x <= lp.ub + 1e-12)
    assert np.all(r.y[lp.m_eq:] >= 0)


def test_planted_optimum_objective():
    lp = lpgen.planted_opt(3)
    r = oracle.solve(lp, oracle.Options(tol=1e-10))
    assert r.status == core.OPTIMAL
    assert r.pobj == pytest.approx(lp.meta["obj_opt"], rel=1e-8, abs=1e-8)


def _farkas_primal_dense(lp, y):
    """Independent dense restatement of the Farkas alternative: y_ineq >= 0
    and q^T y > max_{l<=x<=u} (K^T y)^T x."""
    K = _dense(lp)
    assert np.all(y[lp.m_eq:] >= 0)
    g = K.T @ y
    sup = 0.0
    for gj, lj, uj in zip(g, lp.lb, lp.ub):
        b = uj if gj > 0 else lj
        if gj != 0 and not np.isfinite(b):
            if abs(gj) > 1e-9 * np.abs(y).max():
                return False
            continue
        sup += gj * b if gj != 0 else 0.0
    return float(lp.rhs @ y) > sup


def test_primal_infeasible_certificate():
    lp = lpgen.add_contradictory_rows(lpgen.tiny(5), seed=1)
    assert _highs(lp).status == 2
    for method in ["rhpdhg", "r2hpdhg", "rapdhg"]:
        r = oracle.solve(lp, oracle.Options(method=method, tol=1e-8, max_iter=200_000))
        assert r.status == core.PRIMAL_INFEASIBLE, oracle.STATUS_NAMES[r.status]
        assert _farkas_primal_dense(lp, r.ray)
    # the closed-form ray on the two contradictory rows passes the oracle's check
    y = np.zeros(lp.m)
    i0, i1 = lp.meta["infeasible_rows"]
    y[i0], y[i1] = -1.0, 1.0
    assert oracle.primal_ray_check(lp, y)[0]
    assert not oracle.primal_ray_check(lp, -y)[0]


def test_dual_infeasible_certificate():
    base = lpgen.scaled_powerlaw(6, 40, 120)
    lp = lpgen.add_unbounded_column(base, seed=2)
    assert _highs(lp).status == 3
    j = lp.meta["ray_column"]
    e = np.zeros(lp.n)
    e[j] = 1.0
    assert oracle.dual_ray_check(lp, e)[0]
    for method in ["rhpdhg", "r2hpdhg", "rapdhg"]:
        r = oracle.solve(lp, oracle.Options(method=method, tol=1e-8, max_iter=200_000))
        assert r.status == core.DUAL_INFEASIBLE, oracle.STATUS_NAMES[r.status]
        d = r.ray
        K = _dense(lp)
        kd = K @ d
        assert lp.c @ d < 0
        assert np.linalg.norm(kd[:lp.m_eq]) <= 1e-6 * abs(lp.c @ d)
        assert np.all(kd[lp.m_eq:] >= -1e-6 * abs(lp.c @ d))


def test_iteration_limit_at_check_granularity():
    lp = lpgen.tiny()
    r = oracle.solve(lp, oracle.Options(max_iter=1, tol=1e-12))
    assert r.status == core.ITER_LIMIT
    assert r.iters == 65   # first check: k = 64 of epoch 0, after 65 evaluations of T
    r = oracle.solve(lp, oracle.Options(max_iter=1000, tol=1e-12))
    assert r.status == core.ITER_LIMIT and 1000 <= r.iters <= 1000 + 65


# ---------------------------------------------------------------- primal weight and adaptive restart

def _dense_m_norm(K, dx, dy, tau, sigma):
    """sqrt(z^T M z) with M = [[I/tau, K^T], [K, I/sigma]] assembled as a dense
    matrix (Section 1.2's PDHG norm, square root restored, y = -y_paper)."""
    n, m = dx.shape[0], dy.shape[0]
    Kd = K.toarray()
    M = np.block([[np.eye(n) / tau, Kd.T], [Kd, np.eye(m) / sigma]])
    z = np.concatenate([dx, dy])
    return math.sqrt(max(float(z @ M @ z), 0.0))


def _epochs(lp, **kw):
    """Run the oracle and collect, per epoch, its primal weight (sqrt(sigma/tau)),
    its anchor z^{n,0}, the state at its first T evaluation and at every check."""
    ep = []

    def cb(s):
        if s["k"] == 0:
            ep.append(dict(n=s["n"], t=s["t"], omega=math.sqrt(s["sigma"] / s["tau"]),
                           tau=s["tau"], sigma=s["sigma"], x0=s["x0"].copy(), y0=s["y0"].copy(),
                           first=(s["x"].copy(), s["y"].copy(), s["xp"].copy(), s["yp"].copy()),
                           checks=[]))
        elif s["k"] % 64 == 0:
            ep[-1]["checks"].append((s["k"], s["t"], s["x"].copy(), s["y"].copy(),
                                     s["xp"].copy(), s["yp"].copy()))

    r = oracle.solve(lp, oracle.Options(callback=cb, **kw))
    return r, ep


def test_primal_weight_starts_at_norm_ratio():
    """Primal weight "as cuPDLP" (Section 7): omega_0 = ||c~|| / ||q~|| on the
    rescaled problem, read back from the step sizes tau = eta/omega,
    sigma = eta*omega of the first epoch; omega_0 = 1 when c = 0."""
    lp = lpgen.scaled_powerlaw(5, 200, 600)
    r, ep = _epochs(lp, tol=0.0, max_iter=64)
    P = r.scaled
    want = np.linalg.norm(P.Dc * lp.c) / np.linalg.norm(P.Dr * lp.rhs)
    assert ep[0]["omega"] == pytest.approx(want, rel=1e-13)
    assert ep[0]["tau"] * ep[0]["sigma"] == pytest.approx(r.eta ** 2, rel=1e-13)
    assert abs(math.log(want)) > 0.5          # far from the fallback value 1
    lp0 = lpgen.LP(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, np.zeros(lp.n), lp.rhs,
                   lp.lb, lp.ub)
    _, ep0 = _epochs(lp0, tol=0.0, max_iter=64)
    assert ep0[0]["omega"] == 1.0


def test_primal_weight_update_is_geometric_mean():
    """At each restart the weight moves half way, in log space, toward the ratio
    of the dual and primal distances between consecutive restart points:
    omega_{n+1} = sqrt(omega_n * ||y^{n+1,0} - y^{n,0}|| / ||x^{n+1,0} - x^{n,0}||)."""
    lp = lpgen.scaled_powerlaw(5, 200, 600)
    r, ep = _epochs(lp, tol=1e-7, max_iter=200_000)
    assert len(ep) >= 10
    moved = 0
    for a, b in zip(ep, ep[1:]):
        dx = np.linalg.norm(b["x0"] - a["x0"])
        dy = np.linalg.norm(b["y0"] - a["y0"])
        want = math.sqrt(a["omega"] * dy / dx)
        assert b["omega"] == pytest.approx(want, rel=1e-12)
        moved += abs(math.log(b["omega"] / a["omega"])) > 1e-3
    assert moved >= 5


def test_adaptive_restart_decision_restated():
    """eq. (adaptive-restart) with checks every 64 steps (Section 3): for
    n >= 1, a check restarts iff ||z - T z||_M <= ||z^{n,0} - T z^{n,0}||_M / e
    in the epoch's norm, or (cuPDLP's artificial restart) k >= 0.36 t; the
    first epoch restarts at its first check.  Both residuals are recomputed
    here with a dense M; every kind of decision occurs."""
    lp = lpgen.scaled_powerlaw(5, 200, 600)
    r, ep = _epochs(lp, tol=1e-7, max_iter=200_000)
    assert r.status == core.OPTIMAL
    K = r.scaled.K
    kinds = {"first": 0, "resid": 0, "artificial": 0, "none": 0}
    logi = 0
    for i, e in enumerate(ep):
        x, y, xp, yp = e["first"]
        r0 = _dense_m_norm(K, x - xp, y - yp, e["tau"], e["sigma"])
        for j, (k, t, x, y, xp, yp) in enumerate(e["checks"]):
            res = _dense_m_norm(K, x - xp, y - yp, e["tau"], e["sigma"])
            entry = r.log[logi]
            logi += 1
            assert entry["t"] == t and entry["r0"] == pytest.approx(r0, rel=1e-10)
            assert entry["resid"] == pytest.approx(res, rel=1e-10)
            last = j == len(e["checks"]) - 1
            if last and i == len(ep) - 1:
                break                          # the solve ended at this check
            restarted = last                   # an epoch ends only at a restart
            if e["n"] == 0:
                kind = "first" if k == 64 else None
            elif res <= r0 / math.e:
                kind = "resid"
            elif k >= 0.36 * t:
                kind = "artificial"
            else:
                kind = "none"
            assert restarted == (kind not in ("none", None)), (i, k, res / r0)
            kinds[kind] += 1
    assert logi == len(r.log)
    assert all(v > 0 for v in kinds.values()), kinds


def test_restart_references_contract_by_e():
    """With a fixed norm (no primal-weight update) and restarts only by the
    residual rule, the restart point is T(z) and T is nonexpansive in the
    M-norm, so r0 of the next epoch is at most the residual that triggered the
    restart, which is at most r0 / e: the restart references fall by at least
    a factor e per epoch (Section 3, the mechanism behind Theorem 2's rate)."""
    lp = lpgen.scaled_powerlaw(5, 200, 600)
    r, ep = _epochs(lp, tol=0.0, max_iter=20_000, primal_weight=False, artificial_restart=0.0)
    K = r.scaled.K
    r0s = []
    for e in ep:
        x, y, xp, yp = e["first"]
        r0s.append(_dense_m_norm(K, x - xp, y - yp, e["tau"], e["sigma"]))
    assert len(r0s) >= 5
    for a, b in zip(r0s[1:], r0s[2:]):        # the first epoch restarts at its first check
        assert b <= a / math.e * (1 + 1e-12)


@pytest.mark.parametrize("which", ["objective", "rhs_and_bounds"])
def test_trajectory_equivariant_under_data_scaling(which):
    """Scaling c by a (duals scale by a) or rhs and bounds by a (primals scale
    by a) maps PDHG iterates onto each other exactly when omega scales with
    ||c|| / ||q||: omega_0 by a (or 1/a), each update by the same factor, and
    the M-norm residual ratios that decide restarts are unchanged.  An omega
    built from the inverse ratio, or a restart test on an unscaled quantity,
    breaks the map.  a = 4 keeps every product exact."""
    lp = lpgen.scaled_powerlaw(5, 200, 600)
    a = 4.0
    if which == "objective":
        lp2 = lpgen.LP(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, a * lp.c, lp.rhs, lp.lb, lp.ub)
        fx, fy = 1.0, a
    else:
        lp2 = lpgen.LP(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c, a * lp.rhs,
                       a * lp.lb, a * lp.ub)
        fx, fy = a, 1.0
    kw = dict(tol=0.0, max_iter=6000)
    r1, e1 = _epochs(lp, **kw)
    r2, e2 = _epochs(lp2, **kw)
    assert r1.restarts >= 5 and r1.restarts == r2.restarts
    assert [e["t"] for e in e1] == [e["t"] for e in e2]
    for p, q in zip(e1, e2):
        assert q["omega"] == pytest.approx(p["omega"] * fy / fx, rel=1e-10)
    sx = 1 + np.abs(r1.x).max()
    sy = 1 + np.abs(r1.y).max()
    assert np.abs(r2.x - fx * r1.x).max() <= 1e-9 * fx * sx
    assert np.abs(r2.y - fy * r1.y).max() <= 1e-9 * fy * sy
