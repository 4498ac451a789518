"""GPU parity tests: the HIP solver (through the C ABI) against the CPU oracle.

Tolerances: FP64 trajectories agree to 1e-10 relative after ~1000 iterations
(both sides run the same algorithm; they differ only in rounding order:
tree-ordered reductions and fused multiply-adds on the GPU).  Final answers
are compared through quantities that are unique -- status, objective,
relative KKT error recomputed by the oracle -- never x or y of a possibly
non-unique optimum.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle import core

pytestmark = pytest.mark.gpu

halp = pytest.importorskip("paper_2407_16144_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

METHODS = [("rhpdhg", halp.LP_METHOD_RHPDHG), ("r2hpdhg", halp.LP_METHOD_R2HPDHG),
           ("rapdhg", halp.LP_METHOD_RAPDHG)]


def _rel(a, b):
    """Element by element: max_i |a_i - b_i| / max(|b_i|, 1e-2 max|b|, 1e-300).
    The floor keeps entries far below the vector's scale (which carry the
    rounding of the larger terms they are summed from, in a different order
    on each side) from deciding the comparison."""
    f = max(1e-2 * float(np.max(np.abs(b))), 1e-300) if b.size else 1e-300
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), f))) if b.size else 0.0


def _gpu(lp, tol, max_iter, **kw):
    opt = halp.lp_default_options(**kw)
    return halp.solve_lp(lp, tol=tol, max_iter=max_iter, opt=opt)


# fixed-order sums everywhere (no column-sorted blocks, whose LDS-atomic row
# sums may round differently from run to run): results reproducible to the bit
DET = dict(plain_sort=0, slice_sort=0)


def _same_within_tol(lp, tol, ra, xa, ya, rb, xb, yb, rays=()):
    """Two solves of one LP that may differ in rounding order: same status;
    optimal results both within tol (KKT error recomputed in FP64 by the
    oracle) with matching objectives; the certificates given in `rays`
    valid by the oracle's Farkas tests."""
    assert ra["status"] == rb["status"], (ra, rb)
    if ra["status"] == halp.LP_OPTIMAL:
        for x, y in ((xa, ya), (xb, yb)):
            kkt, parts = oracle.rel_kkt(lp, x, y)
            assert kkt <= tol * (1 + 1e-6), parts
        assert abs(ra["pobj"] - rb["pobj"]) <= 10 * tol * (1 + abs(ra["pobj"]))
    for ray in rays:
        if ra["status"] == halp.LP_PRIMAL_INFEASIBLE:
            assert oracle.primal_ray_check(lp, ray)[0]
        elif ra["status"] == halp.LP_DUAL_INFEASIBLE:
            assert oracle.dual_ray_check(lp, ray)[0]


@pytest.mark.parametrize("name,code", METHODS)
def test_tiny_final_solution_matches_oracle(name, code):
    lp = lpgen.tiny()
    print(f"case tiny {name}", flush=True)
    res, x, y, _ = _gpu(lp, 1e-8, 500_000, method=code)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=1e-8))
    assert res["status"] == halp.LP_OPTIMAL and ref.status == core.OPTIMAL
    kkt, parts = oracle.rel_kkt(lp, x, y)
    assert kkt <= 1e-8 * (1 + 1e-6), parts
    assert abs(res["rel_kkt"] - kkt) <= 1e-10
    assert abs(res["pobj"] - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))
    # same algorithm, same decisions: identical iteration and restart counts
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert res["sigma_hat"] == pytest.approx(ref.sigma_hat, rel=1e-12)
    assert res["power_iters"] == ref.power_iters


@pytest.mark.parametrize("name,code", METHODS)
@pytest.mark.parametrize("seed", [lpgen.BASE_SEED, 17])
def test_trajectory_parity_1000_iterations(name, code, seed):
    """Iterates after ~1000 evaluations of T (the first check at or past
    1000) agree with the oracle to 1e-10 relative."""
    lp = lpgen.tiny(seed)
    print(f"case trajectory {name} seed={seed}", flush=True)
    res, x, y, _ = _gpu(lp, 0.0, 1000, method=code)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=0.0, max_iter=1000))
    margins = [e["margin"] for e in ref.log if e["n"] > 0]
    assert min(margins, default=1.0) > 1e-8, "restart decision too close to call"
    assert res["status"] == halp.LP_ITER_LIMIT == ref.status
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10
    assert _rel(y, ref.y) <= 1e-10


def test_fixed_step_trajectory_parity_powerlaw():
    """A power-law instance with rows long enough for several workgroups,
    empty-ish columns and free variables, run with the oracle's step size."""
    lp = lpgen.scaled_powerlaw(5, 700, 2400)
    print("case powerlaw fixed eta", flush=True)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    eta = 0.9 / s
    res, x, y, _ = _gpu(lp, 0.0, 640, eta=eta)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=640, eta=eta))
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10
    assert _rel(y, ref.y) <= 1e-10


@pytest.mark.parametrize("seed", [lpgen.BASE_SEED, 1, 2, 3])
def test_tiny_copy_brute_force(seed):
    lp = lpgen.tiny_copy(seed)
    best, _ = oracle.vertex_enumeration(lp)
    if best is None:
        pytest.skip("infeasible draw")
    print(f"case tiny_copy seed={seed}", flush=True)
    for _, code in METHODS:
        res, x, y, _ = _gpu(lp, 1e-9, 500_000, method=code)
        assert res["status"] == halp.LP_OPTIMAL
        assert abs(res["pobj"] - best) <= 1e-7 * (1 + abs(best))


@pytest.mark.parametrize("name,code", METHODS)
def test_primal_infeasible_certificate(name, code):
    lp = lpgen.add_contradictory_rows(lpgen.tiny(5), seed=1)
    print(f"case primal infeasible {name}", flush=True)
    res, x, y, ray = _gpu(lp, 1e-8, 200_000, method=code)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=1e-8, max_iter=200_000))
    assert res["status"] == halp.LP_PRIMAL_INFEASIBLE == ref.status
    assert oracle.primal_ray_check(lp, ray)[0]
    assert res["iters"] == ref.iters
    assert _rel(ray, ref.ray) <= 1e-8


@pytest.mark.parametrize("name,code", METHODS)
def test_dual_infeasible_certificate(name, code):
    lp = lpgen.add_unbounded_column(lpgen.scaled_powerlaw(6, 40, 120), seed=2)
    print(f"case dual infeasible {name}", flush=True)
    res, x, y, ray = _gpu(lp, 1e-8, 200_000, method=code)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=1e-8, max_iter=200_000))
    assert res["status"] == halp.LP_DUAL_INFEASIBLE == ref.status
    assert oracle.dual_ray_check(lp, ray)[0]


def test_no_constraints():
    """m = 0: the minimum of c^T x over the box, at a vertex of the box."""
    n = 50
    rng = np.random.default_rng(0)
    c = rng.standard_normal(n)
    lp = lpgen.LP(n, 0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c,
                  np.zeros(0), -np.ones(n), 2 * np.ones(n))
    print("case m=0", flush=True)
    res, x, y, _ = _gpu(lp, 1e-10, 100_000)
    assert res["status"] == halp.LP_OPTIMAL
    assert np.allclose(x, np.where(c > 0, -1.0, 2.0), atol=1e-9)


def test_empty_rows_and_columns():
    """An empty equality row with zero rhs and an empty column are legal."""
    lp = lpgen.tiny(3)
    m = lp.m
    rp = np.concatenate([lp.rowptr[:1], lp.rowptr])        # new empty row 0
    lp2 = lpgen.LP(lp.n + 1, lp.m_eq + 1, lp.m_ineq, rp.astype(np.int32), lp.col, lp.val,
                   np.concatenate([lp.c, [1.0]]), np.concatenate([[0.0], lp.rhs]),
                   np.concatenate([lp.lb, [0.0]]), np.concatenate([lp.ub, [3.0]]))
    print("case empty row/col", flush=True)
    res, x, y, _ = _gpu(lp2, 1e-8, 500_000)
    ref = oracle.solve(lp2, oracle.Options(tol=1e-8))
    assert res["status"] == halp.LP_OPTIMAL == ref.status
    assert res["iters"] == ref.iters
    assert x[-1] == pytest.approx(0.0, abs=1e-8)
    assert abs(res["pobj"] - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))


def test_rows_longer_than_a_workgroup_tile():
    """Rows with more entries than one stream tile (2048) take the long-row
    path; compare the trajectory with the oracle."""
    base = lpgen.scaled_powerlaw(8, 300, 6000)
    rng = np.random.default_rng(4)
    dense_cols = np.sort(rng.choice(base.n, 4500, replace=False)).astype(np.int32)
    vals = rng.standard_normal(4500)
    xs = base.meta["x_plant"]
    rp = base.rowptr.astype(np.int64)
    me = base.m_eq
    col = np.concatenate([base.col[:rp[me]], dense_cols, base.col[rp[me]:]])
    val = np.concatenate([base.val[:rp[me]], vals, base.val[rp[me]:]])
    rowptr = np.concatenate([rp[:me + 1], rp[me:] + 4500]).astype(np.int32)
    rhs = np.concatenate([base.rhs[:me], [vals @ xs[dense_cols]], base.rhs[me:]])
    lp = lpgen.LP(base.n, me + 1, base.m_ineq, rowptr, col, val, base.c, rhs, base.lb, base.ub)
    print("case long row", flush=True)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    res, x, y, _ = _gpu(lp, 0.0, 320, eta=0.9 / s)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=320, eta=0.9 / s))
    assert res["iters"] == ref.iters
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


def test_sorted_block_boundaries():
    """Column-sorted blocks at their limits: a row of exactly 1024 entries
    (the longest a sorted block takes), one of 1025 (a long block of its
    own), and a run of 1000-entry rows that splits blocks at 2^16 entries;
    the trajectory still agrees with the oracle."""
    import scipy.sparse as sp
    rng = np.random.default_rng(11)
    n, m_eq, m_ineq = 3000, 100, 40
    lens = [1024, 1025] + [1000] * (m_eq - 2) + [12] * m_ineq
    cols = [np.sort(rng.choice(n, L, replace=False)) for L in lens]
    col = np.concatenate(cols).astype(np.int32)
    val = rng.standard_normal(col.size)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    xs = rng.uniform(1.0, 9.0, n)
    kx = sp.csr_matrix((val, col, rp), shape=(m_eq + m_ineq, n)) @ xs
    rhs = np.concatenate([kx[:m_eq], kx[m_eq:] - rng.uniform(0.0, 1.0, m_ineq)])
    lp = lpgen.LP(n, m_eq, m_ineq, rp, col, val, rng.standard_normal(n), rhs, np.zeros(n), np.full(n, 10.0))
    print("case sorted block boundaries", flush=True)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    res, x, y, _ = _gpu(lp, 0.0, 500, eta=0.9 / s)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=500, eta=0.9 / s))
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


def test_unsorted_duplicate_columns_are_canonicalised():
    lp = lpgen.tiny(6)
    m = lp.m
    # reverse each row and split every first entry into two halves
    rows_c, rows_v, rp = [], [], [0]
    for i in range(m):
        cs = list(lp.col[lp.rowptr[i]:lp.rowptr[i + 1]][::-1])
        vs = list(lp.val[lp.rowptr[i]:lp.rowptr[i + 1]][::-1])
        cs.append(cs[0])
        vs[0] *= 0.5
        vs.append(vs[0])
        rows_c += cs
        rows_v += vs
        rp.append(len(rows_c))
    lp2 = lpgen.LP(lp.n, lp.m_eq, lp.m_ineq, np.array(rp, np.int32), np.array(rows_c, np.int32),
                   np.array(rows_v), lp.c, lp.rhs, lp.lb, lp.ub)
    print("case canonicalise", flush=True)
    r1, x1, y1, _ = _gpu(lp, 1e-7, 200_000, **DET)
    r2, x2, y2, _ = _gpu(lp2, 1e-7, 200_000, **DET)
    assert r1["iters"] == r2["iters"]
    assert _rel(x1, x2) <= 1e-12 and _rel(y1, y2) <= 1e-12


def test_device_inputs_equal_host_inputs():
    lp = lpgen.tiny(7)
    print("case device inputs", flush=True)
    opt = halp.lp_default_options(**DET)
    r1, x1, y1, _ = halp.solve_lp(lp, tol=1e-8, max_iter=200_000, opt=opt)
    r2, x2, y2, _ = halp.solve_lp(lp, tol=1e-8, max_iter=200_000, opt=opt, on_device=True)
    assert r1["iters"] == r2["iters"]
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)


def test_int64_row_pointers_equal_int32():
    """lp_create64 (int64 row pointers, host or device) gives the same solve,
    bit for bit in fixed-order mode, as lp_create."""
    lp = lpgen.scaled_powerlaw(33, 400, 1400)
    print("case row_ptr int64", flush=True)
    opt = halp.lp_default_options(**DET)
    ref, xr, yr, _ = halp.solve_lp(lp, tol=1e-6, max_iter=200_000, opt=opt)
    t = lambda a, dt: torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()
    for on_device in (0, 1):
        if on_device:
            args = (t(lp.rowptr.astype(np.int64), torch.int64), t(lp.col, torch.int32), t(lp.val, torch.float64),
                    t(lp.c, torch.float64), t(lp.rhs, torch.float64), t(lp.lb, torch.float64),
                    t(lp.ub, torch.float64))
        else:
            args = (lp.rowptr.astype(np.int64), lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub)
        h = halp.lp_create64(lp.n, lp.m_eq, lp.m_ineq, *args, inputs_on_device=on_device, opt=opt)
        try:
            halp.lp_solve(h, 1e-6, 200_000)
            r = halp.lp_status(h).as_dict()
            x, y = halp.lp_get_solution(h, lp.n, lp.m)
        finally:
            halp.lp_destroy(h)
        assert r["status"] == ref["status"] and r["iters"] == ref["iters"], (on_device, r)
        assert np.array_equal(x, xr) and np.array_equal(y, yr), on_device
    bad = lp.rowptr.astype(np.int64)
    bad[3] = 2**31
    with pytest.raises(halp.HalpError) as ei:
        halp.lp_create64(lp.n, lp.m_eq, lp.m_ineq, t(bad, torch.int64), t(lp.col, torch.int32),
                         t(lp.val, torch.float64), t(lp.c, torch.float64), t(lp.rhs, torch.float64),
                         t(lp.lb, torch.float64), t(lp.ub, torch.float64), inputs_on_device=1)
    assert ei.value.code == halp.LP_ERR_INVALID


def _device_create(lp, rowptr=None, col=None, val=None):
    t = lambda a, dt: torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()
    args = (t(lp.rowptr if rowptr is None else rowptr, torch.int32), t(lp.col if col is None else col, torch.int32),
            t(lp.val if val is None else val, torch.float64), t(lp.c, torch.float64), t(lp.rhs, torch.float64),
            t(lp.lb, torch.float64), t(lp.ub, torch.float64))
    h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, *args, inputs_on_device=1)
    halp.lp_destroy(h)


def test_device_inputs_validated_on_the_device():
    """Device-resident CSR input is validated by kernels (row pointers per
    row, entries one per thread): a column out of range, columns not
    strictly increasing within a row, a NaN value or decreasing row
    pointers are rejected with LP_ERR_INVALID; empty rows (first, inner,
    last) are accepted."""
    lp = lpgen.scaled_powerlaw(31, 300, 1200)
    print("case device validation", flush=True)
    _device_create(lp)
    rp, col, val = lp.rowptr.copy(), lp.col.copy(), lp.val.copy()
    long_row = int(np.argmax(np.diff(rp)))
    a, b = int(rp[long_row]), int(rp[long_row + 1])
    cases = []
    c = col.copy(); c[b - 1] = lp.n; cases.append(("column = n", None, c, None))
    c = col.copy(); c[a] = -1; cases.append(("negative column", None, c, None))
    c = col.copy(); c[a + 1], c[a + 2] = c[a + 2], c[a + 1]; cases.append(("unsorted row", None, c, None))
    c = col.copy(); c[a + 1] = c[a]; cases.append(("duplicate column", None, c, None))
    v = val.copy(); v[len(v) // 2] = np.nan; cases.append(("NaN value", None, None, v))
    r = rp.copy(); r[5] = r[6] + 1; cases.append(("decreasing row_ptr", r, None, None))
    for name, r_, c_, v_ in cases:
        with pytest.raises(halp.HalpError) as ei:
            _device_create(lp, r_, c_, v_)
        assert ei.value.code == halp.LP_ERR_INVALID, name
    # empty rows (the first, one inside, the last): their entries removed --
    # accepted
    for k in (0, 7, lp.m - 1):
        a, b = int(rp[k]), int(rp[k + 1])
        r = rp.copy()
        r[k + 1:] -= b - a
        _device_create(lp, r, np.delete(col, np.arange(a, b)), np.delete(val, np.arange(a, b)))


@pytest.mark.parametrize("det", [True, False])
def test_batch_results_equal_single_results(det):
    """Each LP of a ragged batch gives bit-identical results to solving it
    alone (fixed-order sums), or the same result within the tolerance
    (column-sorted blocks, the default)."""
    lps = [lpgen.scaled_powerlaw(100 + i, m, 3 * m) for i, m in enumerate([40, 300, 75, 1200, 10])]
    lps.append(lpgen.add_contradictory_rows(lpgen.tiny(8), seed=2))
    print(f"case batch det={det}", flush=True)
    kw = DET if det else {}
    h = halp.lp_batch_create(lps, opt=halp.lp_default_options(**kw))
    try:
        halp.lp_batch_solve(h, 1e-6, 100_000)
        for i, lp in enumerate(lps):
            rb = halp.lp_batch_status(h, i).as_dict()
            xb, yb = halp.lp_batch_get_solution(h, i, lp.n, lp.m)
            rs, xs, ys, _ = _gpu(lp, 1e-6, 100_000, **kw)
            if not det:
                _same_within_tol(lp, 1e-6, rb, xb, yb, rs, xs, ys)
                continue
            assert rb["status"] == rs["status"] and rb["iters"] == rs["iters"], (i, rb, rs)
            assert np.array_equal(xb, xs) and np.array_equal(yb, ys), i
    finally:
        halp.lp_batch_destroy(h)


def test_xcd_pinned_batch_equals_spread_batch():
    """A batch large enough to be pinned (each LP's workgroups on one XCD)
    gives the same bits as the same batch spread over all XCDs and as the
    single solves."""
    lps = [lpgen.scaled_powerlaw(600 + i, m, 3 * m) for i, m in enumerate([40, 300, 75, 900, 10, 120] * 4)]
    lps.append(lpgen.add_contradictory_rows(lpgen.tiny(8), seed=2))
    print("case pinned batch", flush=True)
    out = []
    for pin in (1, 0):
        h = halp.lp_batch_create(lps, opt=halp.lp_default_options(xcd_pin=pin, **DET))
        try:
            halp.lp_batch_solve(h, 1e-6, 100_000)
            out.append([(halp.lp_batch_status(h, i).as_dict(), halp.lp_batch_get_solution(h, i, lp.n, lp.m))
                        for i, lp in enumerate(lps)])
        finally:
            halp.lp_batch_destroy(h)
    for i, lp in enumerate(lps):
        (ra, (xa, ya)), (rb, (xb, yb)) = out[0][i], out[1][i]
        assert ra["status"] == rb["status"] and ra["iters"] == rb["iters"], i
        assert np.array_equal(xa, xb) and np.array_equal(ya, yb), i
    for i in (0, 3, len(lps) - 1):
        rs, xs, ys, _ = _gpu(lps[i], 1e-6, 100_000, **DET)
        assert rs["iters"] == out[0][i][0]["iters"] and np.array_equal(xs, out[0][i][1][0])

@pytest.mark.parametrize("graph", [0, 1])
def test_graph_and_stream_launch_agree(graph):
    lp = lpgen.tiny(9)
    print(f"case graph={graph}", flush=True)
    r, x, y, _ = _gpu(lp, 1e-8, 200_000, use_graph=graph, **DET)
    r2, x2, y2, _ = _gpu(lp, 1e-8, 200_000, use_graph=1 - graph, chunk=16, **DET)
    assert r["iters"] == r2["iters"]
    assert np.array_equal(x, x2) and np.array_equal(y, y2)




@pytest.mark.parametrize("name,code", METHODS)
@pytest.mark.parametrize("mode,kstar", [("fixed", 150), ("fixed", 64), ("none", 0)])
def test_restart_rules_trajectory_parity(name, code, mode, kstar):
    """eq. (fixed-restart) and no restarts: the same iterates as the oracle."""
    lp = lpgen.scaled_powerlaw(23, 300, 1000)
    print(f"case restart {mode} k*={kstar} {name}", flush=True)
    rm = halp.LP_RESTART_FIXED if mode == "fixed" else halp.LP_RESTART_NONE
    res, x, y, _ = _gpu(lp, 0.0, 1000, method=code, restart_mode=rm, fixed_restart_len=max(kstar, 1))
    ref = oracle.solve(lp, oracle.Options(method=name, tol=0.0, max_iter=1000, restart=mode,
                                          fixed_restart_len=kstar))
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


@pytest.mark.parametrize("name,code", METHODS)
def test_fixed_restart_certificates(name, code):
    """The infeasibility regime of Section 5 (fixed-frequency restarts): a
    primal-infeasible LP is certified at the same check as by the oracle,
    and the ray passes the oracle's Farkas test.  (On the planted unbounded
    LP, fixed restarts do not reach the 1e-8 dual-ray test within 400k
    iterations on either side; adaptive restarts do.)"""
    lp = lpgen.add_contradictory_rows(lpgen.tiny(7), seed=4)
    print(f"case fixed-restart primal infeasible {name}", flush=True)
    opt = dict(method=code, restart_mode=halp.LP_RESTART_FIXED, fixed_restart_len=256)
    res, x, y, ray = _gpu(lp, 1e-8, 200_000, **opt)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=1e-8, max_iter=200_000, restart="fixed",
                                          fixed_restart_len=256))
    assert res["status"] == ref.status == halp.LP_PRIMAL_INFEASIBLE
    assert res["iters"] == ref.iters
    assert oracle.primal_ray_check(lp, ray)[0]

@pytest.mark.parametrize("sliced,budget", [(False, 0), (True, 0), (False, 150_000), (True, 330_000)])
def test_streamed_tiles_give_identical_iterates(sliced, budget):
    """Matrix tiles past the cache budget are read with non-temporal loads:
    the values (and so every iterate) are the same bits as with all tiles
    cached.  Budget 0 streams every tile; the other budgets exceed the
    vectors of this LP (~90 kB, ~270 kB with the slice partial sums) and
    stream only part of the tiles."""
    lp = lpgen.scaled_powerlaw(31, 400, 1500)
    sl = 0 if sliced else -1
    print(f"case streamed tiles sliced={sliced} budget={budget}", flush=True)
    r1, x1, y1, _ = _gpu(lp, 0.0, 1000, slice_min_bytes=sl, cache_budget_bytes=-1, **DET)
    r2, x2, y2, _ = _gpu(lp, 0.0, 1000, slice_min_bytes=sl, cache_budget_bytes=budget, **DET)
    assert r1["iters"] == r2["iters"] and r1["restarts"] == r2["restarts"]
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=1000))
    assert _rel(x2, ref.x) <= 1e-10 and _rel(y2, ref.y) <= 1e-10

def test_fp32_mode_reaches_moderate_accuracy():
    lp = lpgen.tiny()
    print("case fp32", flush=True)
    res, x, y, _ = _gpu(lp, 1e-4, 200_000, precision=halp.LP_PREC_FP32, polish_tol=0.0)
    assert res["status"] == halp.LP_OPTIMAL and res["polish_iters"] == 0
    kkt, parts = oracle.rel_kkt(lp, x, y)
    assert kkt <= 2e-4, parts


def test_fp32_stall_rule_hands_over_to_fp64():
    """An FP32 phase asked for a tolerance below FP32's reach stops at the
    stall rule, and the FP64 phase finishes the solve."""
    lp = lpgen.tiny(4)
    print("case fp32 stall", flush=True)
    # an FP32 phase cannot reach a 1e-9 relative KKT error: without the stall
    # rule it would spend its share of the budget (a tenth) before the polish
    res, x, y, _ = _gpu(lp, 5e-10, 500_000, precision=halp.LP_PREC_FP32, polish_tol=1e-9, stall_checks=20)
    assert res["status"] == halp.LP_OPTIMAL, res
    assert 0 < res["polish_iters"] < res["iters"] < 250_000, res
    # the stall rule, not the FP32 phase's cap (a tenth of max_iter), ended the FP32 phase
    assert res["iters"] - res["polish_iters"] < 50_000 // 2, res
    kkt, parts = oracle.rel_kkt(lp, x, y)
    assert kkt <= 5e-10 * (1 + 1e-6), parts


def _trivial_lp():
    """x = 1 (one equality row, one variable): optimal at the first checks."""
    return lpgen.LP(n=1, m_eq=1, m_ineq=0, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32),
                    val=np.array([1.0]), c=np.array([1.0]), rhs=np.array([1.0]), lb=np.zeros(1),
                    ub=np.full(1, 10.0))


def test_batch_reblocks_its_last_lps():
    """A batch of 6 LPs of 2-4k rows and 12 trivial LPs sizes its
    column-sorted blocks for 18 LPs sharing each launch (256-row blocks);
    once the trivial LPs are optimal it compacts its schedules and re-sorts
    the 6 still running into the smaller blocks (64 rows) sized for 6 LPs,
    mid-run.  Their iterates after 1,600 evaluations equal those of the 6
    LPs batched alone (blocks of that size from the start) and, for one of
    them, the oracle's, to 1e-10 element by element: the re-sorted layout
    holds the same matrix."""
    big = [lpgen.scaled_powerlaw(700 + i, m, 4 * m) for i, m in enumerate([2000, 3000, 4000, 2500, 3500, 2200])]
    lps = big + [_trivial_lp() for _ in range(12)]
    iters = 1600
    print("case batch reblock", flush=True)
    out = {}
    for name, group in (("mixed", lps), ("alone", big)):
        h = halp.lp_batch_create(group)
        try:
            halp.lp_batch_solve(h, 1e-9, iters)
            out[name] = [(halp.lp_batch_status(h, i).as_dict(), halp.lp_batch_get_solution(h, i, lp.n, lp.m))
                         for i, lp in enumerate(group)]
        finally:
            halp.lp_batch_destroy(h)
    for i in range(len(big), len(lps)):
        assert out["mixed"][i][0]["status"] == halp.LP_OPTIMAL and out["mixed"][i][0]["iters"] < iters // 2
    for i in range(len(big)):
        ra, (xa, ya) = out["mixed"][i]
        rb, (xb, yb) = out["alone"][i]
        assert ra["status"] == rb["status"] == halp.LP_ITER_LIMIT and ra["iters"] == rb["iters"]
        assert ra["restarts"] == rb["restarts"], (ra, rb)
        assert _rel(xa, xb) <= 1e-10 and _rel(ya, yb) <= 1e-10, i
    ref = oracle.solve(big[0], oracle.Options(tol=0.0, max_iter=out["mixed"][0][0]["iters"]))
    assert ref.iters == out["mixed"][0][0]["iters"]
    assert _rel(out["mixed"][0][1][0], ref.x) <= 1e-10 and _rel(out["mixed"][0][1][1], ref.y) <= 1e-10


def test_fp32_phase_cap_without_stall_rule():
    """With the stall rule off, the FP32 phase of a polished solve runs until
    its cap, a tenth of max_iter (honoured at check granularity), and the
    FP64 phase gets the rest of the budget."""
    lp = lpgen.tiny(4)
    print("case fp32 cap", flush=True)
    max_iter = 100_000
    res, x, y, _ = _gpu(lp, 5e-10, max_iter, precision=halp.LP_PREC_FP32, polish_tol=1e-9, stall_checks=0)
    fp32_iters = res["iters"] - res["polish_iters"]
    assert max_iter // 10 <= fp32_iters <= max_iter // 10 + 64, res
    assert res["polish_iters"] > 0 and res["iters"] <= max_iter + 64, res
    if res["status"] == halp.LP_OPTIMAL:
        kkt, parts = oracle.rel_kkt(lp, x, y)
        assert kkt <= 5e-10 * (1 + 1e-6), parts


def test_batch_fp32_polish():
    """FP32 batch to the polish tolerance, then FP64 for each LP: statuses
    equal the FP64 batch's, KKT errors (recomputed by the oracle) within the
    request, certificates valid."""
    lps = [lpgen.scaled_powerlaw(400 + i, m, 3 * m) for i, m in enumerate([60, 300, 20, 150])]
    lps.append(lpgen.add_contradictory_rows(lpgen.scaled_powerlaw(410, 80, 240), seed=3, rel_gap=0.1))
    print("case batch fp32 polish", flush=True)
    out = {}
    for prec in (halp.LP_PREC_FP64, halp.LP_PREC_FP32):
        h = halp.lp_batch_create(lps, opt=halp.lp_default_options(precision=prec))
        try:
            halp.lp_batch_solve(h, 1e-6, 300_000)
            out[prec] = [(halp.lp_batch_status(h, i).as_dict(), halp.lp_batch_get_solution(h, i, lp.n, lp.m),
                          halp.lp_batch_get_certificate(h, i, lp.m) if i == len(lps) - 1 else None)
                         for i, lp in enumerate(lps)]
        finally:
            halp.lp_batch_destroy(h)
    for i, lp in enumerate(lps):
        r64, r32 = out[halp.LP_PREC_FP64][i][0], out[halp.LP_PREC_FP32][i][0]
        assert r32["status"] == r64["status"]
        if r32["status"] == halp.LP_OPTIMAL:
            assert r32["polish_iters"] > 0
            x, y = out[halp.LP_PREC_FP32][i][1]
            kkt, parts = oracle.rel_kkt(lp, x, y)
            assert kkt <= 1e-6 * (1 + 1e-6), parts
    assert out[halp.LP_PREC_FP32][-1][0]["status"] == halp.LP_PRIMAL_INFEASIBLE
    assert oracle.primal_ray_check(lps[-1], out[halp.LP_PREC_FP32][-1][2])[0]


def test_fp32_polish_certifies_dual_infeasibility():
    """A planted-unbounded serving request (an added column with c_j = -1 and
    positive entries on inequality rows only) solved in FP32 with the FP64
    polish phase: certified dual infeasible, with a ray that passes the
    oracle's Farkas test, as the FP64 solve certifies it."""
    req = [r for r in lpgen.serving_trace(count=400) if r.seed == 240716148170][0]
    lp = lpgen.request_instance(req)
    print("case fp32 polish unbounded", flush=True)
    for prec in (halp.LP_PREC_FP32, halp.LP_PREC_FP64):
        res, x, y, ray = _gpu(lp, 1e-4, 1_000_000, precision=prec)
        assert res["status"] == halp.LP_DUAL_INFEASIBLE, (prec, res)
        ok, info = oracle.dual_ray_check(lp, ray)
        assert ok, info
        if prec == halp.LP_PREC_FP32:
            assert res["polish_iters"] > 0      # certified by the FP64 phase


def test_time_limit_status():
    lp = lpgen.scaled_powerlaw(5, 300, 1000)
    print("case time limit", flush=True)
    res, *_ = _gpu(lp, 1e-12, 10_000_000, use_graph=0)
    assert res["status"] != halp.LP_TIME_LIMIT
    opt = halp.lp_default_options()
    r, x, y, _ = halp.solve_lp(lp, tol=1e-12, max_iter=10_000_000, time_limit=0.0, opt=opt)
    assert r["status"] == halp.LP_TIME_LIMIT, r
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))


def test_numerical_status():
    """An objective whose norm overflows (finite entries of 1e308) makes the
    initial primal weight infinite, tau = 0 and sigma = inf: the first check
    sees a non-finite reduction and stops with LP_NUMERICAL, as the oracle
    does."""
    lp = lpgen.tiny()
    c = lp.c.copy()
    c[:4] = 1e308
    bad = lpgen.LP(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, c, lp.rhs, lp.lb, lp.ub)
    print("case numerical", flush=True)
    res, *_ = _gpu(bad, 1e-6, 100_000)
    ref = oracle.solve(bad, oracle.Options(tol=1e-6, max_iter=100_000))
    assert ref.status == core.NUMERICAL
    assert res["status"] == halp.LP_NUMERICAL, res


def test_device_outputs_equal_host_outputs():
    """lp_get_solution and lp_get_certificate with to_device = 1 write the
    same values into device memory as into host memory."""
    for lp, kind in ((lpgen.tiny(), "optimal"), (lpgen.add_contradictory_rows(lpgen.tiny(8), seed=3), "infeasible")):
        print(f"case device outputs {kind}", flush=True)
        h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub)
        try:
            halp.lp_solve(h, 1e-6, 200_000)
            xh, yh = halp.lp_get_solution(h, lp.n, lp.m)
            xd = torch.full((lp.n,), float("nan"), dtype=torch.float64, device="cuda")
            yd = torch.full((lp.m,), float("nan"), dtype=torch.float64, device="cuda")
            assert halp._lib.lp_get_solution(h, xd.data_ptr(), yd.data_ptr(), 1) == halp.LP_OK
            assert np.array_equal(xd.cpu().numpy(), xh) and np.array_equal(yd.cpu().numpy(), yh)
            st = halp.lp_status(h).as_dict()["status"]
            if kind == "infeasible":
                assert st == halp.LP_PRIMAL_INFEASIBLE
                rh = halp.lp_get_certificate(h, lp.m)
                rd = torch.full((lp.m,), float("nan"), dtype=torch.float64, device="cuda")
                assert halp._lib.lp_get_certificate(h, rd.data_ptr(), 1) == halp.LP_OK
                assert np.array_equal(rd.cpu().numpy(), rh)
            else:
                assert st == halp.LP_OPTIMAL
        finally:
            halp.lp_destroy(h)


def test_iteration_limit_and_errors():
    lp = lpgen.tiny()
    print("case limits", flush=True)
    res, *_ = _gpu(lp, 1e-12, 1)
    assert res["status"] == halp.LP_ITER_LIMIT and res["iters"] == 65
    h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub)
    try:
        with pytest.raises(halp.HalpError) as ei:
            halp.lp_get_solution(h, lp.n, lp.m)
        assert ei.value.code == halp.LP_ERR_STATE
        halp.lp_solve(h, 1e-4, 100_000)
        with pytest.raises(halp.HalpError):
            halp.lp_get_certificate(h, lp.m)      # optimal: no certificate
        with pytest.raises(halp.HalpError):
            halp.lp_solve(h, 1e-4, 100_000)       # one solve per handle
    finally:
        halp.lp_destroy(h)


# ------------------------------------------------------------------ column-sliced layout

@pytest.mark.parametrize("sort", [0, 1])
@pytest.mark.parametrize("name,code", METHODS)
def test_sliced_layout_trajectory_parity(name, code, sort):
    """K and K^T stored column-sliced (one slice per XCD, forced on a small LP):
    the slice partial sums are added in a fixed order, and sorted slices of K
    change only the order of the additions within a row, so trajectories
    still agree with the oracle to 1e-10."""
    lp = lpgen.scaled_powerlaw(21, 500, 1800)
    print(f"case sliced trajectory {name} sort={sort}", flush=True)
    res, x, y, _ = _gpu(lp, 0.0, 1000, method=code, slice_min_bytes=0, slice_sort=sort)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=0.0, max_iter=1000))
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


def test_sliced_layout_certificates():
    lp = lpgen.add_contradictory_rows(lpgen.tiny(5), seed=1)
    print("case sliced primal infeasible", flush=True)
    res, x, y, ray = _gpu(lp, 1e-8, 200_000, slice_min_bytes=0)
    assert res["status"] == halp.LP_PRIMAL_INFEASIBLE
    assert oracle.primal_ray_check(lp, ray)[0]
    lp = lpgen.add_unbounded_column(lpgen.scaled_powerlaw(6, 40, 120), seed=2)
    print("case sliced dual infeasible", flush=True)
    res, x, y, ray = _gpu(lp, 1e-8, 200_000, slice_min_bytes=0)
    assert res["status"] == halp.LP_DUAL_INFEASIBLE
    assert oracle.dual_ray_check(lp, ray)[0]


@pytest.mark.parametrize("sort", [0, 1])
def test_sliced_long_rows(sort):
    """A row whose share of one column slice exceeds a stream tile (2048
    entries) takes the long-block path of the slice kernel (row-major
    slices), or shares a sorted block with other rows (sorted slices)."""
    base = lpgen.scaled_powerlaw(9, 400, 30000)
    rng = np.random.default_rng(5)
    dense_cols = np.sort(rng.choice(base.n, 20000, replace=False)).astype(np.int32)
    vals = rng.standard_normal(20000)
    xs = base.meta["x_plant"]
    rp = base.rowptr.astype(np.int64)
    me = base.m_eq
    col = np.concatenate([base.col[:rp[me]], dense_cols, base.col[rp[me]:]])
    val = np.concatenate([base.val[:rp[me]], vals, base.val[rp[me]:]])
    rowptr = np.concatenate([rp[:me + 1], rp[me:] + 20000]).astype(np.int32)
    rhs = np.concatenate([base.rhs[:me], [vals @ xs[dense_cols]], base.rhs[me:]])
    lp = lpgen.LP(base.n, me + 1, base.m_ineq, rowptr, col, val, base.c, rhs, base.lb, base.ub)
    print(f"case sliced long row sort={sort}", flush=True)
    P = core.scaled_problem(lp)
    s, _ = oracle.power_iteration(P.K, 0)
    res, x, y, _ = _gpu(lp, 0.0, 320, eta=0.9 / s, slice_min_bytes=0, slice_sort=sort)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=320, eta=0.9 / s))
    assert res["iters"] == ref.iters
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


def test_sliced_batch_equals_single():
    """Fixed-order (row-major) slices: an LP's result does not depend on the
    batch it is in, to the last bit."""
    lps = [lpgen.scaled_powerlaw(300 + i, m, 3 * m) for i, m in enumerate([60, 500, 20])]
    print("case sliced batch", flush=True)
    opt = halp.lp_default_options(slice_min_bytes=0, **DET)
    h = halp.lp_batch_create(lps, opt=opt)
    try:
        halp.lp_batch_solve(h, 1e-6, 100_000)
        for i, lp in enumerate(lps):
            rb = halp.lp_batch_status(h, i).as_dict()
            xb, yb = halp.lp_batch_get_solution(h, i, lp.n, lp.m)
            rs, xs, ys, _ = halp.solve_lp(lp, tol=1e-6, max_iter=100_000, opt=opt)
            assert rb["iters"] == rs["iters"]
            assert np.array_equal(xb, xs) and np.array_equal(yb, ys)
    finally:
        halp.lp_batch_destroy(h)




@pytest.mark.parametrize("sort_rows,budget", [(4096, -1), (37, 0), (300, 100_000)])
def test_sorted_slices_match_fixed_order_slices(sort_rows, budget):
    """Column-sorted slices of K (LDS atomic row sums; groups of sort_rows
    rows, ragged at the end; all, none or part of the tiles streamed past the
    cache budget) give the fixed-order slices' iterates up to the order of
    the additions within a row."""
    lp = lpgen.scaled_powerlaw(31, 400, 1500)
    print(f"case sorted slices rows={sort_rows} budget={budget}", flush=True)
    r0, x0, y0, _ = _gpu(lp, 0.0, 1000, slice_min_bytes=0, slice_sort=0)
    r1, x1, y1, _ = _gpu(lp, 0.0, 1000, slice_min_bytes=0, slice_sort=1, sort_rows=sort_rows,
                         cache_budget_bytes=budget)
    assert r1["iters"] == r0["iters"] and r1["restarts"] == r0["restarts"]
    assert _rel(x1, x0) <= 1e-10 and _rel(y1, y0) <= 1e-10
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=1000))
    assert _rel(x1, ref.x) <= 1e-10 and _rel(y1, ref.y) <= 1e-10


@pytest.mark.parametrize("prec", [halp.LP_PREC_FP64, halp.LP_PREC_FP32])
def test_sorted_slices_batch_solves(prec):
    """A batch of sliced LPs with sorted slices (FP64, and FP32 with its FP64
    polish): every LP is solved to the tolerance, checked in FP64 by the
    oracle's KKT error."""
    lps = [lpgen.scaled_powerlaw(300 + i, m, 3 * m) for i, m in enumerate([60, 500, 20])]
    lps.append(lpgen.add_contradictory_rows(lpgen.scaled_powerlaw(9, 80, 240), seed=4))
    print(f"case sorted sliced batch prec={prec}", flush=True)
    opt = halp.lp_default_options(slice_min_bytes=0, slice_sort=1, precision=prec)
    h = halp.lp_batch_create(lps, opt=opt)
    try:
        halp.lp_batch_solve(h, 1e-6, 200_000)
        for i, lp in enumerate(lps):
            rb = halp.lp_batch_status(h, i).as_dict()
            xb, yb = halp.lp_batch_get_solution(h, i, lp.n, lp.m)
            if i == len(lps) - 1:
                assert rb["status"] == halp.LP_PRIMAL_INFEASIBLE
                continue
            assert rb["status"] == halp.LP_OPTIMAL, (i, rb)
            kkt, parts = oracle.rel_kkt(lp, xb, yb)
            assert kkt <= 1e-6 * (1 + 1e-6), (i, parts)
    finally:
        halp.lp_batch_destroy(h)
@pytest.mark.parametrize("on_device", [False, True])
def test_fp32_with_fp64_polish(on_device):
    """FP32 phase to the polish tolerance, then FP64 from the FP32 candidate."""
    lp = lpgen.tiny(12)
    print(f"case fp32 polish device={on_device}", flush=True)
    opt = halp.lp_default_options(precision=halp.LP_PREC_FP32, polish_tol=1e-5)
    res, x, y, _ = halp.solve_lp(lp, tol=1e-9, max_iter=500_000, opt=opt, on_device=on_device)
    assert res["status"] == halp.LP_OPTIMAL
    assert 0 < res["polish_iters"] < res["iters"]
    kkt, parts = oracle.rel_kkt(lp, x, y)
    assert kkt <= 1e-9 * (1 + 1e-6), parts
    ref = oracle.solve(lp, oracle.Options(tol=1e-9))
    assert abs(res["pobj"] - ref.pobj) <= 1e-8 * (1 + abs(ref.pobj))


@pytest.mark.parametrize("prec,graph,det", [(halp.LP_PREC_FP64, 0, True), (halp.LP_PREC_FP32, 0, True),
                                            (halp.LP_PREC_FP64, 1, True), (halp.LP_PREC_FP64, 0, False),
                                            (halp.LP_PREC_FP32, 1, False)])
def test_server_results_equal_single_results(prec, graph, det):
    """Continuous batching: LPs submitted at different times, admitted as
    memory frees up, give the same result as solving each alone.  FP32: each
    LP's FP32 phase and its FP64 polish phase run in the server's two
    engines, and still match the single solve bit for bit (fixed-order sums),
    or within the tolerance (column-sorted blocks, the default)."""
    lps = [lpgen.scaled_powerlaw(400 + i, m, 3 * m) for i, m in enumerate([50, 400, 120, 900, 30, 250])]
    lps.append(lpgen.add_contradictory_rows(lpgen.tiny(8), seed=3))
    lps.append(lpgen.add_unbounded_column(lpgen.scaled_powerlaw(6, 40, 120), seed=2))
    print(f"case server precision={prec} graph={graph} det={det}", flush=True)
    kw = DET if det else {}
    opt = halp.lp_default_options(use_graph=graph, precision=prec, **kw)
    phases = 2 if prec == halp.LP_PREC_FP32 else 1
    # a budget that holds only a few of these at once, and 3 slots
    h = halp.lp_server_create(40_000_000, 3, opt=opt)
    try:
        tickets = []
        for k, lp in enumerate(lps):
            tickets.append(halp.lp_server_submit(h, lp, 1e-6, 200_000, float(k)))
            halp.lp_server_step(h, 1)
        pending = set(tickets)
        res = {}
        for _ in range(100_000):
            if not pending:
                break
            halp.lp_server_step(h, 4)
            q, live, used = halp.lp_server_info(h)
            assert live <= 3 * phases
            for t in list(pending):
                r, td = halp.lp_server_poll(h, t)
                if r is not None:
                    k = tickets.index(t)
                    x, y = halp.lp_server_get_solution(h, t, lps[k].n, lps[k].m)
                    res[k] = (r.as_dict(), x, y)
                    halp.lp_server_release(h, t)
                    pending.discard(t)
        assert not pending
    finally:
        halp.lp_server_destroy(h)
    # the last two LPs are primal and dual infeasible by construction
    assert res[len(lps) - 2][0]["status"] == halp.LP_PRIMAL_INFEASIBLE
    assert res[len(lps) - 1][0]["status"] == halp.LP_DUAL_INFEASIBLE
    for k, lp in enumerate(lps):
        rs, xs, ys, ray = _gpu(lp, 1e-6, 200_000, use_graph=0, precision=prec, **kw)
        rb, xb, yb = res[k]
        if not det:
            _same_within_tol(lp, 1e-6, rb, xb, yb, rs, xs, ys, rays=[ray] if ray is not None else [])
            continue
        assert rb["status"] == rs["status"] and rb["iters"] == rs["iters"], (k, rb, rs)
        assert rb["polish_iters"] == rs["polish_iters"], k
        assert np.array_equal(xb, xs) and np.array_equal(yb, ys), k
        if prec == halp.LP_PREC_FP32 and rb["status"] == halp.LP_OPTIMAL:
            assert rb["polish_iters"] > 0
            kkt, parts = oracle.rel_kkt(lp, xb, yb)
            assert kkt <= 1e-6 * (1 + 1e-6), parts


def test_server_refuses_lp_larger_than_its_memory():
    """An LP that would not fit even an idle server is refused at submit
    time, also while other LPs are live (queued, it would block the head of
    the queue for good); the live LP still finishes."""
    print("case server capacity", flush=True)
    h = halp.lp_server_create(2_000_000, 3, opt=halp.lp_default_options())
    try:
        small = lpgen.scaled_powerlaw(5, 50, 150)
        t = halp.lp_server_submit(h, small, 1e-6, 200_000, 0.0)
        halp.lp_server_step(h, 1)
        assert halp.lp_server_info(h)[1] == 1
        big = lpgen.scaled_powerlaw(6, 2000, 6000)
        with pytest.raises(halp.HalpError, match="larger than"):
            halp.lp_server_submit(h, big, 1e-6, 200_000, 1.0)
        for _ in range(10_000):
            r, _ = halp.lp_server_poll(h, t)
            if r is not None:
                break
            halp.lp_server_step(h, 4)
        assert r is not None and r.as_dict()["status"] == halp.LP_OPTIMAL
        assert halp.lp_server_info(h)[0] == 0
    finally:
        halp.lp_server_destroy(h)


@pytest.mark.parametrize("prec", [halp.LP_PREC_FP64, halp.LP_PREC_FP32])
def test_server_stays_within_its_budget(prec):
    """The device memory a server takes (free memory before and after, while
    LPs are admitted, solved and polished) stays within hbm_budget_bytes, up
    to the allocator's rounding."""
    budget = 300_000_000
    lps = [lpgen.scaled_powerlaw(500 + i, m, 4 * m) for i, m in enumerate([3000, 1500, 6000, 800, 4000])]
    print(f"case server budget precision={prec}", flush=True)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    h = halp.lp_server_create(budget, 4, opt=halp.lp_default_options(precision=prec))
    worst = 0
    try:
        tickets = [halp.lp_server_submit(h, lp, 1e-4, 200_000, float(k)) for k, lp in enumerate(lps)]
        pending = set(tickets)
        for _ in range(100_000):
            if not pending:
                break
            halp.lp_server_step(h, 2)
            torch.cuda.synchronize()
            worst = max(worst, free0 - torch.cuda.mem_get_info()[0])
            for t in list(pending):
                r, _ = halp.lp_server_poll(h, t)
                if r is not None:
                    assert r.as_dict()["status"] == halp.LP_OPTIMAL
                    halp.lp_server_release(h, t)
                    pending.discard(t)
        assert not pending
    finally:
        halp.lp_server_destroy(h)
    print(f"budget {budget} worst device memory in use {worst}", flush=True)
    assert worst <= budget + 16 * 2**20


def test_mps_model_solves():
    """An LP read from MPS (maximisation, ranged row, objective constant) is
    solved to the optimum HiGHS finds for the same model typed in directly."""
    from scipy.optimize import linprog
    from paper_2407_16144_amd import mps
    import os
    m = mps.read(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_model.mps"))
    print("case mps", flush=True)
    res = linprog(c=[-3, -2, 1, -4],
                  A_ub=[[1, 2, 0, 1], [0, -1, -1, 0], [0, 1, 0, 3], [0, -1, 0, -3]],
                  b_ub=[10, -2, 8, -3], A_eq=[[1, 0, -1, 0]], b_eq=[1],
                  bounds=[(0, 4), (None, 6), (-2, 3), (0, 2.5)], method="highs")
    for code in (halp.LP_METHOD_R2HPDHG, halp.LP_METHOD_RAPDHG):
        r, x, y, _ = _gpu(m, 1e-9, 200_000, method=code)
        assert r["status"] == halp.LP_OPTIMAL
        assert m.objective(x) == pytest.approx(-res.fun + 1.5, rel=1e-7, abs=1e-7)



@pytest.mark.parametrize("name,code", METHODS)
@pytest.mark.parametrize("seed", [0, 3])
def test_activity_diagnostics_match_oracle(name, code, seed):
    """Two-stage diagnostics: the iteration of the last active-set change and
    the last check's change count are the oracle's (integer parity)."""
    lp = lpgen.tiny(seed)
    print(f"case activity {name} seed={seed}", flush=True)
    res, x, y, _ = _gpu(lp, 1e-10, 200_000, method=code)
    ref = oracle.solve(lp, oracle.Options(method=name, tol=1e-10))
    assert res["iters"] == ref.iters
    assert res["ident_iters"] == ref.ident_iters and res["active_changes"] == ref.active_changes



@pytest.mark.parametrize("shape", [dict(tile_rows=128, slice_entries=256, slice_rows=64, **DET),
                                   dict(tile_rows=37, slice_entries=1024, slice_rows=200, **DET),
                                   dict(tile_rows=200, sort_rows=37),
                                   dict(tile_rows=256, sort_rows=1)])
def test_tile_shapes_trajectory_parity(shape):
    """Other SpMV tile shapes (the tuner's search space) change only the
    rounding order inside rows: iterates still agree with the oracle."""
    lp = lpgen.scaled_powerlaw(21, 500, 1800)
    print(f"case tile shape {shape}", flush=True)
    res, x, y, _ = _gpu(lp, 0.0, 1000, slice_min_bytes=0, **shape)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=1000))
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert _rel(x, ref.x) <= 1e-10 and _rel(y, ref.y) <= 1e-10


def test_autotune_picks_a_measured_shape():
    from paper_2407_16144_amd import autotune
    lp = lpgen.scaled_powerlaw(21, 500, 1800)
    print("case autotune", flush=True)
    best, table, secs = autotune.autotune(lp, iters=256, slice_min_bytes=0)
    assert len(table) == len(autotune.FIRST) + len(autotune.GROUP_SHAPES) + len(autotune.SLICE_SHAPES)
    assert best in [shape for shape, _ in table]
    assert all(ms > 0 for _, ms in table)
    r, x, y, _ = _gpu(lp, 1e-4, 100_000, slice_min_bytes=0, **best)
    assert r["status"] == halp.LP_OPTIMAL
