"""The allocation-free entry point lp_solve_static (device memory from the
library's static workspace only) against lp_create + lp_solve +
lp_get_solution with the same options, through the C ABI: two calls in a
row, the second with a smaller LP, then LPs beyond the workspace, which must
be refused with LP_ERR_OOM and leave the workspace usable."""
import numpy as np
import pytest

import lpgen
import oracle

pytestmark = pytest.mark.gpu

halp = pytest.importorskip("paper_2407_16144_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


def _dev(lp):
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return (t(lp.rowptr, torch.int32), t(lp.col, torch.int32), t(lp.val, torch.float64),
            t(lp.c, torch.float64), t(lp.rhs, torch.float64), t(lp.lb, torch.float64),
            t(lp.ub, torch.float64))


def _static(lp, tol, max_iter, opt):
    x = torch.full((lp.n,), float("nan"), dtype=torch.float64, device="cuda")
    y = torch.full((max(lp.m, 1),), float("nan"), dtype=torch.float64, device="cuda")
    r = halp.lp_solve_static(lp.n, lp.m_eq, lp.m_ineq, *_dev(lp), tol, max_iter, x=x, y=y, opt=opt)
    torch.cuda.synchronize()
    return r.as_dict(), x.cpu().numpy(), y.cpu().numpy()[:lp.m]


@pytest.mark.parametrize("fixed_order", [True, False], ids=["fixed-order", "default"])
def test_static_solve_equals_create_solve(fixed_order):
    extra = {"plain_sort": 0, "slice_sort": 0} if fixed_order else {}
    opt = halp.lp_default_options(use_graph=0, **extra)
    cases = [("powerlaw 1500x5000", lpgen.scaled_powerlaw(31, 1500, 5000), 1e-4), ("tiny", lpgen.tiny(), 1e-6)]
    for name, lp, tol in cases:   # two calls in a row, the second LP smaller
        print(f"case {name} fixed_order={fixed_order}", flush=True)
        ref, xr, yr, _ = halp.solve_lp(lp, tol=tol, max_iter=200_000, opt=opt, on_device=True)
        res, x, y = _static(lp, tol, 200_000, opt)
        assert res["status"] == ref["status"] == halp.LP_OPTIMAL, (res, ref)
        if fixed_order:
            # fixed-order sums: the same arithmetic in the same order
            assert res["iters"] == ref["iters"] and res["restarts"] == ref["restarts"]
            assert np.array_equal(x, xr) and np.array_equal(y, yr)
            assert res["pobj"] == ref["pobj"] and res["rel_kkt"] == ref["rel_kkt"]
        else:
            # LDS-atomic row sums round in a run-dependent order: both are
            # solutions at the requested tolerance, by the oracle's KKT error
            kkt, parts = oracle.rel_kkt(lp, x, y)
            assert kkt <= tol * (1 + 1e-6), parts
            assert abs(res["pobj"] - ref["pobj"]) <= 10 * tol * (1 + abs(ref["pobj"]))
        assert res["rel_kkt"] <= tol


def test_static_solve_refuses_lps_beyond_the_workspace():
    opt = halp.lp_default_options()
    cap = halp.LP_STATIC_WORKSPACE_BYTES
    for nnz in (3_000_000, 1_500_000):
        # one dense row over nnz variables: refused by the size floor (3M
        # entries), or while carving the solver's buffers (1.5M entries),
        # before any kernel uses memory beyond the workspace
        print(f"case refuse nnz={nnz}", flush=True)
        n = nnz
        rowptr = torch.tensor([0, nnz], dtype=torch.int32, device="cuda")
        col = torch.arange(nnz, dtype=torch.int32, device="cuda")
        val = torch.ones(nnz, dtype=torch.float64, device="cuda")
        c = torch.ones(n, dtype=torch.float64, device="cuda")
        rhs = torch.ones(1, dtype=torch.float64, device="cuda")
        lb = torch.zeros(n, dtype=torch.float64, device="cuda")
        ub = torch.ones(n, dtype=torch.float64, device="cuda")
        with pytest.raises(halp.HalpError) as ei:
            halp.lp_solve_static(n, 1, 0, rowptr, col, val, c, rhs, lb, ub, 1e-4, 1000, opt=opt)
        assert ei.value.code == halp.LP_ERR_OOM
        assert str(cap) in str(ei.value)
    # the workspace is usable after a refusal
    print("case after refusal", flush=True)
    lp = lpgen.tiny()
    res, x, y = _static(lp, 1e-6, 200_000, halp.lp_default_options(plain_sort=0, slice_sort=0))
    ref, xr, yr, _ = halp.solve_lp(lp, tol=1e-6, max_iter=200_000,
                                   opt=halp.lp_default_options(use_graph=0, plain_sort=0, slice_sort=0),
                                   on_device=True)
    assert res["status"] == halp.LP_OPTIMAL and np.array_equal(x, xr) and np.array_equal(y, yr)


def test_static_solve_rejects_fp32():
    lp = lpgen.tiny()
    with pytest.raises(halp.HalpError) as ei:
        halp.lp_solve_static(lp.n, lp.m_eq, lp.m_ineq, *_dev(lp), 1e-4, 1000,
                             opt=halp.lp_default_options(precision=halp.LP_PREC_FP32))
    assert ei.value.code == halp.LP_ERR_INVALID
