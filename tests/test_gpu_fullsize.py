"""Full-size parity on the large workloads, in the launch configuration the
benchmark times (default options: column-sorted layouts, K column-sliced,
hipGraph chunks of 64 steps).

* Single large LP (150k + 50k rows x 1M variables, 9.8M nnz), FP64: the
  iterates after the first check at or past 1000 evaluations of T agree with
  the oracle's element by element to 1e-10, relative to each entry but with
  a floor of 1e-2 of the vector's largest entry, with the same iteration and
  restart counts, every restart decision of the oracle clear of its
  threshold by more than 1e-8 (so that both sides take the same decisions);
  a GPU solve to a 1e-3 relative KKT error has that error when the oracle
  recomputes it.  The floor: the two sides sum in different orders, and an
  entry far smaller than the terms it is summed from (rows scaled over six
  decades) carries their rounding, not its own: measured after 1000
  iterations, the largest difference relative to the vector's largest entry
  is 8e-13, relative to entries above 1e-2 of it 3e-11, and 2e-8 for entries
  down to 1e-6 of it, alike with run-to-run (LDS-atomic) and fixed-order sums.
* Mixed-size LP (375k + 125k rows x 2M variables, 29.6M nnz): FP64 iterates
  after the first check at or past 320 evaluations (five checks, several
  restarts) agree with the oracle to 1e-10 in the same sense; an FP32 solve
  with its FP64 polish phase reaches the 1e-4 relative KKT error when the
  oracle recomputes it in FP64 from the returned point, and its objective is
  within the tolerance of the FP64 solve's (both printed).  The relative KKT
  error does not bound the objective error by itself (on this LP a point
  whose dual residual is 1.5e-5 of 1 + ||c|| lies 4e-3 from the optimum);
  the check holds because the FP64 phase carries the FP32 phase's weight.
* Batch of 512 power-law LPs (74M nnz, 10% planted infeasible), solved as
  one batch in FP64 to 1e-4 as the benchmark does: every planted
  infeasible LP, and no other, ends PRIMAL_INFEASIBLE with a ray that the
  oracle's Farkas test accepts; every other LP ends OPTIMAL with the
  relative KKT error, recomputed by the oracle from the returned point,
  within the tolerance (all 512 checked).
* The first 100 requests of the serving trace (Poisson arrivals at
  200 LP/s, 2% large, 5% infeasible, 2% unbounded), all submitted at once to
  one server of 512 slots as the benchmark's overloaded run has them: every
  feasible request ends OPTIMAL with the oracle-recomputed KKT error within
  1e-4, every infeasible one PRIMAL_INFEASIBLE with a ray the oracle's
  Farkas test accepts, every unbounded one DUAL_INFEASIBLE with a valid ray
  (or, for the requests on which the method stalls, at the iteration limit).
"""
import numpy as np
import pytest

import lpgen
import oracle

pytestmark = pytest.mark.gpu

halp = pytest.importorskip("paper_2407_16144_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(scope="module")
def large():
    return lpgen.large_single()


@pytest.fixture(scope="module")
def mixed():
    return lpgen.large_mixed()


def _elementwise(a, b, floor=1e-2):
    """max_i |a_i - b_i| / max(|b_i|, floor * max|b|)."""
    f = floor * max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), f)))


def _trajectory(lp, iters, name):
    print(f"case {name} trajectory {iters}", flush=True)
    res, x, y, _ = halp.solve_lp(lp, tol=0.0, max_iter=iters, on_device=True)
    ref = oracle.solve(lp, oracle.Options(tol=0.0, max_iter=iters))
    margins = [e["margin"] for e in ref.log if e["n"] > 0]
    print("gpu", res["iters"], res["restarts"], "oracle", ref.iters, ref.restarts,
          "min margin", min(margins) if margins else None, flush=True)
    assert not margins or min(margins) > 1e-8
    assert res["status"] == halp.LP_ITER_LIMIT == ref.status
    assert res["iters"] == ref.iters and res["restarts"] == ref.restarts
    assert res["sigma_hat"] == pytest.approx(ref.sigma_hat, rel=1e-10)
    ex, ey = _elementwise(x, ref.x), _elementwise(y, ref.y)
    print(f"elementwise relative difference (floor 1e-2) x {ex:.2e} y {ey:.2e}; floor 1e-6: "
          f"x {_elementwise(x, ref.x, 1e-6):.2e} y {_elementwise(y, ref.y, 1e-6):.2e}", flush=True)
    assert ex <= 1e-10 and ey <= 1e-10
    return res, ref


@pytest.mark.timeout(600)
def test_large_trajectory_parity_1000(large):
    res, ref = _trajectory(large, 1000, "large")
    assert res["iters"] >= 1000 and res["restarts"] >= 2


@pytest.mark.timeout(400)
def test_large_solution_kkt_property(large):
    lp = large
    print("case large kkt", flush=True)
    res, x, y, _ = halp.solve_lp(lp, tol=1e-3, max_iter=400_000, on_device=True, time_limit=200)
    assert res["status"] == halp.LP_OPTIMAL, res
    kkt, parts = oracle.rel_kkt(lp, x, y)
    assert kkt <= 1e-3 * (1 + 1e-6), parts
    assert abs(kkt - res["rel_kkt"]) <= 1e-8


@pytest.mark.timeout(600)
def test_mixed_fp64_trajectory_parity_320(mixed):
    res, ref = _trajectory(mixed, 320, "mixed fp64")
    assert res["restarts"] >= 2


@pytest.mark.timeout(600)
def test_mixed_fp32_polish_reaches_tolerance(mixed):
    lp = mixed
    tol = 1e-4
    print("case mixed fp32+polish to 1e-4", flush=True)
    opt = halp.lp_default_options(precision=halp.LP_PREC_FP32)
    res, x, y, _ = halp.solve_lp(lp, tol=tol, max_iter=400_000, opt=opt, on_device=True, time_limit=200)
    assert res["status"] == halp.LP_OPTIMAL, res
    assert res["polish_iters"] > 0          # the FP64 phase ran
    kkt, parts = oracle.rel_kkt(lp, x, y)
    r64, x64, y64, _ = halp.solve_lp(lp, tol=tol, max_iter=400_000, on_device=True, time_limit=200)
    assert r64["status"] == halp.LP_OPTIMAL, r64
    kkt64, _ = oracle.rel_kkt(lp, x64, y64)
    dobj = abs(parts["pobj"] - r64["pobj"]) / (1 + abs(r64["pobj"]))
    print(f"fp32+polish: iters {res['iters']} (polish {res['polish_iters']}) reported kkt {res['rel_kkt']:.3e} "
          f"oracle kkt {kkt:.3e} {parts}; fp64: iters {r64['iters']} oracle kkt {kkt64:.3e}; "
          f"relative objective difference {dobj:.3e}", flush=True)
    # the polish phase computes its KKT error in FP64 from FP64 products
    assert kkt <= tol * (1 + 1e-6), parts
    assert abs(kkt - res["rel_kkt"]) <= 1e-8
    # not implied by the tolerance (see above); measured 1.9e-5
    assert dobj <= tol


@pytest.mark.timeout(900)
def test_batch_512_statuses_certificates_and_kkt():
    tol = 1e-4
    print("case batch 512", flush=True)
    m, n, infeasible = lpgen.batch_sizes(lpgen.BASE_SEED + 3, 512)
    lps = lpgen.batch(512)
    h = halp.lp_batch_create(lps)
    try:
        halp.lp_batch_solve(h, tol, 2_000_000)
        results = []
        for i, lp in enumerate(lps):
            r = halp.lp_batch_status(h, i).as_dict()
            if r["status"] == halp.LP_PRIMAL_INFEASIBLE:
                results.append((r, None, halp.lp_batch_get_certificate(h, i, lp.m)))
            else:
                results.append((r, halp.lp_batch_get_solution(h, i, lp.n, lp.m), None))
    finally:
        halp.lp_batch_destroy(h)
    worst = 0.0
    for i, (lp, (r, sol, ray)) in enumerate(zip(lps, results)):
        if infeasible[i]:
            assert r["status"] == halp.LP_PRIMAL_INFEASIBLE, (i, r)
            ok, info = oracle.primal_ray_check(lp, ray)
            assert ok, (i, info)
        else:
            assert r["status"] == halp.LP_OPTIMAL, (i, r)
            kkt, parts = oracle.rel_kkt(lp, *sol)
            assert kkt <= tol * (1 + 1e-6), (i, parts)
            worst = max(worst, kkt)
    print(f"batch 512: {int(infeasible.sum())} certified infeasible, {int((~infeasible).sum())} optimal, "
          f"largest recomputed KKT {worst:.3e}", flush=True)


@pytest.mark.timeout(900)
def test_serving_trace_first_100_requests():
    tol, max_iter = 1e-4, 2_000_000      # the benchmark's budget: some requests need over 300k
    trace = lpgen.serving_trace(count=100)
    lps = [lpgen.request_instance(r) for r in trace]
    print("case serving trace 100", flush=True)
    h = halp.lp_server_create(64 * 10**9, 512)
    out = {}
    try:
        tickets = {halp.lp_server_submit(h, lp, tol, max_iter, r.t_arrival): i
                   for i, (lp, r) in enumerate(zip(lps, trace))}
        for _ in range(1_000_000):
            if not tickets:
                break
            halp.lp_server_step(h, 2)
            for tk, i in list(tickets.items()):
                r, _ = halp.lp_server_poll(h, tk)
                if r is None:
                    continue
                r = r.as_dict()
                lp = lps[i]
                if r["status"] == halp.LP_PRIMAL_INFEASIBLE:
                    extra = halp.lp_server_get_certificate(h, tk, lp.m)
                elif r["status"] == halp.LP_DUAL_INFEASIBLE:
                    extra = halp.lp_server_get_certificate(h, tk, lp.n)
                else:
                    extra = halp.lp_server_get_solution(h, tk, lp.n, lp.m)
                out[i] = (r, extra)
                halp.lp_server_release(h, tk)
                del tickets[tk]
        assert not tickets
    finally:
        halp.lp_server_destroy(h)
    kinds = {}
    for i, (req, lp) in enumerate(zip(trace, lps)):
        r, extra = out[i]
        kinds.setdefault(req.kind, []).append(r["status"])
        if req.kind == "infeasible":
            assert r["status"] == halp.LP_PRIMAL_INFEASIBLE, (i, r)
            ok, info = oracle.primal_ray_check(lp, extra)
            assert ok, (i, info)
        elif req.kind == "unbounded":
            assert r["status"] in (halp.LP_DUAL_INFEASIBLE, halp.LP_ITER_LIMIT), (i, r)
            if r["status"] == halp.LP_DUAL_INFEASIBLE:
                ok, info = oracle.dual_ray_check(lp, extra)
                assert ok, (i, info)
        else:
            assert r["status"] == halp.LP_OPTIMAL, (i, req.kind, r)
            kkt, parts = oracle.rel_kkt(lp, *extra)
            assert kkt <= tol * (1 + 1e-6), (i, parts)
    print("statuses by kind", {k: {s: v.count(s) for s in set(v)} for k, v in kinds.items()}, flush=True)
