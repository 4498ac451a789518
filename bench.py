#!/usr/bin/env python3
"""Benchmark: solved LPs/s (and latency) of restarted Halpern PDHG on one MI355X.

Default workload: one synthetic LP shaped like the largest of the paper's
MIP-relaxation instances (>10M nonzeros, Table 1): 375k equality + 125k
inequality rows, 2M variables, 29.6M nonzeros with power-law row lengths
(10..5000) and six decades of row scaling, 20% free variables, feasible and
bounded by construction.  Its matrices and vectors (about 1 GB per iteration
in FP64) do not fit the 256 MB Infinity Cache, so the sparse products stream
from HBM.  A step is one whole solve: lp_create (validation, transpose,
scaling, power iteration, layouts) and lp_solve to a relative KKT error of
1e-4, r2HPDHG, FP64 by default (--precision fp32: FP32 streams and an FP64
polish), through the C ABI, with the inputs resident in HBM (torch tensors)
when the timed region starts.  Other workloads: --workload large (150k + 50k
rows x 1M variables, 9.8M nonzeros), tiny, batch (512 LPs), serve (Poisson
arrivals), mps (a file).

Prints one JSON line.  `--gpus N` with N > 1 exits: the solver runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METHODS = {"rhpdhg": 0, "r2hpdhg": 1, "rapdhg": 2}


def algorithmic_bytes(n, m, nnz, s, sorted_blocks=False):
    """Algorithmic bytes of one plain (non-check) step's two kernels.
    dual step : K entries (s + 4 B each), row pointers, one read of the
                gathered 2x+ - x, and the row epilogue (read y, q, y0, write y);
    primal step: K^T entries, row pointers, one read of the gathered y, and
                the column epilogue (read x, c, l, u, x0; write xbar, x).
    Column-sorted blocks read no row pointers (the row is packed into the
    column index)."""
    rp = 0 if sorted_blocks else 1
    dual = nnz * (s + 4) + rp * 4 * (m + 1) + s * n + 4 * s * m
    primal = nnz * (s + 4) + rp * 4 * (n + 1) + s * m + 7 * s * n
    return primal, dual


def kernel_bytes(n, m, nnz, s, primal_sliced, dual_sliced, grouped=False, plain_sorted=False):
    """Algorithmic bytes per launch of each of the four kernels of a plain
    step.  Where a product's sums come from a slice kernel (column-sliced,
    or stored in sorted groups), that kernel is charged the matrix, row
    pointers and gathered vector, and the step kernel only its epilogue; the
    slice partial sums exchanged between the two are not algorithmic traffic
    and are charged to neither.  Sorted groups (grouped) and column-sorted
    plain blocks carry no row pointers (the row is packed into the column
    index)."""
    prp = 0 if (grouped if primal_sliced else plain_sorted) else 4 * (n + 1)
    drp = 0 if (grouped if dual_sliced else plain_sorted) else 4 * (m + 1)
    pmat = nnz * (s + 4) + s * m + prp
    dmat = nnz * (s + 4) + s * n + drp
    pepi, depi = 7 * s * n, 4 * s * m
    return {"primal_slice": pmat if primal_sliced else 0,
            "primal_step": pepi + (0 if primal_sliced else pmat),
            "dual_slice": dmat if dual_sliced else 0,
            "dual_step": depi + (0 if dual_sliced else dmat)}


def batch_roofline(ksum, s, sorted_blocks=False):
    """Roofline of the dominant step kernel of a batch from the library's
    timings: per-kernel average durations (event-pair cost taken out) and the
    average sizes of the LPs the timed steps processed (finished LPs leave the
    schedules).  Small LPs are not column-sliced, so the two step kernels hold
    the whole products."""
    kn = max(ksum.get("steps", 0), 1)
    ev = ksum.get("event_pair_ms", 0.0) / kn
    avg = {k: max(ksum.get(k + "_ms", 0.0) / kn - ev, 0.0) for k in ("primal", "dual")}
    nnz, n, m = (ksum.get(k, 0.0) / kn for k in ("nnz", "n", "m"))
    pb, db = algorithmic_bytes(n, m, nnz, s, sorted_blocks)
    byts = {"primal": pb, "dual": db}
    dom = max(avg, key=lambda k: avg[k])
    ach = byts[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom + "_step",
            "bytes_per_launch": int(byts[dom]), "avg_ms": {k + "_step": round(v, 5) for k, v in avg.items()},
            "avg_scheduled": {"nnz": round(nnz), "n": round(n), "m": round(m)},
            "timed_steps": int(ksum.get("steps", 0)), "event_pair_ms": round(ev, 5)}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary (profiles/traffic_<workload>.json: FETCH_SIZE and
    WRITE_SIZE runs scaled by a streaming-kernel calibration), or None when
    there is none or the kernel sources have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_2407_16144_amd import rocprof_summary
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != rocprof_summary.kernel_source_hash():
        return None
    ks = t.get("kernels", {})
    k = ks.get(kernel)
    if k is None:   # a kernel named by its prefix (template arguments chosen at run time)
        hits = [v for name, v in ks.items() if name.startswith(kernel)]
        k = hits[0] if len(hits) == 1 else None
    return None if k is None else int(round(k["traffic_bytes"]))


def copy_probe(torch, mb):
    """A plain streaming kernel (y = -x over FP64 vectors of `mb` MB: reads and
    writes mb MB per launch) timed with HIP events on the current stream: the
    bandwidth a simple stream reaches on this GPU, as context for the
    roofline fractions (and the known-size kernel that calibrates the HBM byte
    counters)."""
    nel = int(mb * 1e6 / 8)
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    byts = 2 * nel * 8
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_launch": byts, "ms": round(ms, 4), "GBs": round(byts / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def cpu_model():
    """The host CPU's model name (the first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lp, eta, gpu_iters, gpu_power_iters, method, x=None, y=None, gpu_kkt=None):
    """Oracle timed on a bounded sample of the same LP (one process, one
    core): one oracle solve of a single epoch (scaling, then 65 iterations at
    the GPU's step size with one check), timed per phase from the oracle's
    per-iteration callback, and ten power iterations on the scaled matrix;
    extrapolated to a whole solve with the GPU's iteration and
    power-iteration counts.  When the GPU's solution (x, y) is given, the
    oracle also recomputes its relative KKT error in FP64 (independent of
    the solver's own reduction)."""
    import oracle
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    stamps = []
    cb = lambda s: stamps.append(time.perf_counter())
    t0 = time.perf_counter()
    r = oracle.solve(lp, oracle.Options(method=method, tol=0.0, max_iter=64, eta=eta, callback=cb))
    t_end = time.perf_counter()
    t_setup = stamps[0] - t0                        # scaling, start point and the first T
    t_iter = (stamps[-1] - stamps[0]) / max(len(stamps) - 1, 1)
    p0 = time.perf_counter()
    oracle.power_iteration(r.scaled.K, 0, max_iters=10, min_iters=10, rtol=0.0)
    t_pw = (time.perf_counter() - p0) / 10.0
    est = t_setup + gpu_power_iters * t_pw + gpu_iters * t_iter
    out = {"value": 1.0 / est, "unit": "LPs/s", "cores": 1, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cores": os.cpu_count(),
           "sample": (f"same LP, one process: scaling + start ({t_setup:.1f}s), {len(stamps)} "
                      f"iterations ({t_iter:.3f}s each, one check included), 10 power iterations "
                      f"({t_pw:.3f}s each), measured in {t_end - t0 + 10 * t_pw:.1f}s and extrapolated "
                      f"to the GPU's {gpu_power_iters} power and {gpu_iters} solver iterations: "
                      f"est. {est:.0f}s per LP"),
           "seconds_per_iteration": t_iter}
    if x is not None and y is not None:
        kkt, parts = oracle.rel_kkt(lp, x, y)
        out["oracle_rel_kkt_of_gpu_solution"] = kkt
        out["oracle_pobj_of_gpu_solution"] = parts["pobj"]
        if gpu_kkt is not None:
            out["gpu_reported_rel_kkt"] = gpu_kkt
    return out


def _oracle_rate_worker(args):
    """One LP of a pool baseline: oracle time per iteration (65 iterations
    after scaling and a 10-step power iteration), for extrapolation."""
    lp, method, gpu_iters, gpu_pw = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    from oracle import core
    t0 = time.perf_counter()
    P = core.scaled_problem(lp)
    t_scale = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.power_iteration(P.K, 0, max_iters=10, min_iters=10, rtol=0.0)
    t_pw = (time.perf_counter() - t0) / 10.0
    t0 = time.perf_counter()
    r = oracle.solve(lp, oracle.Options(method=method, tol=0.0, max_iter=64, eta=0.5))
    t_iter = max(time.perf_counter() - t0 - t_scale, 1e-9) / r.iters
    return t_scale + gpu_pw * t_pw + gpu_iters * t_iter


def cpu_pool_baseline(lps, results, method, sample=16):
    """The oracle on a pool of host processes (one LP at a time each), timed
    on the first `sample` LPs and extrapolated to the GPU's per-LP iteration
    and power-iteration counts: LPs/s = pool size / mean seconds per LP."""
    import multiprocessing as mp
    k = min(sample, len(lps))
    procs = max(1, min(os.cpu_count() or 1, 16, k))
    jobs = [(lps[i], method, results[i]["iters"], results[i]["power_iters"]) for i in range(k)]
    t0 = time.perf_counter()
    # fresh interpreters: the children import only the oracle (no GPU state is forked)
    with mp.get_context("spawn").Pool(procs) as pool:
        est = pool.map(_oracle_rate_worker, jobs)
    wall = time.perf_counter() - t0
    mean = sum(est) / len(est)
    return {"value": procs / mean, "unit": "LPs/s", "cores": procs, "kind": "oracle",
            "sample": (f"first {k} LPs, {procs} processes: scaling + 10 power iterations + 65 "
                       f"iterations each ({wall:.1f}s), extrapolated to the GPU's iteration counts; "
                       f"mean {mean:.1f}s per LP")}


def _det(args):
    """--fixed-order: no column-sorted blocks (bit-reproducible sums)."""
    return {"plain_sort": 0, "slice_sort": 0} if args.fixed_order else {}


def _opts(halp, args, **kw):
    return halp.lp_default_options(
        method=METHODS[args.method],
        precision=halp.LP_PREC_FP32 if args.precision == "fp32" else halp.LP_PREC_FP64, **_det(args), **kw)


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, math.ceil(q * len(v)) - 1))]


def serial_solve(halp, lps, tol, max_iter, method):
    """One LP at a time, FP64, the same method, device-resident inputs: the
    baseline the batched and serving paths are compared with."""
    opt = halp.lp_default_options(method=METHODS[method])
    t0 = time.perf_counter()
    solved = 0
    for i, lp in enumerate(lps):
        r, *_ = halp.solve_lp(lp, tol=tol, max_iter=max_iter, opt=opt, on_device=True)
        solved += r["status"] in (1, 2, 3)
        if (i + 1) % 16 == 0 or i + 1 == len(lps):
            print(f"serial FP64: {i + 1}/{len(lps)} LPs, {solved} solved, "
                  f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    return solved, time.perf_counter() - t0


def run_batch(args, copy=None):
    """512 power-law LPs of uneven size (10% primal infeasible) solved as one
    batch: per step, create (device-resident inputs) + solve of all of them."""
    import torch
    import lpgen
    import paper_2407_16144_amd as halp
    t0 = time.perf_counter()
    lps = lpgen.batch(count=args.batch_count)
    nnz = sum(lp.nnz for lp in lps)
    print(f"generated {len(lps)} LPs ({nnz} nnz) in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    arr, keep = halp.make_problems(lps, on_device=True)
    torch.cuda.synchronize()
    opt = _opts(halp, args, profile=args.profile_every, verbose=args.verbose,
                use_graph=0 if args.no_graph else 1)
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        c0 = time.perf_counter()
        h = halp.lp_batch_create_from(arr, len(lps), True, stream=stream, opt=opt)
        print(f"batch created in {time.perf_counter() - c0:.2f}s", file=sys.stderr, flush=True)
        try:
            halp.lp_batch_solve(h, args.tol, args.max_iter, args.time_limit)
            res = [halp.lp_batch_status(h, i).as_dict() for i in range(len(lps))]
            kt = halp.lp_batch_kernel_times(h)
        finally:
            halp.lp_batch_destroy(h)
        return res, kt

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    ksum = {}
    res = []
    for i in range(args.steps):
        s0 = time.perf_counter()
        res, kt = step()
        lat.append(time.perf_counter() - s0)
        for k, v in kt.items():
            ksum[k] = ksum.get(k, 0.0) + v
        st = [r["status"] for r in res]
        print(f"batch step {i}: {lat[-1]:.2f}s optimal={st.count(1)} infeasible={st.count(2)} "
              f"limit={st.count(4)}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    solved = sum(r["status"] in (1, 2, 3) for r in res) * args.steps
    s = 8 if args.precision == "fp64" else 4
    # roofline of the bulk phase: a separate solve of the whole batch for
    # its first 1,280 iterations with every chunk timed (all LPs live), so
    # that the figure is not drawn from the tail of the timed solves, where
    # few LPs remain
    popt = _opts(halp, args, profile=1, verbose=0, use_graph=0)
    hp = halp.lp_batch_create_from(arr, len(lps), True, stream=stream, opt=popt)
    try:
        halp.lp_batch_solve(hp, 0.0, 1280, args.time_limit)
        bulk = halp.lp_batch_kernel_times(hp)
    finally:
        halp.lp_batch_destroy(hp)
    roofline = batch_roofline(bulk, s, not args.fixed_order)
    if not args.fixed_order:
        roofline["traffic"] = measured_traffic(f"batch-{args.precision}", roofline["kernel"])
    roofline["sampled"] = "first 1,280 iterations of the whole batch, every chunk timed"
    if copy is not None:
        roofline["copy_kernel"] = copy
    roofline["timed_run"] = batch_roofline(ksum, s, not args.fixed_order)
    st = [r["status"] for r in res]
    out = {"metric": "solved LPs/s + p99 latency at 1e-4 rel. KKT; SpMV HBM GB/s vs peak",
           "value": round(solved / wall, 3), "unit": "LPs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": f"batch of {len(lps)} power-law LPs, {nnz} nnz total, tol {args.tol:g}",
                      "method": args.method, "precision": args.precision,
                      "statuses": {"optimal": st.count(1), "primal_infeasible": st.count(2),
                                   "dual_infeasible": st.count(3), "limit": st.count(4) + st.count(5)},
                      "max_iters": max(r["iters"] for r in res),
                      "iters_sgm10": round(math.exp(sum(math.log(r["iters"] + 10) for r in res) / len(res)) - 10, 1),
                      "p50_latency_s": round(_pct(lat, 0.5), 3), "p99_latency_s": round(_pct(lat, 0.99), 3)},
           "roofline": roofline}
    if args.serial_baseline:
        k = min(args.serial_baseline, len(lps))
        sv, sw = serial_solve(halp, lps[:k], args.tol, args.max_iter, args.method)
        out["serial_fp64"] = {"lps": k, "solved": sv, "seconds": round(sw, 2),
                                     "value": round(sv / sw, 3), "unit": "LPs/s"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_pool_baseline(lps, res, args.method)
    del keep
    return out


def run_serve(args):
    """Continuous batching: Poisson arrivals (rate LP/s) of batched-size LPs
    with 2% large, 5% primal-infeasible and 2% dual-infeasible ones, replayed
    against the server; latency = completion - arrival."""
    import lpgen
    import paper_2407_16144_amd as halp
    trace = lpgen.serving_trace(count=args.requests, rate=args.rate)
    t_gen = time.perf_counter()
    lps = [lpgen.request_instance(r) for r in trace]
    print(f"generated {len(lps)} requests in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    opt = _opts(halp, args, use_graph=0 if args.no_graph else 1)
    h = halp.lp_server_create(int(args.budget_gb * 1e9), 512, opt=opt)
    try:
        t0 = halp.lp_server_clock(h)
        arrivals = [t0 + r.t_arrival for r in trace]
        tickets = {}
        nxt = 0
        done = {}
        last_print = 0.0
        while len(done) < len(trace):
            now = halp.lp_server_clock(h)
            while nxt < len(trace) and arrivals[nxt] <= now:
                tickets[halp.lp_server_submit(h, lps[nxt], args.tol, args.max_iter, arrivals[nxt])] = nxt
                nxt += 1
            q, live, _ = halp.lp_server_info(h)
            if live == 0 and q == 0:
                time.sleep(max(0.0, min(0.002, arrivals[nxt] - now)) if nxt < len(trace) else 0)
                continue
            halp.lp_server_step(h, 1)
            for tk, idx in list(tickets.items()):
                r, td = halp.lp_server_poll(h, tk)
                if r is not None:
                    done[idx] = (r.as_dict(), td)
                    halp.lp_server_release(h, tk)
                    del tickets[tk]
            if now - last_print > 5.0:
                last_print = now
                print(f"t={now - t0:.1f}s submitted={nxt} done={len(done)} queued={q} live={live}",
                      file=sys.stderr, flush=True)
        t_end = max(td for _, td in done.values())
    finally:
        halp.lp_server_destroy(h)
    lat = [done[i][1] - arrivals[i] for i in range(len(trace))]
    solved = sum(done[i][0]["status"] in (1, 2, 3) for i in range(len(trace)))
    span = t_end - arrivals[0]
    kinds = {}
    for i, r in enumerate(trace):
        kinds.setdefault(r.kind, []).append(done[i][0]["status"])
    out = {"metric": "solved LPs/s + p99 latency at 1e-4 rel. KKT; SpMV HBM GB/s vs peak",
           "value": round(solved / span, 3), "unit": "LPs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": round(1e3 * span, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32",
           "data": "synthetic",
           "config": {"workload": f"serving: {len(trace)} Poisson arrivals at {args.rate:g} LP/s, tol {args.tol:g}",
                      "method": args.method, "precision": args.precision,
                      "p50_latency_s": round(_pct(lat, 0.5), 4), "p99_latency_s": round(_pct(lat, 0.99), 4),
                      "solved": solved, "requests": len(trace),
                      "seconds_to_95pct_done": round(sorted(done[i][1] for i in range(len(trace)))[
                          max(0, math.ceil(0.95 * len(trace)) - 1)] - arrivals[0], 2),
                      "solved_per_s_to_last_solved": round(solved / max(
                          max((done[i][1] for i in range(len(trace)) if done[i][0]["status"] in (1, 2, 3)),
                              default=arrivals[0]) - arrivals[0], 1e-9), 3),
                      "status_by_kind": {k: {str(s): v.count(s) for s in set(v)} for k, v in kinds.items()},
                      "unfinished": [{"request": i, "kind": trace[i].kind, "seed": trace[i].seed, "m": trace[i].m,
                                      "n": trace[i].n, "status": done[i][0]["status"], "iters": done[i][0]["iters"],
                                      "polish_iters": done[i][0]["polish_iters"]}
                                     for i in range(len(trace)) if done[i][0]["status"] not in (1, 2, 3)]}}
    if args.serial_baseline:
        k = min(args.serial_baseline, len(lps))
        sv, sw = serial_solve(halp, lps[:k], args.tol, args.max_iter, args.method)
        out["serial_fp64"] = {"lps": k, "solved": sv, "seconds": round(sw, 2),
                                     "value": round(sv / sw, 3), "unit": "LPs/s"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_pool_baseline(lps, [done[i][0] for i in range(len(trace))], args.method)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="r2hpdhg", choices=list(METHODS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=2_000_000)
    ap.add_argument("--time-limit", type=float, default=600.0)
    ap.add_argument("--workload", default="mixed", choices=["large", "mixed", "tiny", "batch", "serve", "mps"])
    ap.add_argument("--mps", default=None, help="workload mps: the LP to solve (.mps or .mps.gz)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--requests", type=int, default=1200)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--serial-baseline", type=int, default=0,
                    help="batch/serve: also solve the first N LPs one at a time (FP64 rHPDHG)")
    ap.add_argument("--profile-every", type=int, default=32)
    ap.add_argument("--verbose", type=int, default=20, help="library progress line every N seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="first run a plain streaming kernel (y = -x, FP64) over this many MB "
                         "(calibration of the HBM byte counters)")
    ap.add_argument("--no-graph", action="store_true", help="launch steps without hipGraphs")
    ap.add_argument("--fixed-order", action="store_true",
                    help="plain tiles and row-major slices with fixed-order sums instead of column-sorted "
                         "blocks with LDS-atomic row sums")
    ap.add_argument("--autotune", action="store_true",
                    help="single-LP workloads: pick the SpMV tile shapes by timing them first "
                         "(outside the timed region; reported in config)")
    ap.add_argument("--cache-budget-mb", type=float, default=None,
                    help="bytes (MiB) of vectors and tiles kept in the last-level cache (< 0: all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import lpgen
    import paper_2407_16144_amd as halp

    torch.cuda.set_device(0)
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    copy = copy_probe(torch, args.copy_probe_mb if args.copy_probe_mb > 0 else 1024.0)
    if args.workload == "batch":
        print(json.dumps(run_batch(args, copy)), flush=True)
        return
    print(f"copy probe: {copy['bytes_per_launch']} B per launch at {copy['GBs']:.0f} GB/s", file=sys.stderr,
          flush=True)
    if args.workload == "mps":
        from paper_2407_16144_amd import mps
        if not args.mps:
            ap.error("--workload mps needs --mps FILE")
        lp = mps.read(args.mps)
    else:
        lp = {"large": lpgen.large_single, "mixed": lpgen.large_mixed, "tiny": lpgen.tiny}[args.workload]()
    dev = torch.device("cuda", 0)
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
    tens = (T(lp.rowptr, torch.int32), T(lp.col, torch.int32), T(lp.val, torch.float64),
            T(lp.c, torch.float64), T(lp.rhs, torch.float64), T(lp.lb, torch.float64),
            T(lp.ub, torch.float64))
    stream = torch.cuda.current_stream()
    tuned, tune_info = {}, None
    if args.autotune:
        from paper_2407_16144_amd import autotune
        tuned, table, secs = autotune.autotune(lp, method=METHODS[args.method],
                                               precision=1 if args.precision == "fp32" else 0,
                                               **({} if args.cache_budget_mb is None else
                                                  {"cache_budget_bytes": int(args.cache_budget_mb * 2**20)}))
        tune_info = {"best": tuned, "seconds": round(secs, 2), "table": table}
        print(f"autotune: {tuned} in {secs:.1f}s", file=sys.stderr, flush=True)
    opt = halp.lp_default_options(
        method=METHODS[args.method],
        precision=halp.LP_PREC_FP32 if args.precision == "fp32" else halp.LP_PREC_FP64,
        profile=args.profile_every, verbose=args.verbose, use_graph=0 if args.no_graph else 1,
        **({} if args.cache_budget_mb is None else {"cache_budget_bytes": int(args.cache_budget_mb * 2**20)}),
        **{**_det(args), **tuned})

    def step(keep=False):
        h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, *tens, inputs_on_device=1,
                           stream=stream.cuda_stream, opt=opt)
        try:
            halp.lp_solve(h, args.tol, args.max_iter, args.time_limit)
            r = halp.lp_status(h).as_dict()
            kt = halp.lp_kernel_times(h)
            sol = halp.lp_get_solution(h, lp.n, lp.m) if keep else None
        finally:
            halp.lp_destroy(h)
        return r, kt, sol

    for i in range(args.warmup):
        r, _, _ = step()
        print(f"warmup {i}: status={halp.STATUS_NAMES[r['status']]} iters={r['iters']} "
              f"kkt={r['rel_kkt']:.2e} t={r['seconds']:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lat, results = [], []
    ksum = {"primal_slice_ms": 0.0, "primal_ms": 0.0, "dual_slice_ms": 0.0, "dual_ms": 0.0,
            "event_pair_ms": 0.0, "steps": 0}
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        r, kt, sol = step(keep=(i == args.steps - 1))
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        results.append(r)
        for k in ksum:
            ksum[k] += kt[k]
        print(f"step {i}: status={halp.STATUS_NAMES[r['status']]} iters={r['iters']} "
              f"kkt={r['rel_kkt']:.2e} t={lat[-1]:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    solved = sum(1 for r in results if r["status"] in (1, 2, 3))
    value = solved / wall
    iters = results[-1]["iters"]
    s = 8 if args.precision == "fp64" else 4
    kn = max(ksum["steps"], 1)
    # each event-timed kernel also holds the cost of its two events (measured
    # on an empty pair in the same steps): take it out
    ev = ksum["event_pair_ms"] / kn
    avg = {k: max(ksum[k + "_ms"] / kn - ev, 0.0) if ksum[k + "_ms"] > 0 else 0.0
           for k in ("primal_slice", "primal", "dual_slice", "dual")}
    primal_sliced, dual_sliced = avg["primal_slice"] > 0, avg["dual_slice"] > 0
    kb = kernel_bytes(lp.n, lp.m, lp.nnz, s, primal_sliced, dual_sliced, opt.slice_sort == 1,
                      opt.plain_sort == 1)
    ty = "double" if s == 8 else "float"
    grouped = opt.slice_sort == 1
    # sorted-group kernels: named up to their run-time template arguments
    # (threads per workgroup, gather order)
    kn = {"primal_slice": f"sorted_group_step<{ty}, false" if grouped
          else f"primal_slice_step<{ty}, {opt.slice_entries}>",
          "primal": f"primal_step<{ty}>",
          "dual_slice": f"sorted_group_step<{ty}, true" if grouped
          else f"dual_slice_step<{ty}, {opt.slice_entries}>",
          "dual": f"dual_step<{ty}>"}
    names = {k: v.split("<")[0] + ("[K]" if k == "dual_slice" and grouped else
                                   "[K^T]" if k == "primal_slice" and grouped else "") for k, v in kn.items()}
    byname = {"primal_slice": kb["primal_slice"], "primal": kb["primal_step"],
              "dual_slice": kb["dual_slice"], "dual": kb["dual_step"]}
    dom = max(avg, key=lambda k: avg[k])
    achieved = byname[dom] / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    tstep = sum(avg.values())
    wl_key = f"{args.workload}-{args.precision}" if args.workload != "mps" else None
    kname = kn[dom]
    tr = measured_traffic(wl_key, kname) if wl_key else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                "kernel": kname, "bytes_per_launch": int(byname[dom]),
                "avg_ms": {names[k]: round(v, 5) for k, v in avg.items()},
                "bytes": {names[k]: int(v) for k, v in byname.items()},
                "timed_steps": ksum["steps"], "event_pair_ms": round(ev, 5),
                "step_achieved_GBs": round(sum(byname.values()) / (tstep * 1e-3) / 1e9, 1) if tstep > 0 else 0,
                "copy_kernel": copy}
    lat_sorted = sorted(lat)
    p50 = lat_sorted[len(lat) // 2]
    p99 = lat_sorted[min(len(lat) - 1, math.ceil(0.99 * len(lat)) - 1)]
    out = {
        "metric": "solved LPs/s + p99 latency at 1e-4 rel. KKT; SpMV HBM GB/s vs peak",
        "value": round(value, 5), "unit": "LPs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "mps file" if args.workload == "mps" else "synthetic",
        "config": {"workload": f"single LP {lp.m_eq}+{lp.m_ineq} rows x {lp.n} vars, "
                               f"{lp.nnz} nnz, " + (f"from {args.mps}" if args.workload == "mps"
                                                   else "power-law rows") + f", tol {args.tol:g}",
                   "method": args.method, "precision": args.precision,
                   "iterations": iters, "iterations_per_s": round(iters / (wall / args.steps), 1),
                   "p50_latency_s": round(p50, 3), "p99_latency_s": round(p99, 3),
                   "rel_kkt": results[-1]["rel_kkt"], "status": halp.STATUS_NAMES[results[-1]["status"]],
                   "power_iters": results[-1]["power_iters"],
                   # lp_create (validation, transpose, scaling, layouts, power
                   # iteration) and lp_solve; the four step kernels' event-timed
                   # time per iteration against the solve's wall time per iteration
                   "create_s": round(sum(l - r["seconds"] for l, r in zip(lat, results)) / len(lat), 4),
                   "solve_s": round(sum(r["seconds"] for r in results) / len(results), 4),
                   "step_kernels_us_per_iter": round(1e3 * tstep, 2),
                   "solve_us_per_iter": round(1e6 * sum(r["seconds"] for r in results) / max(
                       1, sum(r["iters"] for r in results)), 2),
                   **({"autotune": tune_info} if tune_info else {})},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(lp, results[-1]["eta"], iters,
                                               results[-1]["power_iters"], args.method,
                                               x=sol[0], y=sol[1], gpu_kkt=results[-1]["rel_kkt"])
        except Exception as e:  # pragma: no cover
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
