"""Tuner for the SpMV tile shapes of the solver's step kernels.

The sparse products are bound by random gathers and by how many of them a
CU keeps in flight, which depends on the matrix's row-length mix; the best
tile shape is therefore measured, not derived.  `autotune` creates the LP
once per candidate shape, runs a fixed number of steps with every chunk
timed by HIP events (their own cost taken out), and returns the shape with
the least kernel time per step.

Search (coordinate descent, 5 + 4 + 6 candidates):
  1. the products in column-sorted plain blocks or plain tiles (every
     product of small LPs, K^T of some large ones): plain blocks with the
     default row cap (sized for the LPs that share the launches, at most
     2048 rows) or sort_rows 1024 or 128, or fixed-order plain tiles
     (plain_sort 0) of tile_rows in {128, 256};
  2. only if the LP has a product with a slice kernel (sorted groups, the
     default for products whose gathered vector exceeds slice_min_bytes or
     whose groups can hold more rows than a plain block), with the best of
     step 1: sorted groups with group_threads in {256, 512, 1024} (the
     default picks one for about eight waves per CU) or unbatched gathers
     (group_batched 0), then fixed-order slices (slice_sort 0) with
     slice_entries in {256, 512, 1024} x slice_rows in {64, 128}.

Each candidate's solve starts from scratch and its iterates are discarded;
the chosen options are then passed to the real solve.
"""
from __future__ import annotations

import time

from . import (lp_create, lp_default_options, lp_destroy, lp_kernel_times, lp_solve,
               make_problems, lp_batch_create_from, lp_batch_solve, lp_batch_kernel_times,
               lp_batch_destroy)

FIRST = ({}, {"sort_rows": 1024}, {"sort_rows": 128}, {"plain_sort": 0, "tile_rows": 128},
         {"plain_sort": 0, "tile_rows": 256})
GROUP_SHAPES = ({"group_threads": 256}, {"group_threads": 512}, {"group_threads": 1024}, {"group_batched": 0})
SLICE_SHAPES = tuple((e, r) for e in (256, 512, 1024) for r in (64, 128))


def _step_ms(kt):
    n = max(int(kt["steps"]), 1)
    launched = 2 + (kt["primal_slice_ms"] > 0) + (kt["dual_slice_ms"] > 0)
    total = kt["primal_slice_ms"] + kt["primal_ms"] + kt["dual_slice_ms"] + kt["dual_ms"]
    return (total - launched * kt["event_pair_ms"]) / n, kt["primal_slice_ms"] > 0 or kt["dual_slice_ms"] > 0


def _time_single(tensors, lp, opts, iters, stream):
    h = lp_create(lp.n, lp.m_eq, lp.m_ineq, *tensors, inputs_on_device=1, stream=stream, opt=opts)
    try:
        lp_solve(h, 0.0, iters, -1.0)
        return _step_ms(lp_kernel_times(h))
    finally:
        lp_destroy(h)


def _time_batch(arr, count, opts, iters, stream):
    h = lp_batch_create_from(arr, count, True, stream=stream, opt=opts)
    try:
        lp_batch_solve(h, 0.0, iters, -1.0)
        return _step_ms(lp_batch_kernel_times(h))
    finally:
        lp_batch_destroy(h)


def autotune(lp_or_lps, iters: int = 640, stream=None, **base):
    """Tile shape with the least kernel time per step for this LP (or list of
    LPs solved as one batch).  `base` holds the other lp_options fields of
    the real solve (method, precision, ...).  Returns (best, table, seconds):
    best is a dict of lp_options fields, table lists (shape, ms per step)."""
    import numpy as np
    import torch
    t0 = time.perf_counter()
    batch = isinstance(lp_or_lps, (list, tuple))
    if batch:
        arr, keep = make_problems(list(lp_or_lps), on_device=True)
        run = lambda o: _time_batch(arr, len(lp_or_lps), o, iters, stream)
    else:
        lp = lp_or_lps
        dev = torch.device("cuda", torch.cuda.current_device())
        T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
        tensors = (T(lp.rowptr, torch.int32), T(lp.col, torch.int32), T(lp.val, torch.float64),
                   T(lp.c, torch.float64), T(lp.rhs, torch.float64), T(lp.lb, torch.float64),
                   T(lp.ub, torch.float64))
        run = lambda o: _time_single(tensors, lp, o, iters, stream)
    table = []

    def measure(shape):
        o = lp_default_options(**{**base, **shape, "profile": 1, "verbose": 0})
        ms, sliced = run(o)
        table.append((dict(shape), round(ms, 5)))
        return ms, sliced

    best, best_ms, sliced = None, float("inf"), False
    for shape in FIRST:
        ms, sl = measure(shape)
        sliced |= sl
        if ms < best_ms:
            best, best_ms = dict(shape), ms
    if sliced:
        cands = [{**best, **g} for g in GROUP_SHAPES]
        cands += [{**best, "slice_sort": 0, "slice_entries": e, "slice_rows": r} for e, r in SLICE_SHAPES]
        for shape in cands:
            ms, _ = measure(shape)
            if ms < best_ms:
                best, best_ms = shape, ms
    if batch:
        del keep
    return best, table, time.perf_counter() - t0
