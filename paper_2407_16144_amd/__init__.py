"""Python binding of libhalp (include/halp.h): restarted Halpern PDHG for LP on
MI355X.  Argument marshalling only -- every step of the solver runs in the
HIP library.  The functions carry the C names; numpy arrays are passed as
host pointers, torch tensors on the GPU as device pointers.

Importing this package never falls back to anything else: if libhalp.so is
missing it raises ImportError (build it with `python -m
paper_2407_16144_amd.build` or `__graft_entry__.build()`).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # share torch's HIP runtime when torch is present (one runtime per process)
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhalp.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"libhalp.so not built at {LIB_PATH}")
_lib = C.CDLL(LIB_PATH)

LP_OK, LP_ERR_INVALID, LP_ERR_OOM, LP_ERR_DEVICE, LP_ERR_STATE = 0, -1, -2, -3, -4
(LP_UNSOLVED, LP_OPTIMAL, LP_PRIMAL_INFEASIBLE, LP_DUAL_INFEASIBLE, LP_ITER_LIMIT,
 LP_TIME_LIMIT, LP_NUMERICAL) = range(7)
STATUS_NAMES = {0: "UNSOLVED", 1: "OPTIMAL", 2: "PRIMAL_INFEASIBLE", 3: "DUAL_INFEASIBLE",
                4: "ITER_LIMIT", 5: "TIME_LIMIT", 6: "NUMERICAL"}
LP_METHOD_RHPDHG, LP_METHOD_R2HPDHG, LP_METHOD_RAPDHG = 0, 1, 2
LP_PREC_FP64, LP_PREC_FP32 = 0, 1
LP_RESTART_ADAPTIVE, LP_RESTART_FIXED, LP_RESTART_NONE = 0, 1, 2


class lp_options(C.Structure):
    _fields_ = [("method", C.c_int), ("precision", C.c_int), ("ruiz_iters", C.c_int),
                ("pc_alpha", C.c_double), ("check_every", C.c_int), ("restart_beta", C.c_double),
                ("artificial_restart", C.c_double), ("step_safety", C.c_double),
                ("power_max_iters", C.c_int), ("power_min_iters", C.c_int),
                ("power_rtol", C.c_double), ("eps_infeas", C.c_double),
                ("primal_weight", C.c_int), ("seed", C.c_uint64), ("eta", C.c_double),
                ("omega0", C.c_double), ("chunk", C.c_int), ("use_graph", C.c_int),
                ("profile", C.c_int), ("slice_min_bytes", C.c_int64), ("polish_tol", C.c_double),
                ("verbose", C.c_int), ("cache_budget_bytes", C.c_int64), ("stall_checks", C.c_int64),
                ("restart_mode", C.c_int), ("fixed_restart_len", C.c_int64), ("xcd_pin", C.c_int),
                ("tile_rows", C.c_int), ("slice_entries", C.c_int), ("slice_rows", C.c_int),
                ("slice_sort", C.c_int), ("sort_rows", C.c_int), ("plain_sort", C.c_int),
                ("group_threads", C.c_int), ("group_batched", C.c_int), ("group_blocks", C.c_int),
                ("polish_weight", C.c_int)]


class lp_result(C.Structure):
    _fields_ = [("status", C.c_int), ("ray", C.c_int), ("iters", C.c_int64),
                ("restarts", C.c_int64), ("checks", C.c_int64), ("pobj", C.c_double),
                ("dobj", C.c_double), ("rel_kkt", C.c_double), ("rel_primal", C.c_double),
                ("rel_dual", C.c_double), ("rel_gap", C.c_double), ("omega", C.c_double),
                ("eta", C.c_double), ("sigma_hat", C.c_double), ("power_iters", C.c_int),
                ("polish_iters", C.c_int64), ("seconds", C.c_double), ("active_changes", C.c_int64),
                ("ident_iters", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lp_kernel_timing(C.Structure):
    _fields_ = [("primal_slice_ms", C.c_double), ("primal_ms", C.c_double),
                ("dual_slice_ms", C.c_double), ("dual_ms", C.c_double), ("event_pair_ms", C.c_double),
                ("nnz", C.c_double), ("n", C.c_double), ("m", C.c_double), ("steps", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lp_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m_eq", C.c_int64), ("m_ineq", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("c", C.c_void_p), ("rhs", C.c_void_p), ("lb", C.c_void_p), ("ub", C.c_void_p)]


_P = C.c_void_p
_sig = {
    "lp_default_options": (None, [_P]),
    "lp_last_error": (C.c_char_p, []),
    "lp_create": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, _P,
                            C.c_int, _P, _P]),
    "lp_create64": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, _P,
                              C.c_int, _P, _P]),
    "lp_solve": (C.c_int, [_P, C.c_double, C.c_int64, C.c_double]),
    "lp_status": (C.c_int, [_P, _P]),
    "lp_get_solution": (C.c_int, [_P, _P, _P, C.c_int]),
    "lp_get_certificate": (C.c_int, [_P, _P, C.c_int]),
    "lp_kernel_times": (C.c_int, [_P, _P]),
    "lp_get_scaled_matrix": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "lp_destroy": (None, [_P]),
    "lp_batch_create": (C.c_int, [_P, C.c_int, _P, C.c_int, _P, _P]),
    "lp_batch_solve": (C.c_int, [_P, C.c_double, C.c_int64, C.c_double]),
    "lp_batch_status": (C.c_int, [_P, C.c_int, _P]),
    "lp_batch_get_solution": (C.c_int, [_P, C.c_int, _P, _P, C.c_int]),
    "lp_batch_get_certificate": (C.c_int, [_P, C.c_int, _P, C.c_int]),
    "lp_batch_kernel_times": (C.c_int, [_P, _P]),
    "lp_batch_destroy": (None, [_P]),
    "lp_server_create": (C.c_int, [_P, C.c_int64, C.c_int, _P, _P]),
    "lp_server_submit": (C.c_int, [_P, _P, C.c_double, C.c_int64, C.c_double, _P]),
    "lp_server_step": (C.c_int, [_P, C.c_int, _P]),
    "lp_server_poll": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "lp_server_get_solution": (C.c_int, [_P, C.c_int64, _P, _P]),
    "lp_server_get_certificate": (C.c_int, [_P, C.c_int64, _P]),
    "lp_server_release": (C.c_int, [_P, C.c_int64]),
    "lp_server_clock": (C.c_int, [_P, _P]),
    "lp_server_info": (C.c_int, [_P, _P, _P, _P]),
    "lp_server_destroy": (None, [_P]),
    "lp_solve_static": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                  C.c_double, C.c_int64, C.c_double, _P, _P, _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class HalpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _check(rc):
    if rc != LP_OK:
        raise HalpError(rc, lp_last_error())
    return rc


def _ptr(a, dtype):
    """Device pointer of a torch tensor or host pointer of a numpy array."""
    if a is None:
        return None
    if torch is not None and isinstance(a, torch.Tensor):
        return a.data_ptr()
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr


def lp_last_error() -> str:
    return _lib.lp_last_error().decode()


def lp_default_options(**overrides) -> lp_options:
    o = lp_options()
    _lib.lp_default_options(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _marshal_problem(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub, on_device, rp_type=np.int32):
    keep = []
    ptrs = []
    tdt = {np.int32: "torch.int32", np.int64: "torch.int64", np.float64: "torch.float64"}
    for a, dt in ((row_ptr, rp_type), (col_idx, np.int32), (val, np.float64), (c, np.float64),
                  (rhs, np.float64), (lb, np.float64), (ub, np.float64)):
        if on_device:
            if a is None:
                ptrs.append(None)
                continue
            if str(a.dtype) != tdt[dt] or not a.is_contiguous():
                raise TypeError("device inputs must be contiguous tensors of the documented types")
            ptrs.append(a.data_ptr())
        else:
            if a is None:
                ptrs.append(None)
                continue
            arr = np.ascontiguousarray(np.asarray(a), dtype=dt)
            if arr.size == 0:
                arr = np.zeros(1, dtype=dt)
            keep.append(arr)
            ptrs.append(arr.ctypes.data)
    return ptrs, keep


def lp_create(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub, inputs_on_device=0,
              stream=None, opt=None):
    """Returns an opaque handle (c_void_p)."""
    ptrs, keep = _marshal_problem(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub,
                                  inputs_on_device)
    h = C.c_void_p()
    _check(_lib.lp_create(C.byref(h), n, m_eq, m_ineq, *ptrs, int(inputs_on_device),
                          stream, C.byref(opt) if opt is not None else None))
    del keep
    return h


def lp_create64(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub, inputs_on_device=0,
                stream=None, opt=None):
    """lp_create with int64 row pointers; returns an opaque handle."""
    ptrs, keep = _marshal_problem(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub,
                                  inputs_on_device, rp_type=np.int64)
    h = C.c_void_p()
    _check(_lib.lp_create64(C.byref(h), n, m_eq, m_ineq, *ptrs, int(inputs_on_device),
                            stream, C.byref(opt) if opt is not None else None))
    del keep
    return h


def lp_solve(h, rel_kkt_tol, max_iter, time_limit_s=-1.0):
    return _check(_lib.lp_solve(h, rel_kkt_tol, int(max_iter), float(time_limit_s)))


def lp_status(h) -> lp_result:
    r = lp_result()
    _check(_lib.lp_status(h, C.byref(r)))
    return r


def lp_get_solution(h, n, m):
    x = np.empty(max(n, 1))
    y = np.empty(max(m, 1))
    _check(_lib.lp_get_solution(h, x.ctypes.data, y.ctypes.data, 0))
    return x[:n], y[:m]


def lp_get_certificate(h, length):
    r = np.empty(max(length, 1))
    _check(_lib.lp_get_certificate(h, r.ctypes.data, 0))
    return r[:length]


def lp_kernel_times(h):
    """Summed per-kernel durations (ms) of the timed steps, as a dict."""
    t = lp_kernel_timing()
    _check(_lib.lp_kernel_times(h, C.byref(t)))
    return t.as_dict()


def lp_get_scaled_matrix(h, transpose, rows, nnz):
    """The scaled K (transpose 0, `rows` = m) or K^T (1, `rows` = n) as
    stored: (row_ptr, col_idx, val) numpy arrays."""
    rp = np.empty(rows + 1, dtype=np.int32)
    ci = np.empty(max(nnz, 1), dtype=np.int32)
    v = np.empty(max(nnz, 1))
    _check(_lib.lp_get_scaled_matrix(h, int(transpose), rp.ctypes.data, ci.ctypes.data, v.ctypes.data))
    return rp, ci[:nnz], v[:nnz]


def lp_destroy(h):
    _lib.lp_destroy(h)


def make_problems(lps, on_device=False):
    """An lp_problem array (and the arrays it points into) for lpgen.LP-like
    objects; with on_device the arrays are copied to GPU tensors first."""
    arr = (lp_problem * len(lps))()
    keep = []
    for i, lp in enumerate(lps):
        if on_device:
            t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to("cuda")
            arrays = (t(lp.rowptr, torch.int32), t(lp.col, torch.int32), t(lp.val, torch.float64),
                      t(lp.c, torch.float64), t(lp.rhs, torch.float64), t(lp.lb, torch.float64),
                      t(lp.ub, torch.float64))
            ptrs = [a.data_ptr() if a.numel() else None for a in arrays]
            keep.append(arrays)
        else:
            ptrs, k = _marshal_problem(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c,
                                       lp.rhs, lp.lb, lp.ub, 0)
            keep.append(k)
        arr[i] = lp_problem(lp.n, lp.m_eq, lp.m_ineq, *ptrs)
    return arr, keep


def lp_batch_create_from(arr, count, on_device, stream=None, opt=None):
    """lp_batch_create over an existing lp_problem array."""
    h = C.c_void_p()
    _check(_lib.lp_batch_create(C.byref(h), count, arr, int(on_device), stream,
                                C.byref(opt) if opt is not None else None))
    return h


def lp_batch_create(lps, stream=None, opt=None):
    arr, keep = make_problems(lps)
    h = C.c_void_p()
    _check(_lib.lp_batch_create(C.byref(h), len(lps), arr, 0, stream,
                                C.byref(opt) if opt is not None else None))
    del keep
    return h


def lp_batch_solve(h, rel_kkt_tol, max_iter, time_limit_s=-1.0):
    return _check(_lib.lp_batch_solve(h, rel_kkt_tol, int(max_iter), float(time_limit_s)))


def lp_batch_status(h, i) -> lp_result:
    r = lp_result()
    _check(_lib.lp_batch_status(h, i, C.byref(r)))
    return r


def lp_batch_get_solution(h, i, n, m):
    x = np.empty(max(n, 1))
    y = np.empty(max(m, 1))
    _check(_lib.lp_batch_get_solution(h, i, x.ctypes.data, y.ctypes.data, 0))
    return x[:n], y[:m]


def lp_batch_get_certificate(h, i, length):
    r = np.empty(max(length, 1))
    _check(_lib.lp_batch_get_certificate(h, i, r.ctypes.data, 0))
    return r[:length]


def lp_batch_kernel_times(h):
    t = lp_kernel_timing()
    _check(_lib.lp_batch_kernel_times(h, C.byref(t)))
    return t.as_dict()


def lp_batch_destroy(h):
    _lib.lp_batch_destroy(h)


def lp_server_create(hbm_budget_bytes, max_slots, stream=None, opt=None):
    h = C.c_void_p()
    _check(_lib.lp_server_create(C.byref(h), int(hbm_budget_bytes), int(max_slots), stream,
                                 C.byref(opt) if opt is not None else None))
    return h


def lp_server_submit(h, lp, rel_kkt_tol, max_iter, t_arrival):
    arr, keep = make_problems([lp])
    t = C.c_int64()
    _check(_lib.lp_server_submit(h, C.byref(arr[0]), rel_kkt_tol, int(max_iter), float(t_arrival),
                                 C.byref(t)))
    del keep
    return t.value


def lp_server_step(h, chunks=1):
    nd = C.c_int()
    _check(_lib.lp_server_step(h, int(chunks), C.byref(nd)))
    return nd.value


def lp_server_poll(h, ticket):
    d = C.c_int()
    r = lp_result()
    t = C.c_double()
    _check(_lib.lp_server_poll(h, int(ticket), C.byref(d), C.byref(r), C.byref(t)))
    return (r, t.value) if d.value else (None, None)


def lp_server_get_solution(h, ticket, n, m):
    x = np.empty(max(n, 1))
    y = np.empty(max(m, 1))
    _check(_lib.lp_server_get_solution(h, int(ticket), x.ctypes.data, y.ctypes.data))
    return x[:n], y[:m]


def lp_server_get_certificate(h, ticket, length):
    r = np.empty(max(length, 1))
    _check(_lib.lp_server_get_certificate(h, int(ticket), r.ctypes.data))
    return r[:length]


def lp_server_release(h, ticket):
    return _check(_lib.lp_server_release(h, int(ticket)))


def lp_server_clock(h):
    t = C.c_double()
    _check(_lib.lp_server_clock(h, C.byref(t)))
    return t.value


def lp_server_info(h):
    q, l, b = C.c_int(), C.c_int(), C.c_int64()
    _check(_lib.lp_server_info(h, C.byref(q), C.byref(l), C.byref(b)))
    return q.value, l.value, b.value


def lp_server_destroy(h):
    _lib.lp_server_destroy(h)


LP_STATIC_WORKSPACE_BYTES = 64 << 20


def lp_solve_static(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub, rel_kkt_tol, max_iter,
                    time_limit_s=-1.0, x=None, y=None, stream=None, opt=None) -> lp_result:
    """The allocation-free solve: device tensors in, the unscaled solution
    written into the device tensors x (n) and y (m) when given."""
    ptrs, keep = _marshal_problem(n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub, 1)
    for a in (x, y):
        if a is not None and (a.dtype != torch.float64 or not a.is_contiguous() or not a.is_cuda):
            raise TypeError("x and y must be contiguous float64 device tensors")
    if x is not None and x.numel() < n:
        raise ValueError("x holds fewer than n entries")
    if y is not None and y.numel() < m_eq + m_ineq:
        raise ValueError("y holds fewer than m entries")
    r = lp_result()
    _check(_lib.lp_solve_static(n, m_eq, m_ineq, *ptrs, stream, C.byref(opt) if opt is not None else None,
                                float(rel_kkt_tol), int(max_iter), float(time_limit_s),
                                None if x is None else x.data_ptr(), None if y is None else y.data_ptr(),
                                C.byref(r)))
    del keep
    return r


def solve_lp(lp, tol=1e-4, max_iter=1_000_000, time_limit=-1.0, opt=None, on_device=False,
             stream=None):
    """Convenience: create, solve, fetch (status dict, x, y, ray) and destroy."""
    if on_device:
        dev = "cuda"
        t = lambda a, dt: torch.as_tensor(np.asarray(a), dtype=dt, device=dev).contiguous()
        args = (t(lp.rowptr, torch.int32), t(lp.col, torch.int32), t(lp.val, torch.float64),
                t(lp.c, torch.float64), t(lp.rhs, torch.float64), t(lp.lb, torch.float64),
                t(lp.ub, torch.float64))
    else:
        args = (lp.rowptr, lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub)
    h = lp_create(lp.n, lp.m_eq, lp.m_ineq, *args, inputs_on_device=int(on_device),
                  stream=stream, opt=opt)
    try:
        lp_solve(h, tol, max_iter, time_limit)
        r = lp_status(h)
        x, y = lp_get_solution(h, lp.n, lp.m)
        ray = None
        if r.status == LP_PRIMAL_INFEASIBLE:
            ray = lp_get_certificate(h, lp.m)
        elif r.status == LP_DUAL_INFEASIBLE:
            ray = lp_get_certificate(h, lp.n)
        return r.as_dict(), x, y, ray
    finally:
        lp_destroy(h)
