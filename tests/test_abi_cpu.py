"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, the binding's structs match the header, and host-side
validation rejects malformed LPs before any GPU work."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "halp.h")

halp = pytest.importorskip("paper_2407_16144_amd")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(lp_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(halp._lib, n), n
    assert set(names) == set(halp.EXPORTED)


def test_struct_layouts_match_header():
    src = open(HEADER).read()

    def fields(struct):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + ";", src).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        out = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            toks = decl.replace(",", " , ").split()
            ty = toks[0] if toks[0] != "const" else toks[1]
            names = [t.strip("*") for t in decl.split(ty, 1)[1].split(",")]
            out += [n.strip().strip("*").strip() for n in names]
        return out

    assert fields("lp_options") == [f for f, _ in halp.lp_options._fields_]
    assert fields("lp_result") == [f for f, _ in halp.lp_result._fields_]
    assert fields("lp_problem") == [f for f, _ in halp.lp_problem._fields_]
    assert fields("lp_kernel_timing") == [f for f, _ in halp.lp_kernel_timing._fields_]


def test_enum_values_match_header():
    src = open(HEADER).read()
    for name in ["LP_METHOD_RHPDHG", "LP_METHOD_R2HPDHG", "LP_METHOD_RAPDHG",
                 "LP_RESTART_ADAPTIVE", "LP_RESTART_FIXED", "LP_RESTART_NONE", "LP_OPTIMAL",
                 "LP_PRIMAL_INFEASIBLE", "LP_DUAL_INFEASIBLE", "LP_ITER_LIMIT"]:
        m = re.search(name + r"\s*=\s*(\d+)", src)
        assert m, name
        assert int(m.group(1)) == getattr(halp, name), name


def test_default_options():
    o = halp.lp_default_options()
    assert o.method == halp.LP_METHOD_R2HPDHG and o.precision == halp.LP_PREC_FP64
    assert o.ruiz_iters == 10 and o.pc_alpha == 1.0 and o.check_every == 64
    assert abs(o.restart_beta - np.exp(-1)) < 1e-16
    assert o.step_safety == 0.9 and o.eps_infeas == 1e-8 and o.primal_weight == 1


def _tiny_arrays():
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 1], np.int32)
    val = np.array([1.0, 1.0, 2.0])
    return dict(n=2, m_eq=1, m_ineq=1, row_ptr=rp, col_idx=ci, val=val, c=np.ones(2),
                rhs=np.array([1.0, 0.5]), lb=np.zeros(2), ub=np.full(2, 5.0))


@pytest.mark.parametrize("mutate,needle", [
    (lambda a: a.update(n=0), "n >= 1"),
    (lambda a: a.update(row_ptr=np.array([1, 2, 3], np.int32)), "row_ptr"),
    (lambda a: a.update(row_ptr=np.array([0, 2, 1], np.int32)), "row_ptr"),
    (lambda a: a.update(col_idx=np.array([0, 5, 1], np.int32)), "column index"),
    (lambda a: a.update(val=np.array([1.0, np.nan, 2.0])), "non-finite matrix"),
    (lambda a: a.update(c=np.array([np.inf, 1.0])), "non-finite objective"),
    (lambda a: a.update(rhs=np.array([np.nan, 1.0])), "right-hand side"),
    (lambda a: a.update(lb=np.array([3.0, 0.0]), ub=np.array([1.0, 5.0])), "bounds"),
    (lambda a: a.update(lb=np.array([np.inf, 0.0])), "bounds"),
    (lambda a: a.update(ub=np.array([np.nan, 1.0])), "bounds"),
])
def test_invalid_lp_rejected_on_host(mutate, needle):
    a = _tiny_arrays()
    mutate(a)
    with pytest.raises(halp.HalpError) as ei:
        halp.lp_create(a["n"], a["m_eq"], a["m_ineq"], a["row_ptr"], a["col_idx"], a["val"], a["c"],
                       a["rhs"], a["lb"], a["ub"])
    assert ei.value.code == halp.LP_ERR_INVALID
    assert needle in str(ei.value)


def test_invalid_options_rejected():
    a = _tiny_arrays()
    for kw in [dict(method=3), dict(precision=2), dict(check_every=0), dict(step_safety=0.0),
               dict(restart_mode=3), dict(restart_mode=halp.LP_RESTART_FIXED, fixed_restart_len=0),
               dict(tile_rows=0), dict(tile_rows=257), dict(slice_rows=300), dict(slice_entries=700),
               dict(slice_sort=2), dict(sort_rows=0), dict(sort_rows=16385), dict(plain_sort=-1),
               dict(group_threads=300), dict(group_batched=2), dict(group_blocks=-1), dict(polish_weight=3)]:
        with pytest.raises(halp.HalpError) as ei:
            halp.lp_create(a["n"], a["m_eq"], a["m_ineq"], a["row_ptr"], a["col_idx"], a["val"],
                           a["c"], a["rhs"], a["lb"], a["ub"], opt=halp.lp_default_options(**kw))
        assert ei.value.code == halp.LP_ERR_INVALID


def test_package_fails_loudly_without_library(tmp_path):
    """The binding has no fallback: a package copy without libhalp.so refuses to import."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2407_16144_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2407_16144_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_2407_16144_amd"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0 and "libhalp.so not built" in r.stderr


def test_int64_row_pointers_checked_on_host():
    a = _tiny_arrays()
    rp = np.asarray(a["row_ptr"], dtype=np.int64)
    for bad, what in ((2**31, "above 2^31 - 1"), (-1, "negative")):
        r = rp.copy()
        r[1] = bad
        with pytest.raises(halp.HalpError) as ei:
            halp.lp_create64(a["n"], a["m_eq"], a["m_ineq"], r, a["col_idx"], a["val"], a["c"], a["rhs"],
                             a["lb"], a["ub"])
        assert ei.value.code == halp.LP_ERR_INVALID, what
