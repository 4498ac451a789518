"""MPS reader (host only): the parsed form of a hand-written model, its
optimum against HiGHS on the model written out independently, a round trip
through MPS text of a generated LP, and error reporting."""
import math
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import lpgen
import oracle
from oracle import core

halp = pytest.importorskip("paper_2407_16144_amd")
from paper_2407_16144_amd import mps  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "small_model.mps")


def _as_lp(m):
    return lpgen.LP(m.n, m.m_eq, m.m_ineq, m.rowptr, m.col, m.val, m.c, m.rhs, m.lb, m.ub)


def test_parse_fixture():
    m = mps.read(FIXTURE)
    assert (m.n, m.m_eq, m.m_ineq) == (4, 1, 4)
    dense = np.zeros((m.m, m.n))
    for i in range(m.m):
        for p in range(m.rowptr[i], m.rowptr[i + 1]):
            dense[i, m.col[p]] += m.val[p]
    want = np.array([[1, 0, -1, 0],      # BAL:    x1 - x3 = 1
                     [-1, -2, 0, -1],    # CAP1:   x1 + 2 x2 + x4 <= 10
                     [0, 1, 1, 0],       # DEMAND: x2 + x3 >= 2
                     [0, 1, 0, 3],       # RANGED: 3 <= x2 + (2 + 1) x4 <= 8
                     [0, -1, 0, -3]], dtype=float)
    assert np.array_equal(dense, want)
    assert np.array_equal(m.rhs, [1, -10, 2, 3, -8])
    assert np.array_equal(m.c, [-3, -2, 1, -4])          # maximisation: costs negated
    assert np.array_equal(m.lb, [0, -np.inf, -2, 0])
    assert np.array_equal(m.ub, [4, 6, 3, 2.5])
    assert m.meta["objsense"] == -1.0 and m.meta["obj_constant"] == 1.5
    assert m.meta["integer"] == [2]


def test_fixture_optimum_matches_highs():
    """The same model typed in directly for HiGHS (maximise, so negate)."""
    res = linprog(c=[-3, -2, 1, -4],
                  A_ub=[[1, 2, 0, 1], [0, -1, -1, 0], [0, 1, 0, 3], [0, -1, 0, -3]],
                  b_ub=[10, -2, 8, -3], A_eq=[[1, 0, -1, 0]], b_eq=[1],
                  bounds=[(0, 4), (None, 6), (-2, 3), (0, 2.5)], method="highs")
    assert res.status == 0
    best = -res.fun + 1.5
    m = mps.read(FIXTURE)
    r = oracle.solve(_as_lp(m), oracle.Options(tol=1e-10))
    assert r.status == core.OPTIMAL
    assert m.objective(r.x) == pytest.approx(best, rel=1e-8, abs=1e-8)


def _to_mps(lp):
    """Writes an LP in the solver's form as MPS text (E rows, then G rows)."""
    out = ["NAME TEST", "ROWS", " N OBJ"]
    out += [f" E R{i}" for i in range(lp.m_eq)] + [f" G R{i}" for i in range(lp.m_eq, lp.m)]
    out.append("COLUMNS")
    rp = lp.rowptr.astype(np.int64)
    cols = {}
    for i in range(lp.m):
        for p in range(rp[i], rp[i + 1]):
            cols.setdefault(int(lp.col[p]), []).append((i, float(lp.val[p])))
    for j in range(lp.n):
        out.append(f"    C{j} OBJ {float(lp.c[j])!r}")
        for i, v in cols.get(j, []):
            out.append(f"    C{j} R{i} {v!r}")
    out.append("RHS")
    out += [f"    RHS R{i} {float(lp.rhs[i])!r}" for i in range(lp.m)]
    out.append("BOUNDS")
    for j in range(lp.n):
        lo, hi = lp.lb[j], lp.ub[j]
        if lo == -math.inf and hi == math.inf:
            out.append(f" FR BND C{j}")
            continue
        if lo == -math.inf:
            out.append(f" MI BND C{j}")
        elif lo != 0.0:
            out.append(f" LO BND C{j} {float(lo)!r}")
        if hi != math.inf:
            out.append(f" UP BND C{j} {float(hi)!r}")
    out.append("ENDATA")
    return "\n".join(out) + "\n"


def test_round_trip_of_a_generated_lp():
    lp = lpgen.scaled_powerlaw(5, 60, 200)
    m = mps.parse(_to_mps(lp))
    assert (m.n, m.m_eq, m.m_ineq) == (lp.n, lp.m_eq, lp.m_ineq)
    assert np.array_equal(m.rhs, lp.rhs) and np.array_equal(m.c, lp.c)
    assert np.array_equal(m.lb, lp.lb) and np.array_equal(m.ub, lp.ub)
    assert np.array_equal(m.rowptr, lp.rowptr)
    for i in range(lp.m):
        a, b = slice(lp.rowptr[i], lp.rowptr[i + 1]), slice(m.rowptr[i], m.rowptr[i + 1])
        o1, o2 = np.argsort(lp.col[a]), np.argsort(m.col[b])
        assert np.array_equal(lp.col[a][o1], m.col[b][o2])
        assert np.array_equal(lp.val[a][o1], m.val[b][o2])


@pytest.mark.parametrize("text,needle", [
    ("ROWS\n N OBJ\nCOLUMNS\n    X OBJ 1 NOPE 2\nENDATA\n", "unknown row"),
    ("ROWS\n N OBJ\n E R\nCOLUMNS\n    X OBJ one\nENDATA\n", "not a number"),
    ("ROWS\n N OBJ\nCOLUMNS\n    X OBJ 1\nBOUNDS\n XX BND X 1\nENDATA\n", "unknown bound type"),
    ("ROWS\n Q OBJ\nENDATA\n", "unknown row type"),
])
def test_errors_name_the_line(text, needle):
    with pytest.raises(ValueError) as ei:
        mps.parse(text)
    assert needle in str(ei.value) and "line" in str(ei.value)
