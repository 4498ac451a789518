"""Reader for LPs in MPS format (free or fixed columns, names without blanks).

Turns an MPS model into the solver's form

    min c^T x  s.t.  A x = b (equality rows first),  G x >= h,  l <= x <= u

as host arrays ready for `lp_create` / `lp_batch_create` (the same fields as
the solver's other inputs: n, m_eq, m_ineq, rowptr, col, val, c, rhs, lb, ub).

  * N rows: the first is the objective (its RHS entry is minus the objective
    constant); later N rows are free rows and are dropped.
  * L rows become -a x >= -b; G rows stay; E rows go to the equality block.
  * RANGES: E rows with R > 0 give [b, b + R], with R < 0 give [b + R, b];
    L rows give [b - |R|, b], G rows [b, b + |R|].  A range with two finite
    sides becomes two inequality rows (one if the sides coincide: equality).
  * BOUNDS: UP, LO, FX, FR, MI, PL, BV, LI, UI (integer bounds are kept as
    bounds: the model is solved as its LP relaxation, integer markers are
    recorded and ignored).  An UP bound below 0 on a column whose lower bound
    is still the default 0 sets the lower bound to -inf (the usual MPS rule).
  * OBJSENSE MAX negates c (meta["objsense"] = -1); the original model's
    objective at x is objsense * c^T x + constant (MPSModel.objective).
  * Repeated (row, column) entries are summed.

Errors raise ValueError naming the line.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import gzip
import math

import numpy as np

_INF = math.inf


@dataclass
class MPSModel:
    n: int
    m_eq: int
    m_ineq: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    c: np.ndarray
    rhs: np.ndarray
    lb: np.ndarray
    ub: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.m_eq + self.m_ineq

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def objective(self, x) -> float:
        """Objective of the original model at x: c holds objsense times the
        model's costs, so this is objsense * c^T x + constant."""
        return self.meta["objsense"] * float(self.c @ np.asarray(x)) + self.meta["obj_constant"]


def _number(tok, lineno):
    try:
        return float(tok)
    except ValueError:
        raise ValueError(f"line {lineno}: '{tok}' is not a number") from None


def parse(text: str, name: str = "") -> MPSModel:
    section = None
    objsense = 1.0
    obj_row = None
    row_type = {}          # name -> 'E' | 'L' | 'G' | 'N'
    row_order = []         # constraint rows in file order
    col_index = {}
    col_names = []
    entries = {}           # (row, col) -> value
    obj = {}               # col -> value
    rhs = {}
    ranges = {}
    bounds = []            # (type, col, value or None, lineno)
    integer = set()
    in_int = False
    obj_constant = 0.0
    for lineno, raw in enumerate(text.splitlines(), 1):
        line = raw.rstrip()
        if not line.strip() or line.lstrip().startswith("*"):
            continue
        toks = line.split()
        if not raw[0].isspace():
            head = toks[0].upper()
            if head == "NAME":
                section = "NAME"
                continue
            if head == "OBJSENSE":
                section = "OBJSENSE"
                if len(toks) > 1:
                    objsense = -1.0 if toks[1].upper() in ("MAX", "MAXIMIZE") else 1.0
                continue
            if head in ("ROWS", "COLUMNS", "RHS", "RANGES", "BOUNDS"):
                section = head
                continue
            if head == "ENDATA":
                break
            raise ValueError(f"line {lineno}: unknown section '{toks[0]}'")
        if section == "OBJSENSE":
            objsense = -1.0 if toks[0].upper() in ("MAX", "MAXIMIZE") else 1.0
        elif section == "ROWS":
            if len(toks) != 2:
                raise ValueError(f"line {lineno}: ROWS entry needs a type and a name")
            t, r = toks[0].upper(), toks[1]
            if t not in ("N", "E", "L", "G"):
                raise ValueError(f"line {lineno}: unknown row type '{toks[0]}'")
            if r in row_type:
                raise ValueError(f"line {lineno}: row '{r}' defined twice")
            row_type[r] = t
            if t == "N":
                if obj_row is None:
                    obj_row = r
            else:
                row_order.append(r)
        elif section == "COLUMNS":
            if len(toks) >= 3 and toks[1].strip("'").upper() == "MARKER":
                mk = toks[2].strip("'").upper()
                if mk == "INTORG":
                    in_int = True
                elif mk == "INTEND":
                    in_int = False
                continue
            if len(toks) not in (3, 5):
                raise ValueError(f"line {lineno}: COLUMNS entry needs 1 or 2 (row, value) pairs")
            cname = toks[0]
            if cname not in col_index:
                col_index[cname] = len(col_names)
                col_names.append(cname)
            j = col_index[cname]
            if in_int:
                integer.add(j)
            for r, v in zip(toks[1::2], toks[2::2]):
                if r not in row_type:
                    raise ValueError(f"line {lineno}: unknown row '{r}'")
                val = _number(v, lineno)
                if r == obj_row:
                    obj[j] = obj.get(j, 0.0) + val
                elif row_type[r] != "N":
                    entries[(r, j)] = entries.get((r, j), 0.0) + val
        elif section in ("RHS", "RANGES"):
            pairs = toks[1:] if len(toks) % 2 == 1 else toks
            if len(pairs) not in (2, 4):
                raise ValueError(f"line {lineno}: {section} entry needs 1 or 2 (row, value) pairs")
            for r, v in zip(pairs[0::2], pairs[1::2]):
                if r not in row_type:
                    raise ValueError(f"line {lineno}: unknown row '{r}'")
                val = _number(v, lineno)
                if section == "RHS":
                    if r == obj_row:
                        obj_constant = -val
                    elif row_type[r] != "N":
                        rhs[r] = val
                elif row_type[r] != "N":
                    ranges[r] = val
        elif section == "BOUNDS":
            t = toks[0].upper()
            if t in ("FR", "MI", "PL", "BV"):
                if len(toks) not in (3, 4):
                    raise ValueError(f"line {lineno}: {t} bound needs a set and a column")
                cname, val = toks[2] if len(toks) >= 3 else toks[1], None
                if len(toks) == 4 and t == "BV":
                    val = _number(toks[3], lineno)
            elif t in ("UP", "LO", "FX", "LI", "UI", "SC"):
                if len(toks) != 4:
                    raise ValueError(f"line {lineno}: {t} bound needs a set, a column and a value")
                cname, val = toks[2], _number(toks[3], lineno)
            else:
                raise ValueError(f"line {lineno}: unknown bound type '{toks[0]}'")
            if cname not in col_index:
                raise ValueError(f"line {lineno}: unknown column '{cname}'")
            bounds.append((t, col_index[cname], val, lineno))
        else:
            raise ValueError(f"line {lineno}: data outside a section")
    if obj_row is None and not col_names:
        raise ValueError("no objective row and no columns")
    n = len(col_names)
    lb = np.zeros(n)
    ub = np.full(n, _INF)
    lb_set = np.zeros(n, dtype=bool)
    for t, j, v, lineno in bounds:
        if t in ("UP", "UI"):
            ub[j] = v
            if v < 0 and not lb_set[j] and lb[j] == 0.0:
                lb[j] = -_INF
        elif t in ("LO", "LI"):
            lb[j] = v
            lb_set[j] = True
        elif t == "FX":
            lb[j] = ub[j] = v
            lb_set[j] = True
        elif t == "FR":
            lb[j], ub[j] = -_INF, _INF
            lb_set[j] = True
        elif t == "MI":
            lb[j] = -_INF
            lb_set[j] = True
        elif t == "PL":
            ub[j] = _INF
        elif t == "BV":
            lb[j], ub[j] = 0.0, 1.0
            lb_set[j] = True
            integer.add(j)
        elif t == "SC":
            ub[j] = v
    # constraint rows -> (coefficient row, sense, rhs) in the solver's form
    by_row = {}
    for (r, j), v in entries.items():
        by_row.setdefault(r, []).append((j, v))
    eq_rows, ineq_rows = [], []   # (list of (j, v), rhs, source row name, sign)
    for r in row_order:
        t = row_type[r]
        a = sorted(by_row.get(r, []))
        b = rhs.get(r, 0.0)
        if r in ranges:
            rv = ranges[r]
            if t == "E":
                lo, hi = (b, b + rv) if rv >= 0 else (b + rv, b)
            elif t == "L":
                lo, hi = b - abs(rv), b
            else:
                lo, hi = b, b + abs(rv)
        elif t == "E":
            lo = hi = b
        elif t == "L":
            lo, hi = -_INF, b
        else:
            lo, hi = b, _INF
        if lo == hi:
            eq_rows.append((a, lo, r, 1.0))
            continue
        if math.isfinite(lo):
            ineq_rows.append((a, lo, r, 1.0))
        if math.isfinite(hi):
            ineq_rows.append(([(j, -v) for j, v in a], -hi, r, -1.0))
    rows = eq_rows + ineq_rows
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    cols, vals = [], []
    for i, (a, _, _, _) in enumerate(rows):
        for j, v in a:
            cols.append(j)
            vals.append(v)
        rowptr[i + 1] = len(cols)
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("more than 2^31 - 1 nonzeros")
    c = np.zeros(n)
    for j, v in obj.items():
        c[j] = v
    c *= objsense
    meta = dict(name=name, objsense=objsense, obj_constant=obj_constant,
                col_names=col_names, row_source=[(r, s) for _, _, r, s in rows],
                integer=sorted(integer))
    return MPSModel(n, len(eq_rows), len(ineq_rows), rowptr.astype(np.int32),
                    np.asarray(cols, dtype=np.int32), np.asarray(vals, dtype=np.float64),
                    c, np.asarray([b for _, b, _, _ in rows], dtype=np.float64), lb, ub, meta)


def read(path: str) -> MPSModel:
    """Reads an .mps (or .mps.gz) file."""
    opener = gzip.open if path.endswith(".gz") else open
    with opener(path, "rt") as fh:
        return parse(fh.read(), name=path)
