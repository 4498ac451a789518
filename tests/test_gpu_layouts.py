"""The layout builders on the GPU.  The explicit transpose K~^T that the
solver builds for the K^T y product (a stable radix sort of K~'s entries by
column) equals SciPy's transpose of the stored K~ bit for bit: row pointers,
column order within each row and values.  Cases: several radix tiles and a
ragged last tile, sort keys of one to three 8-bit digits, a dense column
(many equal keys: order within a column must follow the rows), empty rows
and columns, a single entry.  The stored K~ keeps the input's sparsity
pattern.  Column-sorted layouts (also built by the radix sort) are covered by
the parity tests that compare them with row order."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen

pytestmark = pytest.mark.gpu

halp = pytest.importorskip("paper_2407_16144_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

ROW_ORDER = dict(plain_sort=0, slice_sort=0, slice_min_bytes=-1)


def _dense_column_lp(seed, m=6000, n=300):
    """Every row holds column 0 and up to 4 others; some rows and columns are
    empty."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        if i % 97 == 5:
            continue
        rows.append(i)
        cols.append(0)
        for j in rng.choice(np.arange(1, n - 3), size=rng.integers(0, 5), replace=False):
            rows.append(i)
            cols.append(int(j))
    a = sp.csr_matrix((rng.uniform(0.5, 2.0, len(rows)), (rows, cols)), shape=(m, n))
    a.sort_indices()
    return lpgen.LP(n=n, m_eq=m // 2, m_ineq=m - m // 2, rowptr=a.indptr.astype(np.int32),
                    col=a.indices.astype(np.int32), val=a.data, c=rng.normal(size=n), rhs=rng.normal(size=m),
                    lb=np.zeros(n), ub=np.full(n, 10.0))


def _single_entry_lp():
    return lpgen.LP(n=3, m_eq=1, m_ineq=0, rowptr=np.array([0, 1], np.int32), col=np.array([2], np.int32),
                    val=np.array([1.5]), c=np.array([1.0, 0.0, -1.0]), rhs=np.array([1.0]),
                    lb=np.zeros(3), ub=np.ones(3))


CASES = {
    "powerlaw 3k x 9k": lambda: lpgen.scaled_powerlaw(11, 3000, 9000),
    "powerlaw 40k x 200k": lambda: lpgen.scaled_powerlaw(12, 40000, 200000),
    "dense column": lambda: _dense_column_lp(13),
    "single entry": _single_entry_lp,
}


@pytest.mark.parametrize("name", list(CASES))
def test_transpose_equals_scipy(name):
    lp = CASES[name]()
    print(f"case transpose {name} m={lp.m} n={lp.n} nnz={lp.nnz}", flush=True)
    h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub,
                       opt=halp.lp_default_options(**ROW_ORDER))
    try:
        rp, ci, v = halp.lp_get_scaled_matrix(h, 0, lp.m, lp.nnz)
        rpt, cit, vt = halp.lp_get_scaled_matrix(h, 1, lp.n, lp.nnz)
    finally:
        halp.lp_destroy(h)
    # K~ = D1 K D2 keeps the input's pattern
    assert np.array_equal(rp, lp.rowptr) and np.array_equal(ci, lp.col)
    assert np.all(np.isfinite(v)) and np.all(np.sign(v) == np.sign(lp.val))
    ref = sp.csr_matrix((v, ci, rp), shape=(lp.m, lp.n)).T.tocsr()
    ref.sort_indices()
    assert np.array_equal(rpt, ref.indptr)
    assert np.array_equal(cit, ref.indices)
    assert np.array_equal(vt.view(np.uint64), ref.data.view(np.uint64))


def test_sorted_layout_refuses_readback():
    """A product kept in a column-sorted layout cannot be read in row order."""
    lp = lpgen.scaled_powerlaw(14, 3000, 9000)
    print("case sorted readback", flush=True)
    h = halp.lp_create(lp.n, lp.m_eq, lp.m_ineq, lp.rowptr, lp.col, lp.val, lp.c, lp.rhs, lp.lb, lp.ub,
                       opt=halp.lp_default_options(slice_sort=1, plain_sort=1, sort_rows=256))
    try:
        with pytest.raises(halp.HalpError) as ei:
            halp.lp_get_scaled_matrix(h, 0, lp.m, lp.nnz)
        assert ei.value.code == halp.LP_ERR_STATE
    finally:
        halp.lp_destroy(h)
