"""Host-side helpers: the rocprofv3 counter summary and the benchmark's byte
accounting (CPU only)."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(name, path):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


rs = _load("rocprof_summary", os.path.join(ROOT, "paper_2407_16144_amd", "rocprof_summary.py"))
bench = _load("bench_mod", os.path.join(ROOT, "bench.py"))

HDR = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(HDR)
        for i, (k, v) in enumerate(rows):
            w.writerow([i, i, k, counter, v])


def test_counter_scaling(tmp_path):
    step = "void halp::primal_step<double>(halp::IterArgs<double>, int)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>(int)"
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 1000.0), (copy, 1000.0), (step, 10.0), (step, 30.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 500.0), (step, 4.0)])
    t = rs.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "neg_kernel", 2048000.0)
    assert t["scale_fetch"] == pytest.approx(2.0)
    assert t["scale_write"] == pytest.approx(4.0)
    k = t["kernels"]["primal_step<double>"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == pytest.approx(20 * 1024 * 2.0)
    assert k["write_bytes"] == pytest.approx(4 * 1024 * 4.0)
    assert k["traffic_bytes"] == pytest.approx(20 * 2048 + 4 * 4096)
    assert "primal_step<double>" in rs.traffic_table(t)


def test_short_names():
    assert rs.short_name('"void halp::dual_slice_step<float>(halp::IterArgs<float>, int)"') == \
        "dual_slice_step<float>"
    assert rs.short_name("halp::tick_kernel(long*, long)") == "tick_kernel"


def test_kernel_bytes_split():
    n, m, nnz, s = 1000, 300, 5000, 8
    p, d = bench.algorithmic_bytes(n, m, nnz, s)
    plain = bench.kernel_bytes(n, m, nnz, s, False, False)
    assert plain["primal_slice"] == plain["dual_slice"] == 0
    assert plain["primal_step"] == p and plain["dual_step"] == d
    sl = bench.kernel_bytes(n, m, nnz, s, True, True)
    # slicing moves the matrix and gather bytes to the slice kernels, nothing is lost
    assert sl["primal_slice"] + sl["primal_step"] == p
    assert sl["dual_slice"] + sl["dual_step"] == d
    assert sl["dual_step"] == 4 * s * m and sl["primal_step"] == 7 * s * n
    # sorted groups drop the row pointers of both products (packed into the column index)
    so = bench.kernel_bytes(n, m, nnz, s, True, True, True)
    assert so["dual_slice"] == sl["dual_slice"] - 4 * (m + 1)
    assert so["primal_slice"] == sl["primal_slice"] - 4 * (n + 1)
    assert so["dual_step"] == sl["dual_step"] and so["primal_step"] == sl["primal_step"]
    # products without a slice kernel: sorted groups do not apply; sorted plain blocks do
    assert bench.kernel_bytes(n, m, nnz, s, False, False, True) == plain
    ps = bench.kernel_bytes(n, m, nnz, s, False, False, False, True)
    assert ps["primal_step"] == p - 4 * (n + 1) and ps["dual_step"] == d - 4 * (m + 1)


def test_measured_traffic_lookup(tmp_path, monkeypatch):
    """The benchmark reads a kernel's HBM bytes from the committed counter
    summary only while the kernel sources are unchanged, and names a kernel
    by the prefix of its templated name."""
    import json
    prof = tmp_path / "profiles"
    prof.mkdir()
    good = {"source_sha256": rs.kernel_source_hash(),
            "kernels": {"sorted_group_step<double, true, 512, true>": {"traffic_bytes": 381.4e6},
                        "sorted_group_step<double, false, 512, true>": {"traffic_bytes": 378.6e6},
                        "dual_step<double>": {"traffic_bytes": 50.4e6}}}
    (prof / "traffic_w.json").write_text(json.dumps(good))
    (prof / "traffic_old.json").write_text(json.dumps({**good, "source_sha256": "0" * 64}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "sorted_group_step<double, true") == 381400000
    assert bench.measured_traffic("w", "dual_step") == 50400000
    assert bench.measured_traffic("w", "sorted_group_step<double") is None     # two kernels match
    assert bench.measured_traffic("old", "dual_step") is None                  # sources changed since
    assert bench.measured_traffic("none", "dual_step") is None                 # no summary
