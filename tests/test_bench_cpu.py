"""Host logic of the benchmark: the HBM traffic figure from two rocprofv3
counter passes, and the rule that a committed figure counts only for the
kernel sources it was taken on."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counters(path, counter, rows):
    """A counter_collection.csv with (kernel, value in KiB) rows."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, v) in enumerate(rows):
            w.writerow([i, k, counter, v])


def test_traffic_scales_each_counter_by_the_copy_kernel(bench, tmp_path):
    k0, k1, k2 = ("void drts::(anonymous namespace)::%s(args)" % k for k in bench.STEP_KERNELS)
    calib = "void at::native::%s<...>(args)" % bench.CALIB_KERNEL
    gib_kib = bench.CALIB_BYTES / 1024.0
    # the copy kernel reads 1 GiB and writes 1 GiB; its FETCH_SIZE reads half
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [(k0, 1000.0), (k0, 3000.0), (k1, 10.0), (k2, 1.0),
                                                 (calib, gib_kib / 2), ("other", 7.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [(k0, 50.0), (k0, 150.0), (k1, 4.0), (k2, 0.0), (calib, gib_kib)])
    t = bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert t["fetch_kib"] == {bench.STEP_KERNELS[0]: 2000.0, bench.STEP_KERNELS[1]: 10.0,
                              bench.STEP_KERNELS[2]: 1.0}      # per-dispatch means
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["bytes_per_launch"] == (2000.0 + 10.0 + 1.0) * 1024 * 2 + (100.0 + 4.0) * 1024
    assert t["source_sha256"] == bench.step_source_hash()


def test_traffic_needs_both_kernels(bench, tmp_path):
    _counters(tmp_path / "f.csv", "FETCH_SIZE", [("other", 1.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", [("other", 1.0)])
    with pytest.raises(SystemExit):
        bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))


def test_committed_traffic_counts_only_for_its_sources(bench, tmp_path, monkeypatch):
    good = {"bytes_per_launch": 123.0, "source_sha256": bench.step_source_hash()}
    stale = dict(good, source_sha256="0" * 16)
    for d, expect in ((good, 123.0), (stale, None)):
        p = tmp_path / "traffic.txt"
        p.write_text("# header\n" + json.dumps(d) + "\n")
        monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
        assert bench.load_traffic() == expect
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.load_traffic() is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_grouped_bytes_against_the_csr_count(bench):
    """With every row in a fast group the format's bytes are the CSR count
    minus the columns (4 per entry) and the row pointers, plus 5 per row and
    36 (+ a bit) per group; rows taken one by one cost what the CSR costs."""
    n_vox = 1000
    R = 26 * n_vox + 2000            # states and escape rows
    n_states = 26 * n_vox
    nnz = 26 * R
    csr = bench.spmv_bytes(nnz, R, n_states)
    fast = bench.grouped_bytes(R, n_states, n_vox + 100, n_vox + 100, 0, 0)
    assert fast == csr - 4 * nnz - 4 * (R + 1) + 5 * R + 36 * (n_vox + 100) + (n_vox + 100 + 7) // 8
    # moving 10 rows of 40 entries from the groups to the row list
    slow = bench.grouped_bytes(R + 10, n_states, n_vox + 100, n_vox + 100, 10, 400)
    assert slow - fast == 4 * 10 + 8 * 400 + 9 * 10


def test_traffic_by_kernel_names_and_scales(bench, tmp_path):
    """Every kernel of the passes, by its short name, scaled by its pass's
    calibration kernel; the calibration kernel itself is not listed."""
    for counter, fn, calib in (("FETCH_SIZE", "f.csv", 0.5), ("WRITE_SIZE", "w.csv", 1.0)):
        with open(tmp_path / fn, "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for v in (1000000, 3000000):
                w.writerow({"Kernel_Name": "void drts::(anonymous namespace)::step_struct_dm<2>(drts::StructArgs)",
                            "Counter_Name": counter, "Counter_Value": str(v)})
            w.writerow({"Kernel_Name": bench.CALIB_KERNEL + "<float>(x)", "Counter_Name": counter,
                        "Counter_Value": str(bench.CALIB_BYTES / 1024 * calib)})
    out = bench.traffic_by_kernel(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert out["_fetch_factor"] == 2.0 and out["_write_factor"] == 1.0
    k = out["step_struct_dm<2>"]
    assert k["fetch_GB"] == round(2e6 * 1024 * 2 / 1e9, 4) and k["write_GB"] == round(2e6 * 1024 / 1e9, 4)
    assert set(out) == {"step_struct_dm<2>", "_fetch_factor", "_write_factor"}
