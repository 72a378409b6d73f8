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
    ks = ["void drts::(anonymous namespace)::%s(args)" % k for k in bench.STEP_KERNELS]
    calib = "void at::native::%s<...>(args)" % bench.CALIB_KERNEL
    gib_kib = bench.CALIB_BYTES / 1024.0
    fetch = [1000.0, 10.0, 5.0, 1.0]
    write = [50.0, 4.0, 2.0, 0.0]
    # the copy kernel reads 1 GiB and writes 1 GiB; its FETCH_SIZE reads half;
    # the first kernel has two dispatches (1x and 3x its value: mean 2x)
    frows = [(ks[0], fetch[0]), (ks[0], 3 * fetch[0])] + [(k, v) for k, v in zip(ks[1:], fetch[1:])]
    wrows = [(ks[0], write[0]), (ks[0], 3 * write[0])] + [(k, v) for k, v in zip(ks[1:], write[1:])]
    _counters(tmp_path / "f.csv", "FETCH_SIZE", frows + [(calib, gib_kib / 2), ("other", 7.0)])
    _counters(tmp_path / "w.csv", "WRITE_SIZE", wrows + [(calib, gib_kib)])
    t = bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    want_f = [2 * fetch[0]] + fetch[1:]        # per-dispatch means
    want_w = [2 * write[0]] + write[1:]
    assert t["fetch_kib"] == dict(zip(bench.STEP_KERNELS, want_f))
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["bytes_per_launch"] == sum(want_f) * 1024 * 2 + sum(want_w) * 1024
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
    36 (+ a bit) per group; listed rows cost what the CSR costs, two-voxel
    rows their values and 16 bytes of info."""
    n_vox = 1000
    R = 26 * n_vox + 2000            # states and escape rows
    n_states = 26 * n_vox
    nnz = 26 * R
    csr = bench.spmv_bytes(nnz, R, n_states)
    g = {"n_groups": n_vox + 100, "n_fast": n_vox + 100, "n_vox2_rows": 0, "n_list_rows": 0, "n_list_entries": 0}
    fast = bench.grouped_bytes(R, n_states, g)
    assert fast == csr - 4 * nnz - 4 * (R + 1) + 5 * R + 36 * (n_vox + 100) + (n_vox + 100 + 7) // 8
    # 10 more rows of 40 entries in the row list
    slow = bench.grouped_bytes(R + 10, n_states, dict(g, n_list_rows=10, n_list_entries=400))
    assert slow - fast == 4 * 10 + 8 * 400 + 9 * 10
    # 7 more two-voxel rows
    v2 = bench.grouped_bytes(R + 7, n_states, dict(g, n_vox2_rows=7))
    assert v2 - fast == 4 * 7 + (4 * 52 + 16) * 7
    # value-indexed fast groups: a 32-byte slot (indices and row) and the
    # material a member, 16 bytes and a bit a group
    vi = bench.grouped_bytes(R, n_states, dict(g, value_tables=3))
    n_g = n_vox + 100
    assert fast - vi == (104 + 5 - 33) * R + (36 - 16) * n_g



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
