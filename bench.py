#!/usr/bin/env python3
"""Benchmark of the DRTS time step on one MI355X.

Workload (the one the headline metric is quoted on): 128^3 voxels x 26
directions, three planar layers with Fresnel interfaces, FP32 CSR values and
state, Gaussian 100 fs source on the top face, two face detectors.  A step is
one pass of the hot path: SpMV over [A; L] with the fused rescale, source
injection, FP64 totals and detector sums, plus the finalize reduction.  The
matrix is assembled on the device before the timed region; inputs are
resident in HBM when timing starts.

Prints one JSON line.  --gpus above 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
STEP_SOURCES = ("paper_1611_08536_amd/csrc/drts_step.hip", "paper_1611_08536_amd/csrc/drts_step.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_spmv_c2_traffic.txt")
SPMV_KERNEL = "step_spmv<float, int, 256, 256, 0>"
CALIB_KERNEL = "vectorized_elementwise_kernel"
CALIB_BYTES = 2 ** 30          # the calibration kernel reads and writes 1 GiB


def step_source_hash():
    """sha256 of the step kernel sources: counters taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def _counter_means(path, counter):
    """Mean per-dispatch value of one counter, by kernel name, from a rocprofv3
    counter_collection.csv (values in KiB for FETCH_SIZE and WRITE_SIZE)."""
    import csv
    sums = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"]
        a = sums.setdefault(k, [0.0, 0])
        a[0] += float(r["Counter_Value"])
        a[1] += 1
    return {k: v[0] / v[1] for k, v in sums.items()}


def traffic_from_counters(fetch_csv, write_csv):
    """HBM bytes per launch of the SpMV step from the FETCH_SIZE and WRITE_SIZE
    passes, each scaled by what the same counter reads for a plain elementwise
    kernel that reads and writes CALIB_BYTES."""
    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        m = _counter_means(path, "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE")
        spmv = [v for k, v in m.items() if SPMV_KERNEL in k]
        calib = [v for k, v in m.items() if CALIB_KERNEL in k]
        if len(spmv) != 1 or not calib:
            raise SystemExit("counter file %s lacks the step or the calibration kernel" % path)
        factor = CALIB_BYTES / (max(calib) * 1024.0)
        out[name + "_kib"] = spmv[0]
        out[name + "_factor"] = round(factor, 4)
        out[name + "_bytes"] = spmv[0] * 1024.0 * factor
    out["bytes_per_launch"] = out["fetch_bytes"] + out["write_bytes"]
    out["kernel"] = SPMV_KERNEL
    out["source_sha256"] = step_source_hash()
    return out


def load_traffic():
    """Traffic of the committed counter summary, or None when it is missing or
    was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    line = [ln for ln in open(TRAFFIC_FILE).read().splitlines() if ln.startswith("{")]
    if not line:
        return None
    d = json.loads(line[-1])
    if d.get("source_sha256") != step_source_hash():
        return None
    return d["bytes_per_launch"]


def spmv_bytes(nnz, n_rows, n_states, val_bytes=4):
    """Algorithmic bytes of one SpMV step over [A; L]: values and columns once,
    row pointers once, x once, y once."""
    return val_bytes * nnz + 4 * nnz + 4 * (n_rows + 1) + val_bytes * n_states + val_bytes * n_rows


def cpu_baseline(n=64, steps=40):
    """The FP64 oracle (as it stands) on the host cores: one bounded sample of
    the same layered workload at a smaller edge, timed per step."""
    import oracle
    import workloads as W
    wl = W.c2(n=n, n_steps=steps)
    A = oracle.Matrix(wl.medium)
    t0 = time.perf_counter()
    oracle.run_workload(A, wl, n_steps=steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(A.nnz * steps / dt / 1e9, 4), "unit": "GNNZ/s", "cores": threads,
            "kind": "oracle",
            "sample": "C2 layered medium at %d^3 (%d nnz), %d FP64 steps, %.1f s" % (n, A.nnz, steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=128, help="grid edge (128 = the headline workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, launch an elementwise kernel that reads and writes 1 GiB (counter scale)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="print the traffic JSON line from two rocprofv3 --pmc counter files and exit")
    args = ap.parse_args()
    if args.traffic_from:
        print(json.dumps(traffic_from_counters(*args.traffic_from)))
        return
    if args.gpus != 1:
        print("the step runs on one GPU: --gpus %d is not supported (a multi-GPU run would give "
              "each GPU its own slab of voxels and exchange halo planes)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1611_08536_amd import drts, solve

    torch.cuda.set_device(0)
    total = args.warmup + args.steps
    wl = W.c2(n=args.n, n_steps=total)
    print("bench: assembling %d^3 layered medium" % args.n, file=sys.stderr, flush=True)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(A, 1, wl.detectors, max_steps=total)
    tab = solve.source_table(A, wl)
    S.run(tab, args.warmup)
    torch.cuda.synchronize()

    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    S.profile(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    S.run(tab, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    launches, kernel_ms = S.profile_stats()
    S.profile(False)
    ms_step = ms_total / args.steps
    avg_kernel_ms = kernel_ms / max(launches, 1)

    r = S.readout(0, total)
    assert (r["tot"][:, 0, 0] > 0).all()

    nbytes = spmv_bytes(A.nnz, A.n_rows, A.n_states)
    achieved = nbytes / (avg_kernel_ms * 1e-3) / 1e9
    traffic = load_traffic()
    if args.copy_calibration:
        a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    line = {
        "metric": "DRTS step GNNZ/s & % HBM peak; batched solves/s + p99 latency vs plain",
        "value": round(A.nnz * args.steps / (ms_total * 1e-3) / 1e9, 3),
        "unit": "GNNZ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C2: %d^3 voxels x 26 directions, 3 Fresnel layers, FP32 CSR [A;L], "
                               "Gaussian 100 fs top-face source, 2 detectors" % args.n,
                   "n_states": A.n_states, "n_rows": A.n_rows, "nnz": A.nnz, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None if traffic is None else round(traffic / 1e9, 3),
                     "kernel": "step_spmv<float,int32>", "kernel_ms": round(avg_kernel_ms, 4),
                     "algorithmic_bytes": nbytes, "traffic_unit": "GB per launch"},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
