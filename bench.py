#!/usr/bin/env python3
"""Benchmark of the DRTS time step on one MI355X.

Workload (the one the headline metric is quoted on): 128^3 voxels x 26
directions, three planar layers with Fresnel interfaces, FP32 CSR values and
state, Gaussian 100 fs source on the top face, two face detectors.  A step is
one pass of the hot path: SpMV over [A; L] with the fused rescale, source
injection, FP64 totals and detector sums, plus the finalize reduction.  The
matrix is assembled on the device before the timed region; inputs are
resident in HBM when timing starts.

Prints one JSON line.  --gpus above 1 exits: the step runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
F64SUM_NOTE = ("FP32 values and state, each row summed in FP64 and rounded once: outside the "
               "FP32-accumulation precision pattern (more accurate than it)")
STEP_SOURCES = ("paper_1611_08536_amd/csrc/drts_step.hip", "paper_1611_08536_amd/csrc/drts_step.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_spmv_grouped_c2_traffic.txt")
# the kernels of one headline step launch (the finalize aside): the fast
# groups, the row list, the two-voxel rows, the detector sums
STEP_KERNELS = ("step_spmv_grouped_vi", "step_spmv_rowlist", "step_spmv_vox2", "spmv_detectors")
CALIB_KERNEL = "vectorized_elementwise_kernel"
CALIB_BYTES = 2 ** 30          # the calibration kernel reads and writes 1 GiB
GRAPH_STEPS = 50               # steps per hipGraph replay in the timed run


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
    """HBM bytes per headline step launch (the STEP_KERNELS, per-dispatch means
    added) from the FETCH_SIZE and WRITE_SIZE passes, each scaled by what the
    same counter reads for a plain elementwise kernel that reads and writes
    CALIB_BYTES."""
    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        m = _counter_means(path, "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE")
        per = {}
        for kern in STEP_KERNELS:
            hits = [v for k, v in m.items() if kern + "(" in k or kern + "<" in k]
            if len(hits) != 1:
                raise SystemExit("counter file %s: %d entries for %s" % (path, len(hits), kern))
            per[kern] = hits[0]
        calib = [v for k, v in m.items() if CALIB_KERNEL in k]
        if not calib:
            raise SystemExit("counter file %s lacks the calibration kernel" % path)
        factor = CALIB_BYTES / (max(calib) * 1024.0)
        out[name + "_kib"] = {k: round(v, 2) for k, v in per.items()}
        out[name + "_factor"] = round(factor, 4)
        out[name + "_bytes"] = sum(per.values()) * 1024.0 * factor
    out["bytes_per_launch"] = out["fetch_bytes"] + out["write_bytes"]
    out["kernel"] = " + ".join(STEP_KERNELS)
    out["source_sha256"] = step_source_hash()
    return out


def traffic_by_kernel(fetch_csv, write_csv):
    """Per-kernel HBM GB per dispatch (mean over the dispatches of each kernel
    name) from a FETCH_SIZE and a WRITE_SIZE pass, each scaled by the
    calibration kernel of its pass; kernels of fewer than 1 MB are left out."""
    out, factors = {}, {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        m = _counter_means(path, "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE")
        calib = [v for k, v in m.items() if CALIB_KERNEL in k]
        if not calib:
            raise SystemExit("counter file %s lacks the calibration kernel" % path)
        factors[name] = CALIB_BYTES / (max(calib) * 1024.0)
        for k, v in m.items():
            if CALIB_KERNEL in k:
                continue
            short = k.replace("drts::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            out.setdefault(short, {})[name + "_GB"] = round(v * 1024.0 * factors[name] / 1e9, 4)
    out = {k: v for k, v in out.items() if v.get("fetch_GB", 0) + v.get("write_GB", 0) >= 1e-3}
    out["_fetch_factor"] = round(factors["fetch"], 4)
    out["_write_factor"] = round(factors["write"], 4)
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
    """Algorithmic bytes of one SpMV step over [A; L] held as CSR: values and
    columns once, row pointers once, x once, y once."""
    return val_bytes * nnz + 4 * nnz + 4 * (n_rows + 1) + val_bytes * n_states + val_bytes * n_rows


def grouped_bytes(n_rows, n_states, g):
    """Bytes the step by row groups must move (g: the matrix's groups info).
    Members of fast groups (26 entries a row): their values in group order
    (4 per entry), row id (4) and material (1), per fast group its
    descriptor (32), list entry (4) and source bit; value-indexed, a 32-byte
    slot (indices and row) and the material (1) per member, 16 per group and
    its source bit.  Two-voxel rows: their
    52 values (4 each) and their info (16).  Listed rows: their CSR entries
    (8 per entry), row pointer (4), material (1) and list entry (4).  x once,
    y once."""
    fast_rows = n_rows - g["n_vox2_rows"] - g["n_list_rows"]
    if g.get("value_tables", 0) > 0:
        # a 32-byte slot per member (26 one-byte indices, the dictionary's
        # number, the brick position, the member's row) and its material; a
        # 16-byte descriptor per fast group and its source bit
        fast = 33 * fast_rows + 16 * g["n_fast"] + (g["n_fast"] + 7) // 8
    else:
        fast = 4 * 26 * fast_rows + 5 * fast_rows + 36 * g["n_fast"] + (g["n_groups"] + 7) // 8
    vox2 = (4 * 52 + 16) * g["n_vox2_rows"]
    listed = 8 * g["n_list_entries"] + 9 * g["n_list_rows"]
    return fast + vox2 + listed + 4 * n_states + 4 * n_rows


def cpu_baseline(n=128, steps=50, steps_1=3):
    """The FP64 oracle (as it stands) on the host cores: a bounded sample of the
    same workload (the first `steps` steps of the 128^3 layered medium), timed
    after its assembly."""
    import oracle
    import workloads as W
    wl = W.c2(n=n, n_steps=steps)
    A = oracle.Matrix(wl.medium)
    t0 = time.perf_counter()
    oracle.run_workload(A, wl, n_steps=steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the same oracle on one thread, over the first steps_1 steps
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run_workload(A, wl, n_steps=steps_1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": round(A.nnz * steps / dt / 1e9, 4), "unit": "GNNZ/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d of the 2000 FP64 steps of the %d^3 layered workload (%d nnz), %.1f s" %
                      (steps, n, A.nnz, dt),
            "value_1_thread": round(A.nnz * steps_1 / dt1 / 1e9, 4),
            "sample_1_thread": "first %d steps, %.1f s" % (steps_1, dt1)}


def _log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def _timed(fn, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def spmm_vs_plain(torch, steps=20):
    """C3: 96^3 homogeneous slab, 64 right-hand sides (one source voxel each),
    16 FP64 detectors.  SpMM steps of all 64 against plain single-rhs steps of
    the same matrix (64 plain runs take 64 times the single run's time)."""
    import copy
    import workloads as W
    from paper_1611_08536_amd import drts, solve
    wl = W.c3(n_steps=steps + 4)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(A, wl.n_rhs, wl.detectors, max_steps=3 * steps + 12)
    tab = solve.source_table(A, wl)
    S.run(tab, 2)
    S.profile(True)
    t_mm = _timed(lambda: S.run(tab, steps), torch)
    n_l, k_ms = S.profile_stats()
    # the same step with FP64 row sums
    S.set_options(variant=drts.SPMM_GROUPED_F64SUM)
    S.run(tab, 2)
    S.profile(True)
    t_s64 = _timed(lambda: S.run(tab, steps), torch)
    n_s, s_ms = S.profile_stats()
    # the matrix-free many-rhs step (FP64 row sums) on the same solver
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    S.set_options(kernel=drts.KERNEL_STRUCTURED_F64SUM, variant=drts.SPMM_GROUPED, grid=16 * cus)
    S.run(tab, 2)
    S.profile(True)
    t_mf = _timed(lambda: S.run(tab, steps), torch)
    n_f, f_ms = S.profile_stats()
    S.close()
    w1 = copy.copy(wl)
    w1.sources = [copy.copy(x) for x in wl.sources if x.rhs == 0]
    for x in w1.sources:
        x.rhs = 0
    w1.n_rhs = 1
    S1 = drts.Solver(A, 1, wl.detectors, max_steps=steps + 4)
    tab1 = solve.source_table(A, w1)
    S1.run(tab1, 2)
    t_1 = _timed(lambda: S1.run(tab1, steps), torch)
    S1.close()
    k = wl.n_rhs
    nbytes = 8 * A.nnz + 4 * (A.n_rows + 1) + 4 * k * A.n_states + 4 * k * A.n_rows
    kern_s = k_ms / max(n_l, 1) * 1e-3
    out = {"workload": "C3: 96^3 homogeneous, %d rhs, %d nnz, %d steps timed" % (k, A.nnz, steps),
           "solve_steps_per_s": round(k * steps / t_mm, 1),
           "plain_solve_steps_per_s": round(steps / t_1, 1),
           "speedup_vs_plain": round((k * steps / t_mm) / (steps / t_1), 2),
           "ms_per_step": round(t_mm / steps * 1e3, 3), "plain_ms_per_step": round(t_1 / steps * 1e3, 3),
           "kernel": "step_spmm_grouped<int32> + spmm_detectors", "kernel_ms": round(kern_s * 1e3, 3),
           "achieved_GBs": round(nbytes / kern_s / 1e9, 1), "frac": round(nbytes / kern_s / 1e9 / PEAK_HBM_GBS, 4)}
    mf_s = f_ms / max(n_f, 1) * 1e-3
    mf_bytes = 4 * k * A.n_states + 4 * k * A.n_rows + A.n_states // 26
    out["precision"] = "FP32 values, state and accumulation (CSR SpMM)"
    s64_s = s_ms / max(n_s, 1) * 1e-3
    out["f64sum"] = {"kernel": "step_spmm_grouped<int32, FP64 row sums, value-indexed> + spmm_detectors",
                     "precision": F64SUM_NOTE,
                     "ms_per_step": round(t_s64 / steps * 1e3, 3), "kernel_ms": round(s64_s * 1e3, 3),
                     "achieved_GBs": round(nbytes / s64_s / 1e9, 1),
                     "frac": round(nbytes / s64_s / 1e9 / PEAK_HBM_GBS, 4)}
    out["matrix_free"] = {"kernel": "step_struct_mm<2> + step_struct_mm_x<2> (FP64 row sums)",
                          "precision": F64SUM_NOTE,
                          "ms_per_step": round(t_mf / steps * 1e3, 3), "kernel_ms": round(mf_s * 1e3, 3),
                          "solve_steps_per_s": round(k * steps / t_mf, 1),
                          "speedup_vs_plain": round((k * steps / t_mf) / (steps / t_1), 2),
                          "algorithmic_bytes": mf_bytes, "achieved_GBs": round(mf_bytes / mf_s / 1e9, 1),
                          "frac": round(mf_bytes / mf_s / 1e9 / PEAK_HBM_GBS, 4)}
    A.close()
    # the exact matrix-free step (FP32 accumulation, equal to the CSR step bit
    # for bit) takes nearest-rounded values: the same slab assembled so
    torch.cuda.empty_cache()
    An = drts.Matrix(wl.medium, wl.value_type, "nearest", wl.n_ref)
    Sn = drts.Solver(An, wl.n_rhs, wl.detectors, max_steps=steps + 4)
    Sn.set_options(kernel=drts.KERNEL_STRUCTURED, grid=16 * cus)
    tabn = solve.source_table(An, wl)
    Sn.run(tabn, 2)
    Sn.profile(True)
    t_ex = _timed(lambda: Sn.run(tabn, steps), torch)
    n_x, x_ms = Sn.profile_stats()
    Sn.close()
    An.close()
    ex_s = x_ms / max(n_x, 1) * 1e-3
    out["matrix_free_exact"] = {"kernel": "step_struct_mm<1> + step_struct_mm_x<1> (nearest-rounded values)",
                                "precision": "FP32 values, state and accumulation (equal to the CSR step)",
                                "ms_per_step": round(t_ex / steps * 1e3, 3), "kernel_ms": round(ex_s * 1e3, 3),
                                "solve_steps_per_s": round(k * steps / t_ex, 1),
                                "speedup_vs_plain": round((k * steps / t_ex) / (steps / t_1), 2),
                                "achieved_GBs": round(mf_bytes / ex_s / 1e9, 1),
                                "frac": round(mf_bytes / ex_s / 1e9 / PEAK_HBM_GBS, 4)}
    return out


def batch_vs_sequential(torch, steps=40):
    """C4: 256 independent homogeneous cubes (edges 16..64), advanced together
    by one launch per step, against the same solvers stepped one after another."""
    import workloads as W
    from paper_1611_08536_amd import drts, solve
    wls = W.c4(n_steps=500)
    _log("C4: assembling %d media" % len(wls))
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, [], max_steps=2 * steps + 4) for m in mats]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    n_own = sum(m.n_rows >= drts.BATCH_OWN_ROWS for m in mats)
    _log("C4: autotuning the batch's launch shape")
    t0 = time.perf_counter()
    chosen = B.autotune()
    t_tune = time.perf_counter() - t0
    B.run(tabs, [2] * len(solvers))
    t_b = _timed(lambda: B.run(tabs, [steps] * len(solvers)), torch)
    B.close()
    for S in solvers:
        S.close()
    # the same media stepped one after another by fresh solvers with their
    # default step (by row groups)
    solvers = [drts.Solver(m, 1, [], max_steps=steps + 4) for m in mats]

    def seq():
        for S, t in zip(solvers, tabs):
            S.run(t, steps)
    for S, t in zip(solvers, tabs):
        S.run(t, 2)
    t_s = _timed(seq, torch)
    nnz = sum(m.nnz for m in mats)
    for S in solvers:
        S.close()
    # the same media with the matrix-free step (FP64 row sums, 8 tiles per
    # chunk): one batch (one launch per kernel and step), then one after another
    _log("C4: matrix-free batch")
    mf = {"kernel": drts.KERNEL_STRUCTURED_F64SUM, "tiles_per_chunk": 8}
    solvers = [drts.Solver(m, 1, [], max_steps=2 * steps + 4) for m in mats]
    for S in solvers:
        S.set_options(**mf)
    B = drts.Batch(solvers)
    B.run(tabs, [2] * len(solvers))
    t_mb = _timed(lambda: B.run(tabs, [steps] * len(solvers)), torch)
    B.close()
    t_ms = _timed(seq, torch)
    for S in solvers:
        S.close()
    for m in mats:
        m.close()
    # the exact matrix-free step (FP32 accumulation) on the same media with
    # nearest-rounded values, one batch
    _log("C4: exact matrix-free batch (nearest-rounded values)")
    torch.cuda.empty_cache()
    mats = [drts.Matrix(w.medium, w.value_type, "nearest", w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, [], max_steps=2 * steps + 4) for m in mats]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    for S in solvers:
        S.set_options(kernel=drts.KERNEL_STRUCTURED, tiles_per_chunk=8)
    B = drts.Batch(solvers)
    B.run(tabs, [2] * len(solvers))
    t_xb = _timed(lambda: B.run(tabs, [steps] * len(solvers)), torch)
    B.close()
    for S in solvers:
        S.close()
    for m in mats:
        m.close()
    n = len(wls)
    return {"workload": "C4: %d media, %d nnz in all, %d of the 500 steps timed" % (n, nnz, steps),
            "instance_steps_per_s": round(n * steps / t_b, 1),
            "sequential_instance_steps_per_s": round(n * steps / t_s, 1),
            "speedup_vs_sequential": round(t_s / t_b, 2),
            "solves_per_s": round(n * steps / t_b / 500, 3),
            "sequential_solves_per_s": round(n * steps / t_s / 500, 3),
            "GNNZ_per_s": round(nnz * steps / t_b / 1e9, 1),
            "batch_shape": "%d members of at least %d rows on their own grouped step, %d in the shared tiled "
                           "launch, its shape autotuned in %.1f s: %d rows per tile, %d tiles per chunk, variant %d, "
                           "%d workgroups" % (n_own, drts.BATCH_OWN_ROWS, n - n_own, t_tune, chosen["rows_per_tile"],
                                              chosen["tiles_per_chunk"], chosen["variant"], chosen["grid"]),
            "sequential": "fresh solvers with their default step (by row groups), one after another",
            "precision": "FP32 values, state and accumulation (CSR)",
            "matrix_free": {"kernel": "step_struct_dm<2, true> + step_struct_x<float, 2, true> (FP64 row sums)",
                            "precision": F64SUM_NOTE,
                            "instance_steps_per_s": round(n * steps / t_mb, 1),
                            "sequential_instance_steps_per_s": round(n * steps / t_ms, 1),
                            "speedup_vs_sequential": round(t_ms / t_mb, 2),
                            "cross_kernel_speedup_vs_csr_sequential": round(t_s / t_mb, 2),
                            "GNNZ_equiv_per_s": round(nnz * steps / t_mb / 1e9, 1)},
            "matrix_free_exact": {"kernel": "step_struct_dm<1, true> + step_struct_x<float, 0, true> "
                                            "(nearest-rounded values)",
                                  "precision": "FP32 values, state and accumulation (equal to the CSR step)",
                                  "instance_steps_per_s": round(n * steps / t_xb, 1),
                                  "cross_kernel_speedup_vs_csr_sequential": round(t_s / t_xb, 2),
                                  "GNNZ_equiv_per_s": round(nnz * steps / t_xb / 1e9, 1)}}


def serving_vs_fifo(torch, n_req=32, step_scale=0.1, kinds=("csr", "mf_f64sum", "mf_exact")):
    """C5 sample: the first n_req requests of the Poisson (200/s) stream of
    sphere-inclusion media (edges 32..128), step counts scaled by step_scale,
    through the serving loop and through sequential FIFO runs of the same
    step, for each step kind: the CSR step, the matrix-free step with FP64 row
    sums, and the exact matrix-free step (FP32 accumulation) on
    nearest-rounded requests."""
    import copy
    import workloads as W
    from paper_1611_08536_amd import drts, serve
    lo, hi = int(500 * step_scale), int(5000 * step_scale)
    reqs = W.c5(n_req=n_req, steps=(lo, hi))
    r = lambda d: {k: round(v, 4) if isinstance(v, float) else v for k, v in d.items()}
    out = {"workload": "C5%s: first %d requests, 200/s Poisson arrivals, edges 32..128, steps %d..%d" %
                       ("" if n_req == 256 and step_scale == 1.0 else " sample", n_req, lo, hi),
           "server": "least work first, at most 4 admitted, 50 steps per tick, budget 70% of free HBM"}
    step = {"csr": (drts.KERNEL_CSR, "FP32 values, state and accumulation (CSR)"),
            "mf_f64sum": (drts.KERNEL_STRUCTURED_F64SUM, F64SUM_NOTE),
            "mf_exact": (drts.KERNEL_STRUCTURED, "FP32 values, state and accumulation (equal to the CSR step); "
                                                 "nearest-rounded requests")}
    fifo_csr = None
    for kind in kinds:
        kernel, note = step[kind]
        rq = reqs
        if kind == "mf_exact":
            rq = [copy.copy(q) for q in reqs]
            for q in rq:
                q.workload = copy.copy(q.workload)
                q.workload.rounding = "nearest"
        torch.cuda.empty_cache()
        budget = serve.footprint_budget(0.7)
        _log("C5 %s: serving %d requests (budget %.1f GB)" % (kind, n_req, budget / 1e9))
        sv = serve.serve(rq, budget, quantum=50, max_active=4, policy="shortest", kernel=kernel,
                         log=_log if n_req > 64 else None)
        _log("C5 %s: FIFO runs of the same step" % kind)
        torch.cuda.empty_cache()
        ff = serve.fifo_plain(rq, kernel=kernel, log=_log if n_req > 64 else None)
        out[kind] = {"precision": note, "served": r(sv), "fifo": r(ff),
                     "speedup_solves_per_s": round(sv["solves_per_s"] / ff["solves_per_s"], 2)}
        if kind == "csr":
            fifo_csr = ff
        elif fifo_csr is not None:
            out[kind]["cross_kernel_speedup_vs_fifo_csr"] = round(sv["solves_per_s"] / fifo_csr["solves_per_s"], 2)
    return out


def lebedev_step(torch, n=64, steps=20):
    """The paper's own discretisation: Lebedev-86 directions with the
    multi-voxel weights of Eq. (18)-(19), a homogeneous n^3 cube (mu_s 10,
    mu_a 0.01, g 0.9), light path one voxel per step, FP32 values; rows of
    about 640 entries step with the wave-per-row SpMV."""
    import workloads as W
    from paper_1611_08536_amd import drts, solve
    med = W.homogeneous(n, W.C3_MAT)
    med.directions = "lebedev86"
    c = n // 2
    wl = W.Workload("lebedev", med, [W.point_source(c, c, 0)], [], steps + 4, 1, "f32", "dither", 1.4)
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = drts.Matrix(med, "f32", "dither", 1.4)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    S = drts.Solver(A, 1, [], max_steps=2 * steps + 4)
    tab = solve.source_table(A, wl)
    S.run(tab, 2)
    t = _timed(lambda: S.run(tab, steps), torch)
    S.profile(True)
    S.run(tab, steps)
    n_l, k_ms = S.profile_stats()
    S.close()
    kern_s = k_ms / max(n_l, 1) * 1e-3
    nbytes = 8 * A.nnz + 8 * (A.n_rows + 1) + 4 * A.n_states + 4 * A.n_rows
    out = {"workload": "%d^3 homogeneous (10, 0.01, 0.9), Lebedev-86 directions, Eq. 18-19 weights, c dt = h, "
                       "FP32 CSR" % n,
           "n_rows": A.n_rows, "nnz": A.nnz, "entries_per_row": round(A.nnz / A.n_rows, 1),
           "assembly_s": round(t_asm, 3), "ms_per_step": round(t / steps * 1e3, 3),
           "GNNZ_per_s": round(A.nnz * steps / t / 1e9, 1), "kernel": "step_spmv_long<float, long>",
           "kernel_ms": round(kern_s * 1e3, 3), "algorithmic_bytes": nbytes,
           "roofline": {"bound": "hbm", "achieved": round(nbytes / kern_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(nbytes / kern_s / 1e9 / PEAK_HBM_GBS, 4)}}
    A.close()
    torch.cuda.empty_cache()
    return out


def medium_variant_step(torch, label, change, n=128, steps=20):
    """The 128^3 layered medium with one discretisation choice changed (same
    kernel): its assembly time and step rate."""
    import workloads as W
    from paper_1611_08536_amd import drts, solve
    wl = W.c2(n=n, n_steps=steps + 4)
    change(wl.medium)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    S = drts.Solver(A, 1, wl.detectors, max_steps=steps + 4)
    tab = solve.source_table(A, wl)
    S.run(tab, 2)
    t = _timed(lambda: S.run(tab, steps), torch)
    S.close()
    out = {"workload": "C2 medium, %s" % label, "nnz": A.nnz, "assembly_s": round(t_asm, 3),
           "ms_per_step": round(t / steps * 1e3, 4), "GNNZ_per_s": round(A.nnz * steps / t / 1e9, 1)}
    A.close()
    return out


def structured_step(torch, A, wl, tab, steps=50):
    """The matrix-free step (FP64 row sums) on the same 128^3 workload, and the
    exact matrix-free step on its nearest-rounded twin."""
    from paper_1611_08536_amd import drts, solve
    S = drts.Solver(A, 1, wl.detectors, max_steps=steps + 4)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    S.set_options(kernel=drts.KERNEL_STRUCTURED_F64SUM, tiles_per_chunk=8, grid=16 * cus)
    S.run(tab, 2)
    S.profile(True)
    t = _timed(lambda: S.run(tab, steps), torch)
    n_l, k_ms = S.profile_stats()
    S.close()
    kern_s = k_ms / max(n_l, 1) * 1e-3
    nbytes = 4 * A.n_states + 4 * A.n_rows + A.n_states // 26
    out = {"kernel": "step_struct_dm<2> + step_struct_x<float,2> (matrix-free, FP64 row sums)",
           "precision": F64SUM_NOTE,
           "ms_per_step": round(t / steps * 1e3, 4),
           "kernel_ms": round(kern_s * 1e3, 4), "GNNZ_equiv_per_s": round(A.nnz / kern_s / 1e9, 1),
           "algorithmic_bytes": nbytes, "achieved_GBs": round(nbytes / kern_s / 1e9, 1)}
    # the exact matrix-free step (FP32 accumulation, equal to the CSR step bit
    # for bit) on the same medium with nearest-rounded values
    An = drts.Matrix(wl.medium, wl.value_type, "nearest", wl.n_ref)
    Sn = drts.Solver(An, 1, wl.detectors, max_steps=steps + 4)
    Sn.set_options(kernel=drts.KERNEL_STRUCTURED, tiles_per_chunk=8, grid=16 * cus)
    tabn = solve.source_table(An, wl)
    Sn.run(tabn, 2)
    Sn.profile(True)
    tn = _timed(lambda: Sn.run(tabn, steps), torch)
    n_x, x_ms = Sn.profile_stats()
    Sn.close()
    An.close()
    ex_s = x_ms / max(n_x, 1) * 1e-3
    out["exact"] = {"kernel": "step_struct_dm<1> + step_struct_x<float,0> (nearest-rounded values)",
                    "precision": "FP32 values, state and accumulation (equal to the CSR step)",
                    "ms_per_step": round(tn / steps * 1e3, 4), "kernel_ms": round(ex_s * 1e3, 4),
                    "GNNZ_equiv_per_s": round(A.nnz / ex_s / 1e9, 1),
                    "achieved_GBs": round(nbytes / ex_s / 1e9, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=128, help="grid edge (128 = the headline workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the SpMM, batch, serving and matrix-free measurements")
    ap.add_argument("--struct-only", action="store_true",
                    help="of the extra measurements, run only the matrix-free step (for profiling)")
    ap.add_argument("--spmm-only", action="store_true",
                    help="of the extra measurements, run only the 64-rhs steps (for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="of the extra measurements, run only the uneven batch of 256 media (for profiling)")
    ap.add_argument("--lebedev-only", action="store_true",
                    help="of the extra measurements, run only the Lebedev-86 step (for profiling)")
    ap.add_argument("--serving-full", action="store_true",
                    help="only the serving loop on all 256 requests of C5 with their full step counts, "
                         "matrix-free server against FIFO plain runs (about 15 minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, launch an elementwise kernel that reads and writes 1 GiB (counter scale)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="print the traffic JSON line from two rocprofv3 --pmc counter files and exit")
    ap.add_argument("--traffic-by-kernel", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="print every kernel's HBM GB per dispatch from two rocprofv3 --pmc counter files and exit")
    args = ap.parse_args()
    if args.traffic_by_kernel:
        print(json.dumps(traffic_by_kernel(*args.traffic_by_kernel), indent=1))
        return
    if args.traffic_from:
        print(json.dumps(traffic_from_counters(*args.traffic_from)))
        return
    if args.gpus != 1:
        print("the step runs on one GPU: --gpus %d is not supported (a multi-GPU run would give "
              "each GPU its own slab of voxels and exchange halo planes)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.serving_full:
        print(json.dumps({"serving_full": serving_vs_fifo(torch, n_req=256, step_scale=1.0,
                                                          kinds=("mf_f64sum",))}), flush=True)
        return
    import workloads as W
    from paper_1611_08536_amd import drts, solve

    torch.cuda.set_device(0)
    prof_steps = min(args.steps, 200)
    total = args.warmup + args.steps + 2 * prof_steps
    wl = W.c2(n=args.n, n_steps=total)
    _log("assembling %d^3 layered medium" % args.n)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(A, 1, wl.detectors, max_steps=total + prof_steps)
    tab = solve.source_table(A, wl)
    # what ships: the default step (by row groups: the matrix's groups are
    # built at the first run, before the timed region), drts_run replaying
    # hipGraphs of GRAPH_STEPS steps, no per-launch events
    S.set_options(graph_steps=GRAPH_STEPS)
    S.run(tab, args.warmup)
    torch.cuda.synchronize()
    group_bytes = A.device_bytes() - A.bytes
    groups = A.groups()

    _log("timing %d steps (graph replay)" % args.steps)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    S.run(tab, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps

    # the step kernel's own duration: a separate pass with HIP events around
    # every launch (eager launches on the same stream)
    _log("kernel timing pass (%d steps)" % prof_steps)
    S.profile(True)
    S.run(tab, prof_steps)
    launches, kernel_ms = S.profile_stats()
    S.profile(False)
    avg_kernel_ms = kernel_ms / max(launches, 1)
    # eager launches without events, for comparison with the graph replay
    S.set_options(graph_steps=0)
    e0.record(stream)
    S.run(tab, prof_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms_step = e0.elapsed_time(e1) / prof_steps
    # the tiled step (values straight into LDS, 4 tiles per chunk) on the same
    # solver, for comparison
    _log("tiled step timing pass (%d steps)" % prof_steps)
    S.set_options(variant=drts.SPMV_LDS, tiles_per_chunk=4)
    S.profile(True)
    S.run(tab, prof_steps)
    t_launches, t_ms = S.profile_stats()
    S.profile(False)
    tiled_kernel_ms = t_ms / max(t_launches, 1)

    r = S.readout(0, total)
    assert (r["tot"][:, 0, 0] > 0).all()
    # windowed measurement (Eq. 27 over 101 steps) of the run's two detectors
    taps = np.exp(-0.5 * ((np.arange(101) - 50) / 12.0) ** 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.window(np.stack([taps, taps]), tap0=-50)
    t_win = time.perf_counter() - t0

    nbytes = spmv_bytes(A.nnz, A.n_rows, A.n_states)
    achieved = nbytes / (avg_kernel_ms * 1e-3) / 1e9
    fbytes = None if not groups or groups["n_groups"] == 0 else grouped_bytes(A.n_rows, A.n_states, groups)
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
        "config": {"workload": "C2: %d^3 voxels x 26 directions, 3 Fresnel layers, FP32 [A;L], "
                               "Gaussian 100 fs top-face source, 2 detectors" % args.n,
                   "n_states": A.n_states, "n_rows": A.n_rows, "nnz": A.nnz, "parallelism": "1 GPU",
                   "launch": "drts_run, hipGraph replay of %d steps; the default step (by row groups)" % GRAPH_STEPS},
        "eager_ms_per_step": round(eager_ms_step, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None if traffic is None else round(traffic / 1e9, 3),
                     "kernel": " + ".join(STEP_KERNELS), "kernel_ms": round(avg_kernel_ms, 4),
                     "kernel_timing": "HIP events around each of %d eager launches on the launch stream "
                                      "(the step's kernels, without the finalize)" % launches,
                     "algorithmic_bytes": nbytes,
                     "algorithmic_bytes_basis": "CSR [A;L]: 8 B per entry, row pointers, x and y once",
                     "format_bytes": fbytes,
                     "format_frac": None if fbytes is None else
                     round(fbytes / (avg_kernel_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "format_bytes_basis": "what the step by row groups must move: fast groups' values (one-byte "
                                           "dictionary indices and the row in a 32-byte slot per member when "
                                           "value-indexed, else FP32 in group order and the row), members' "
                                           "materials, descriptors; two-voxel rows' values and info; the listed "
                                           "rows' CSR entries; x and y once",
                     "note": "the step streams fewer bytes than the CSR count (no columns; value-indexed "
                             "entries), so frac can exceed 1; format_frac is the fraction of peak on the "
                             "bytes the step must move; instruction counters show the fast-group kernel "
                             "bound by VALU issue rather than by HBM (profiles/"
                             "step_spmv_grouped_c2_instructions.md)",
                     "traffic_unit": "GB per launch"},
        "row_groups": None if groups is None else dict(groups, device_bytes=group_bytes),
        "tiled_step": {"kernel": "step_spmv<float, int, 256, 2> (values straight into LDS, 4 tiles per chunk)",
                       "kernel_ms": round(tiled_kernel_ms, 4),
                       "frac": round(nbytes / (tiled_kernel_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "windowed_measurement": {"detectors": 2, "steps": total, "taps": 101,
                                 "call_ms": round(t_win * 1e3, 3)},
    }
    only = args.struct_only or args.spmm_only or args.batch_only or args.lebedev_only
    if not args.no_extras and args.n == 128 and (args.struct_only or not only):
        _log("structured step")
        line["structured"] = structured_step(torch, A, wl, tab)
    S.close()
    A.close()
    if not args.no_extras and (args.spmm_only or not only):
        _log("C3 SpMM")
        line["spmm"] = spmm_vs_plain(torch)
    if not args.no_extras and (args.batch_only or not only):
        _log("C4 batch")
        line["batch"] = batch_vs_sequential(torch)
    if not args.no_extras and not only:
        line["serving"] = serving_vs_fifo(torch)
    if not args.no_extras and (args.lebedev_only or not only):
        _log("Lebedev-86 step")
        line["lebedev86"] = lebedev_step(torch)
    if not args.no_extras and not only:
        _log("scatter order 4")
        line["higher_order"] = medium_variant_step(torch, "scatter order 4 (Eq. 4)",
                                                   lambda m: setattr(m, "scatter_order", 4))
        _log("interfaces crossed within the step")
        line["interface_substep"] = medium_variant_step(
            torch, "interfaces crossed within the step (path absorption, tangential landing; Sec. 4.2)",
            lambda m: setattr(m, "interface", "substep"))
    if not args.no_cpu:
        _log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
