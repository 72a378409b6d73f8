#!/usr/bin/env python3
"""Writes the stored expected values of the full-size workloads.

Calls only the oracle (``oracle/``) and the seeded inputs (``workloads``).
Outputs, per workload, under tests/golden/:
  <name>_csr.json   sha256 of the oracle's CSR in 64 row chunks (int64 row
                    pointers, int32 columns, values as stored by the library:
                    FP32 under the workload's rounding, or FP64), plus sizes;
  <name>_spmv.npz   one product y = [A; L] x for a seeded FP32-valued x at
                    sampled rows (FP64 arithmetic on the stored values);
  <name>_run.npz    the FP64 series of the full run (totals, detectors, with
                    exponents) and sampled entries of the final state.

  c2_same.npz       the 2000-step C2 run under FP64 arithmetic on the
                    FP32-rounded matrix (the same-matrix oracle): series and
                    the final state at the entries c2_run.npz samples;
  c3_run.npz        the 96^3 slab with 64 right-hand sides: right-hand
                    sides 0, 31 and 63 over all 1000 steps (series, sampled
                    final state, its L1 norm), each also under FP64
                    arithmetic on the FP32-rounded matrix (the same-matrix
                    oracle, which isolates the kernels' arithmetic);
  c4_run.npz        the first 16 of the 256 uneven-batch media over all 500
                    steps (series), also on the same-matrix oracle;
  c5_run.npz        the 8 smallest requests of the serving stream (sphere
                    inclusions with Fresnel interfaces and total internal
                    reflection) over their full step counts (series), also on
                    the same-matrix oracle.

Usage: python tests/golden/make_golden.py c2|c1|c2same|c3|c4|c5 [--steps N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_CHUNKS = 64


def chunk_bounds(n_rows, k):
    return (k * n_rows) // N_CHUNKS, ((k + 1) * n_rows) // N_CHUNKS


def csr_hashes(row_ptr, col, val):
    n_rows = row_ptr.size - 1
    out = []
    for k in range(N_CHUNKS):
        r0, r1 = chunk_bounds(n_rows, k)
        b, e = int(row_ptr[r0]), int(row_ptr[r1])
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(row_ptr[r0:r1 + 1], dtype="<i8").tobytes())
        h.update(np.ascontiguousarray(col[b:e], dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(val[b:e]).tobytes())
        out.append(h.hexdigest())
    return out


def sample_rows(A, rng, n=6000):
    """Random rows plus every kind of special row: escape rows, interface rows."""
    rows = set(rng.integers(0, A.n_rows, size=n).tolist())
    rows |= set(rng.integers(A.n_states, A.n_rows, size=500).tolist())
    lens = np.diff(A.row_ptr)
    long_rows = np.flatnonzero(lens > 26)
    if long_rows.size:
        rows |= set(rng.choice(long_rows, size=min(500, long_rows.size), replace=False).tolist())
    short_rows = np.flatnonzero(lens < 26)
    if short_rows.size:
        rows |= set(rng.choice(short_rows, size=min(200, short_rows.size), replace=False).tolist())
    return np.array(sorted(rows), dtype=np.int64)


def make(name, wl, steps, out_dir):
    t0 = time.time()
    A = oracle.Matrix(wl.medium)
    print("%s: assembled %d rows, %d nnz in %.1f s" % (name, A.n_rows, A.nnz, time.time() - t0), flush=True)
    vals = A.val if wl.value_type == "f64" else A.round_f32(wl.rounding)
    meta = {"workload": name, "n_states": int(A.n_states), "n_escape": int(A.n_escape), "nnz": int(A.nnz),
            "value_type": wl.value_type, "rounding": wl.rounding, "chunks": N_CHUNKS,
            "sha256": csr_hashes(A.row_ptr, A.col, vals)}
    json.dump(meta, open(os.path.join(out_dir, name + "_csr.json"), "w"), indent=1)
    print("%s: hashes done %.1f s" % (name, time.time() - t0), flush=True)

    rng = np.random.default_rng([W.SEED, 77])
    x = W.seeded_state(A.n_states, 2).astype(np.float32).astype(np.float64)
    y = A.spmv(x, vals32=None if wl.value_type == "f64" else vals)
    rows = sample_rows(A, rng)
    np.savez_compressed(os.path.join(out_dir, name + "_spmv.npz"), rows=rows, y=y[rows])
    del y
    print("%s: one-step sample done %.1f s" % (name, time.time() - t0), flush=True)

    r = oracle.run_workload(A, wl, n_steps=steps)
    st = rng.integers(0, A.n_states, size=4000)
    top = np.argsort(r["x"])[-200:]
    idx = np.unique(np.concatenate([st, top]))
    np.savez_compressed(os.path.join(out_dir, name + "_run.npz"), steps=steps, tot=r["tot"], tot_exp=r["tot_exp"],
                        det=r["det"], det_exp=r["det_exp"], x_idx=idx, x_val=r["x"][idx], x_exp=r["x_exp"],
                        x_l1=np.abs(r["x"]).sum())
    print("%s: run of %d steps done %.1f s" % (name, steps, time.time() - t0), flush=True)


def make_c2_same(out_dir):
    """The same-matrix oracle of the C2 run: the FP32-rounded values under
    FP64 arithmetic, sampled at the entries c2_run.npz holds (both files
    come from the oracle alone)."""
    t0 = time.time()
    wl = W.c2()
    g = np.load(os.path.join(out_dir, "c2_run.npz"))
    steps = int(g["steps"])
    A = oracle.Matrix(wl.medium)
    vals = A.round_f32(wl.rounding)
    print("c2same: assembled %d rows, %d nnz in %.1f s" % (A.n_rows, A.nnz, time.time() - t0), flush=True)
    r = oracle.run_workload(A, wl, n_steps=steps, vals32=vals)
    idx = g["x_idx"]
    out = {"steps": steps, "x_idx": idx, "x_val": r["x"][idx], "x_exp": r["x_exp"], "x_l1": np.abs(r["x"]).sum()}
    _series(r, "", out)
    np.savez_compressed(os.path.join(out_dir, "c2_same.npz"), **out)
    print("c2same: run of %d steps done %.1f s" % (steps, time.time() - t0), flush=True)


def _series(r, prefix, out):
    for k in ("tot", "tot_exp", "det", "det_exp"):
        out[prefix + k] = r[k]


C3_RHS = (0, 31, 63)
C3_STATE_SAMPLES = 4000


def make_c3(out_dir, steps=None):
    t0 = time.time()
    wl = W.c3()
    steps = steps or wl.n_steps
    A = oracle.Matrix(wl.medium)
    vals = A.round_f32(wl.rounding)
    print("c3: assembled %d rows, %d nnz in %.1f s" % (A.n_rows, A.nnz, time.time() - t0), flush=True)
    out = {"steps": steps, "rhs": np.array(C3_RHS)}
    rng = np.random.default_rng([W.SEED, 33])
    for k in C3_RHS:
        r = oracle.run_workload(A, wl, rhs=k, n_steps=steps)
        _series(r, "r%d_" % k, out)
        st = rng.integers(0, A.n_states, size=C3_STATE_SAMPLES)
        top = np.argsort(r["x"])[-200:]
        idx = np.unique(np.concatenate([st, top]))
        out["r%d_x_idx" % k] = idx
        out["r%d_x_val" % k] = r["x"][idx]
        out["r%d_x_exp" % k] = r["x_exp"]
        out["r%d_x_l1" % k] = np.abs(r["x"]).sum()
        s = oracle.run_workload(A, wl, rhs=k, n_steps=steps, vals32=vals)
        _series(s, "r%d_same_" % k, out)
        out["r%d_same_x_val" % k] = s["x"][idx]
        out["r%d_same_x_exp" % k] = s["x_exp"]
        print("c3: rhs %d done %.1f s" % (k, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(out_dir, "c3_run.npz"), **out)


C4_MEMBERS = 16


def make_c4(out_dir, steps=None):
    t0 = time.time()
    wls = W.c4()[:C4_MEMBERS]
    steps = steps or wls[0].n_steps
    out = {"steps": steps, "members": np.arange(C4_MEMBERS)}
    for i, wl in enumerate(wls):
        A = oracle.Matrix(wl.medium)
        vals = A.round_f32(wl.rounding)
        _series(oracle.run_workload(A, wl, n_steps=steps), "m%d_" % i, out)
        _series(oracle.run_workload(A, wl, n_steps=steps, vals32=vals), "m%d_same_" % i, out)
        A.close()
        print("c4: member %d (edge %d) done %.1f s" % (i, wl.medium.nx, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(out_dir, "c4_run.npz"), **out)


C5_REQUESTS = 8


def c5_smallest(reqs):
    """Indices of the C5_REQUESTS smallest requests (grid edge, then arrival)."""
    order = sorted(range(len(reqs)), key=lambda i: (reqs[i].workload.medium.nx, i))
    return order[:C5_REQUESTS]


def make_c5(out_dir):
    t0 = time.time()
    reqs = W.c5()
    pick = c5_smallest(reqs)
    out = {"requests": np.array(pick)}
    for i in pick:
        wl = reqs[i].workload
        A = oracle.Matrix(wl.medium)
        vals = A.round_f32(wl.rounding)
        _series(oracle.run_workload(A, wl), "q%d_" % i, out)
        _series(oracle.run_workload(A, wl, vals32=vals), "q%d_same_" % i, out)
        out["q%d_steps" % i] = wl.n_steps
        A.close()
        print("c5: request %d (edge %d, %d steps) done %.1f s" % (i, wl.medium.nx, wl.n_steps, time.time() - t0),
              flush=True)
    np.savez_compressed(os.path.join(out_dir, "c5_run.npz"), **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c1", "c2same", "c3", "c4", "c5"])
    ap.add_argument("--steps", type=int, default=None)
    a = ap.parse_args()
    if a.which == "c2same":
        make_c2_same(HERE)
    elif a.which == "c3":
        make_c3(HERE, a.steps)
    elif a.which == "c4":
        make_c4(HERE, a.steps)
    elif a.which == "c5":
        make_c5(HERE)
    else:
        wl = W.c2() if a.which == "c2" else W.c1()
        make(a.which, wl, a.steps or wl.n_steps, HERE)


if __name__ == "__main__":
    main()
