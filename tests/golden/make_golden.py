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

Usage: python tests/golden/make_golden.py c2 [--steps N]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c1"])
    ap.add_argument("--steps", type=int, default=None)
    a = ap.parse_args()
    wl = W.c2() if a.which == "c2" else W.c1()
    make(a.which, wl, a.steps or wl.n_steps, HERE)


if __name__ == "__main__":
    main()
