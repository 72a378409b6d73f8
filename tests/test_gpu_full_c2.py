"""The full-size layered workload (128^3 voxels x 26 directions, three Fresnel
layers, FP32 values under dithered rounding) against stored oracle values.

The expected values in tests/golden/ are written by tests/golden/make_golden.py,
which calls only the oracle.  The library runs in the launch configuration the
benchmark times (default options).  Bars:
  - assembly: sha256 of every one of 64 row chunks (int64 row pointers, int32
    columns, FP32 values) equal to the oracle's: bit-exact;
  - one product y = [A; L] x of a seeded FP32 x at 7200 sampled rows (random,
    escape, interface and short rows): within the FP32 summation bound,
    |y - y_ref| <= 64 u sum |a x| with u = 2^-24 (all terms are nonnegative);
  - the 2000-step series (photon count, escaped, absorbed, two detectors):
    relative error <= 1e-5 against the FP64 oracle, for the CSR step and for
    the matrix-free step with FP64 row sums;
  - the final state: relative L1 error <= 1e-5 over sampled entries and of
    the whole state's L1 norm.
The error against the same-matrix oracle (FP64 arithmetic on the FP32-rounded
values, tests/golden/c2_same.npz: the kernels' own arithmetic error) and the
elementwise maximum relative error of the sampled state (entries above
1e-30 x the largest) are printed beside each bar; the same-matrix series and
sampled state are held to 1e-5 as well.
"""
import hashlib
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def c2():
    wl = W.c2()
    M = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    yield wl, M
    M.close()


def test_c2_assembly_chunk_hashes(c2):
    wl, M = c2
    meta = json.load(open(os.path.join(GOLDEN, "c2_csr.json")))
    assert (M.n_states, M.n_escape, M.nnz) == (meta["n_states"], meta["n_escape"], meta["nnz"])
    assert meta["value_type"] == wl.value_type and meta["rounding"] == wl.rounding
    n_rows, nch = M.n_rows, meta["chunks"]

    def one(k):
        r0, r1 = (k * n_rows) // nch, ((k + 1) * n_rows) // nch
        rp, col, val = M.export_rows(r0, r1 - r0)
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(rp, dtype="<i8").tobytes())
        h.update(np.ascontiguousarray(col, dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(val).tobytes())
        return h.hexdigest()

    with ThreadPoolExecutor(8) as ex:
        got = list(ex.map(one, range(nch)))
    bad = [k for k in range(nch) if got[k] != meta["sha256"][k]]
    assert not bad, "row chunks differing from the oracle: %s" % bad


def test_c2_one_product_sampled_rows(c2):
    wl, M = c2
    g = np.load(os.path.join(GOLDEN, "c2_spmv.npz"))
    rows, y_ref = g["rows"], g["y"]
    x = np.zeros(M.n_rows, dtype=np.float32)
    x[:M.n_states] = W.seeded_state(M.n_states, 2).astype(np.float32)
    S = drts.Solver(M, 1, [], max_steps=1)
    S.set_state(x, [0], 0)
    S.step(None)
    y, e, t = S.state()
    assert t == 1
    y_gpu = np.ldexp(y[rows, 0].astype(np.float64), int(e[0]))
    # sum |a x| of each sampled row, from the exported rows of the device matrix
    bound = np.empty(rows.size)
    for i, r in enumerate(rows):
        rp, col, val = M.export_rows(int(r), 1)
        bound[i] = np.abs(val.astype(np.float64) * x[col].astype(np.float64)).sum()
    err = np.abs(y_gpu - y_ref)
    assert np.all(err <= 64 * 2.0 ** -24 * bound + 1e-300), float((err / np.maximum(bound, 1e-300)).max())
    assert np.array_equal(y_gpu == 0, y_ref == 0)
    S.close()


@pytest.mark.parametrize("kernel", [drts.KERNEL_CSR, drts.KERNEL_STRUCTURED_F64SUM], ids=["csr", "struct_f64sum"])
def test_c2_2000_steps_against_oracle(c2, kernel):
    wl, M = c2
    g = np.load(os.path.join(GOLDEN, "c2_run.npz"))
    steps = int(g["steps"])
    S = drts.Solver(M, 1, wl.detectors, max_steps=steps)
    if kernel != drts.KERNEL_CSR:
        S.set_options(kernel=kernel)
    S.run(solve.source_table(M, wl), steps)
    r = S.readout(0, steps)
    e = r["exp2"][:, 0]
    same_path = os.path.join(GOLDEN, "c2_same.npz")
    if not os.path.exists(same_path):
        pytest.fail("missing stored oracle values c2_same.npz (tests/golden/make_golden.py c2same)")
    gs = np.load(same_path)
    assert int(gs["steps"]) == steps and np.array_equal(gs["x_idx"], g["x_idx"])
    worst = {}
    for ref, key in ((g, "fp64"), (gs, "same")):
        err = 0.0
        for c in range(3):
            err = max(err, parity.rel_err_series(r["tot"][:, c, 0], e, ref["tot"][:, c], ref["tot_exp"][:, c]))
        for d in range(2):
            err = max(err, parity.rel_err_series(r["det"][:, d, 0], e, ref["det"][:, d], ref["det_exp"][:, d]))
        worst[key] = err
    x, xe, t = S.state()
    assert t == steps
    idx = g["x_idx"]
    l1s, emaxs = {}, {}
    for ref, key in ((g, "fp64"), (gs, "same")):
        l1s[key] = parity.rel_l1(x[idx, 0], xe[0], ref["x_val"], int(ref["x_exp"]))
        xs = np.ldexp(x[idx, 0].astype(np.float64), int(xe[0]) - int(ref["x_exp"]))
        rv = ref["x_val"]
        keep = rv > 1e-30 * rv.max()
        emaxs[key] = float(np.max(np.abs(xs[keep] - rv[keep]) / rv[keep]))
    l1 = np.ldexp(np.abs(x[:M.n_states, 0].astype(np.float64)).sum(), int(xe[0]) - int(g["x_exp"]))
    enorm = abs(l1 - float(g["x_l1"])) / float(g["x_l1"])
    print("C2 %d steps, kernel %d: series %.3g (same-matrix %.3g), state L1 %.3g (same-matrix %.3g), "
          "elementwise max %.3g (same-matrix %.3g), L1 norm %.3g"
          % (steps, kernel, worst["fp64"], worst["same"], l1s["fp64"], l1s["same"], emaxs["fp64"], emaxs["same"],
             enorm), flush=True)
    assert worst["fp64"] <= 1e-5 and worst["same"] <= 1e-5, worst
    assert l1s["fp64"] <= 1e-5 and l1s["same"] <= 1e-5, l1s
    assert enorm <= 1e-5
    S.close()
