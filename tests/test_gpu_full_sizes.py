"""Many right-hand sides and uneven batches at their full sizes, in the launch
configuration the benchmark times, checked through properties that hold at
any size (the single-rhs step they are compared with is itself held to the
FP64 oracle at full size by the 128^3 layered tests):
  - 96^3 slab, 64 right-hand sides: sampled SpMM columns equal the single-rhs
    runs of their own sources, bit for bit (state, exponents, series), and
    sampled matrix-free columns equal the single-rhs matrix-free runs;
  - 256 media of edges 16..64 in one batch: sampled members equal the same
    solver run alone, bit for bit;
  - a medium beyond 2^31 nonzeros (int64 row pointers): CSR steps equal the
    exact matrix-free steps bit for bit.
"""
import copy

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def test_c3_full_spmm_columns_equal_single_rhs_runs():
    steps = 12
    wl = W.c3(n_steps=steps)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    out = solve.run(wl, n_steps=steps, matrix=A)
    assert out["x"].shape == (A.n_rows, 64)
    for j in (0, 31, 63):
        w = copy.copy(wl)
        w.sources = [copy.copy(s) for s in wl.sources if s.rhs == j]
        for s in w.sources:
            s.rhs = 0
        w.n_rhs = 1
        one = solve.run(w, n_steps=steps, matrix=A)
        assert np.array_equal(out["x"][:, j], one["x"][:, 0]), j
        assert out["x_exp"][j] == one["x_exp"][0]
        assert np.array_equal(out["exp2"][:, j], one["exp2"][:, 0])
        assert np.allclose(out["tot"][:, :, j], one["tot"][:, :, 0], rtol=1e-13, atol=0)
        assert np.allclose(out["det"][:, :, j], one["det"][:, :, 0], rtol=1e-13, atol=0)
        one["solver"].close()
    out["solver"].close()
    A.close()


def test_c3_full_matrix_free_columns_equal_single_rhs_runs():
    """The matrix-free step for 64 right-hand sides (push and pull kernels,
    FP64 row sums) at full C3 size in the launch shape the benchmark times:
    sampled columns equal the single-rhs matrix-free runs of their own
    sources bit for bit (state, exponents), series to 1e-13."""
    import torch
    steps = 12
    wl = W.c3(n_steps=steps)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    opts = {"kernel": drts.KERNEL_STRUCTURED_F64SUM, "grid": 16 * cus}
    out = solve.run(wl, n_steps=steps, matrix=A, options=opts)
    for j in (0, 40, 63):
        w = copy.copy(wl)
        w.sources = [copy.copy(s) for s in wl.sources if s.rhs == j]
        for s in w.sources:
            s.rhs = 0
        w.n_rhs = 1
        one = solve.run(w, n_steps=steps, matrix=A, options={"kernel": drts.KERNEL_STRUCTURED_F64SUM})
        assert np.array_equal(out["x"][:, j], one["x"][:, 0]), j
        assert out["x_exp"][j] == one["x_exp"][0]
        assert np.array_equal(out["exp2"][:, j], one["exp2"][:, 0])
        assert np.allclose(out["tot"][:, :, j], one["tot"][:, :, 0], rtol=1e-13, atol=0)
        assert np.allclose(out["det"][:, :, j], one["det"][:, :, 0], rtol=1e-13, atol=0)
        one["solver"].close()
    out["solver"].close()
    A.close()


def test_int64_row_pointers_equal_matrix_free():
    """A 165^3 three-layer medium has more than 2^31 nonzeros, so its CSR
    takes int64 row pointers (assembly and step kernels of that width): its
    steps in the launch shape of the benchmark equal the exact matrix-free
    steps (nearest-rounded values), which never read the CSR, bit for bit."""
    steps = 6
    wl = W.c2(n=165, n_steps=steps, rounding="nearest")
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    assert A.nnz > 2 ** 31 - 1, A.nnz
    csr = solve.run(wl, n_steps=steps, matrix=A)
    mf = solve.run(wl, n_steps=steps, matrix=A, options={"kernel": drts.KERNEL_STRUCTURED})
    assert np.array_equal(csr["x"], mf["x"]) and np.array_equal(csr["x_exp"], mf["x_exp"])
    assert np.array_equal(csr["exp2"], mf["exp2"])
    assert np.allclose(csr["tot"], mf["tot"], rtol=1e-13, atol=0)
    assert np.allclose(csr["det"], mf["det"], rtol=1e-13, atol=0)
    assert (csr["tot"][:, 0, 0] > 0).all()
    csr["solver"].close()
    mf["solver"].close()
    A.close()


def test_c4_full_batch_members_equal_solo_runs():
    steps = 20
    wls = W.c4(n_steps=steps)
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, [], max_steps=steps) for m in mats]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    B.run(tabs, [steps] * len(solvers))
    B.close()
    for i in (0, 77, 150, 255):
        # the same step as in the batch: its own grouped step for a large
        # member, the tiled step for one of the shared launch
        opts = None if mats[i].n_rows >= drts.BATCH_OWN_ROWS else {"variant": drts.SPMV_LDS}
        solo = solve.run(wls[i], n_steps=steps, matrix=mats[i], options=opts)
        x, e, t = solvers[i].state()
        assert t == steps
        assert np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"]), i
        r = solvers[i].readout(0, steps)
        assert np.array_equal(r["tot"], solo["tot"]) and np.array_equal(r["exp2"], solo["exp2"]), i
        solo["solver"].close()
    for S in solvers:
        S.close()
    for m in mats:
        m.close()
