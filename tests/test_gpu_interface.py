"""Crossing an interface within the step (Sec. 4.2, DRTS_INTERFACE_SUBSTEP) on
the GPU: path-proportional absorption of the transmitted part, the reflected
part landing one voxel over along a planar interface.

Bars: assembly bit-exact against the oracle (FP64 and FP32 values) on layered
and sphere media; FP32 runs within 1e-5 of the FP64 oracle with the CSR step,
the matrix-free step with FP64 row sums and the exact matrix-free step; the
128^3 three-layer medium (the benchmark's workload with this model) bit-exact
on sampled rows of every kind and within 1e-5 of the oracle over 50 steps.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _substep(med):
    med.interface = "substep"
    return med


def _absorbing_layers():
    return [W.Material(5.0, 0.05, 0.8, 1.33), W.Material(15.0, 0.5, 0.9, 1.45), W.Material(10.0, 0.2, 0.85, 1.40)]


def _media():
    return [("layers10", _substep(W.layered(10, _absorbing_layers()))),
            ("sphere12", _substep(W.sphere_inclusion(12, W.Material(10.0, 0.01, 0.9, 1.33),
                                                     W.Material(10.0, 0.08, 0.9, 1.45), (5.3, 6.1, 5.7), 3.4)))]


MEDIA = _media()


@pytest.mark.parametrize("name,med", MEDIA, ids=[m[0] for m in MEDIA])
@pytest.mark.parametrize("vt,rnd", [("f64", "nearest"), ("f32", "dither")])
def test_substep_assembly_bitexact(name, med, vt, rnd):
    A = oracle.Matrix(med)
    M = drts.Matrix(med, vt, rnd, 1.4)
    rp, col, val = M.export_rows()
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(col, A.col)
    want = A.val if vt == "f64" else A.round_f32(rnd)
    assert np.array_equal(val.view(np.uint8), want.view(np.uint8))
    M.close()


@pytest.mark.parametrize("kernel,rounding", [(0, "dither"), (2, "dither"), (1, "nearest")],
                         ids=["csr", "mf_f64sum", "mf_exact"])
def test_substep_layers_fp32_parity(kernel, rounding):
    base = W.c2(n=24, n_steps=300, rounding=rounding)
    med = _substep(W.layered(24, _absorbing_layers()))
    wl = W.Workload("substep", med, base.sources, [W.face_escape_detector(med, "top"),
                                                   W.face_escape_detector(med, "bottom")], 300, 1, "f32", rounding,
                    1.33)
    A = oracle.Matrix(med)
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl, options=None if kernel == 0 else {"kernel": kernel})
    e = out["exp2"][:, 0]
    for j in range(3):
        err = parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j])
        assert err <= 1e-5, (j, err)
    for d in range(2):
        err = parity.rel_err_series(out["det"][:, d, 0], e, ref["det"][:, d], ref["det_exp"][:, d])
        assert err <= 1e-5, (d, err)
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-5
    out["solver"].close()


def test_substep_sphere_fp32_parity():
    wl = W.c5(n_req=1, edge=(20, 20))[0].workload
    _substep(wl.medium)
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl, n_steps=250)
    out = solve.run(wl, n_steps=250)
    e = out["exp2"][:, 0]
    for j in range(3):
        assert parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j]) <= 1e-5
    assert parity.rel_err_series(out["det"][:, 0, 0], e, ref["det"][:, 0], ref["det_exp"][:, 0]) <= 1e-5
    out["solver"].close()


def test_substep_128_three_layers_sampled_rows_and_steps():
    steps = 50
    wl = W.c2(n_steps=steps)
    _substep(wl.medium)
    print("substep 128^3: oracle assembly", flush=True)
    A = oracle.Matrix(wl.medium)
    vals = A.round_f32(wl.rounding)
    M = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    assert (M.n_states, M.n_escape, M.nnz) == (A.n_states, A.n_escape, A.nnz)
    rng = np.random.default_rng([161108536, 42])
    lens = np.diff(A.row_ptr)
    rows = np.unique(np.concatenate([rng.integers(0, A.n_rows, 3000), rng.integers(A.n_states, A.n_rows, 300),
                                     rng.choice(np.flatnonzero(lens > 26), 1000),
                                     rng.choice(np.flatnonzero(lens < 26), 300)]))
    rp = A.row_ptr
    for r in rows:
        _, col, val = M.export_rows(int(r), 1)
        assert np.array_equal(col, A.col[rp[r]:rp[r + 1]]), r
        assert np.array_equal(val, vals[rp[r]:rp[r + 1]]), r
    print("substep 128^3: %d sampled rows equal; oracle run of %d steps" % (rows.size, steps), flush=True)
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl, matrix=M)
    e = out["exp2"][:, 0]
    for j in range(3):
        assert parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j]) <= 1e-5
    for d in range(2):
        assert parity.rel_err_series(out["det"][:, d, 0], e, ref["det"][:, d], ref["det_exp"][:, d]) <= 1e-5
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-5
    out["solver"].close()
    M.close()
