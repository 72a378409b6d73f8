"""Several scatterings within one step (Eq. (4)-(5)) on the GPU.

A medium's scatter order K changes only its direction blocks (Poisson-weighted
powers of the scattering kernel); the assembly and every step kernel are the
ones of the single-scatter path.  Bars: assembly bit-exact against the
oracle (FP64 and FP32 values); FP64 runs within 1e-12 and FP32 runs within
1e-5 of the FP64 oracle, for the CSR step and the matrix-free step."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _with_order(wl, K):
    wl.medium.scatter_order = K
    return wl


@pytest.mark.parametrize("K", [2, 4])
def test_assembly_bitexact_higher_order(K):
    for med in (W.c2(n=14).medium, W.c5(n_req=1, edge=(16, 16))[0].workload.medium):
        med.scatter_order = K
        A = oracle.Matrix(med)
        for vt, rnd in (("f64", "nearest"), ("f32", "dither")):
            M = drts.Matrix(med, vt, rnd, 1.4)
            rp, col, val = M.export_rows()
            assert np.array_equal(rp, A.row_ptr) and np.array_equal(col, A.col)
            want = A.val if vt == "f64" else A.round_f32(rnd)
            assert np.array_equal(val.view(np.uint8), want.view(np.uint8)), (K, vt)
            M.close()


def test_c1_order4_fp64_parity():
    """16^3, mu_s c dt = 1 (where several scatterings per step matter), FP64."""
    wl = _with_order(W.c1(), 4)
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl)
    single = oracle.run_workload(oracle.Matrix(W.c1().medium), W.c1())
    out = solve.run(wl)
    tot, e = out["tot"][:, :, 0], out["exp2"][:, 0]
    for j in range(3):
        assert parity.rel_err_series(tot[:, j], e, ref["tot"][:, j], ref["tot_exp"][:, j]) <= 1e-12
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-12
    # and the order changes the result (the escaped series differs from order 1)
    assert parity.rel_err_series(tot[:, 1], e, single["tot"][:, 1], single["tot_exp"][:, 1]) > 1e-3


@pytest.mark.parametrize("kernel", [drts.KERNEL_CSR, drts.KERNEL_STRUCTURED_F64SUM], ids=["csr", "mf_f64sum"])
def test_layers_order3_fp32_parity(kernel):
    wl = _with_order(W.c2(n=20, n_steps=200), 3)
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl, options=None if kernel == drts.KERNEL_CSR else {"kernel": kernel})
    e = out["exp2"][:, 0]
    for j in range(3):
        err = parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j])
        assert err <= 1e-5, (j, err)
    for d in range(2):
        err = parity.rel_err_series(out["det"][:, d, 0], e, ref["det"][:, d], ref["det_exp"][:, d])
        assert err <= 1e-5, (d, err)
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-5
