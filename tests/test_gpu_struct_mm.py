"""The matrix-free step for many right-hand sides (push and pull kernels),
through the C ABI.

Bars:
  - exact mode (nearest-rounded values) against the CSR SpMM: states bit for
    bit (both add the same FP32 products per row in column order), FP64
    series to 1e-13 (their chunk partials differ);
  - FP64-sum mode: every column equals the single-rhs FP64-sum run of its own
    sources, state bit for bit, on a layered medium with Fresnel interfaces,
    face detectors and sources in several columns; and against the FP64
    oracle within 1e-5 on the many-source slab.
"""
import copy

import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _single(wl, j):
    w = copy.copy(wl)
    w.sources = [copy.copy(s) for s in wl.sources if s.rhs == j]
    for s in w.sources:
        s.rhs = 0
    w.n_rhs = 1
    return w


def _layered_many(n=16, k=4, n_steps=60):
    """The layered medium with k top-face Gaussian sources of different widths."""
    wl = copy.copy(W.c2(n=n, n_steps=n_steps))
    base = wl.sources[0]
    wl.sources = []
    for j in range(k):
        s = copy.copy(base)
        s.fwhm_fs = 80.0 + 60.0 * j
        s.w = np.asarray(base.w) * (1.0 + 0.25 * j)
        s.rhs = j
        wl.sources.append(s)
    wl.n_rhs = k
    return wl


def test_exact_mode_equals_csr_spmm():
    wl = W.c3(n=20, k=8, n_steps=40, rounding="nearest")
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    a = solve.run(wl, matrix=A)
    b = solve.run(wl, matrix=A, options={"kernel": drts.KERNEL_STRUCTURED})
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["x_exp"], b["x_exp"])
    assert np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["tot"], b["tot"], rtol=1e-13, atol=0)
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)


def _reflecting_many(n=10, k=3, n_steps=30):
    """A closed box (reflecting walls: no escape rows) with k sources."""
    wl = copy.copy(W.c3(n=n, k=k, n_steps=n_steps))
    wl.medium = copy.copy(wl.medium)
    wl.medium.bc = "reflect"
    wl.detectors = []
    return wl


def _ten_layers_many(n=20, k=3, n_steps=30):
    """Ten layers, ten materials (more than the single-rhs direction-major
    kernel takes, so the single-rhs runs take the gather kernel) and k
    top-face sources."""
    mats = [W.Material(4.0 + j, 0.01 * (j + 1), 0.7 + 0.02 * j, 1.33 + 0.01 * (j % 3)) for j in range(10)]
    med = W.layered(n, mats)
    srcs = [W.point_source(3 + 5 * j, 4 + 3 * j, 0, kind="gaussian", fwhm_fs=100.0 + 50.0 * j, rhs=j)
            for j in range(k)]
    return W.Workload("ten_layers", med, srcs, [W.face_escape_detector(med, "top")], n_steps, k, "f32",
                      "dither", 1.33)


@pytest.mark.parametrize("make", [lambda: _layered_many(), lambda: W.c3(n=18, k=6, n_steps=40),
                                  lambda: _reflecting_many(), lambda: _ten_layers_many()],
                         ids=["layered_4rhs", "slab_6rhs", "reflecting_3rhs", "ten_materials_3rhs"])
def test_f64sum_columns_equal_single_rhs_runs(make):
    wl = make()
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    out = solve.run(wl, matrix=A, options={"kernel": drts.KERNEL_STRUCTURED_F64SUM})
    for j in range(wl.n_rhs):
        one = solve.run(_single(wl, j), matrix=A, options={"kernel": drts.KERNEL_STRUCTURED_F64SUM})
        assert np.array_equal(out["x"][:, j], one["x"][:, 0]), j
        assert out["x_exp"][j] == one["x_exp"][0]
        assert np.array_equal(out["exp2"][:, j], one["exp2"][:, 0])
        assert np.allclose(out["tot"][:, :, j], one["tot"][:, :, 0], rtol=1e-13, atol=0)
        assert np.allclose(out["det"][:, :, j], one["det"][:, :, 0], rtol=1e-13, atol=0)


def test_f64sum_against_oracle():
    wl = W.c3(n=22, k=64, n_steps=50)
    out = solve.run(wl, options={"kernel": drts.KERNEL_STRUCTURED_F64SUM})
    A = oracle.Matrix(wl.medium)
    for j in (0, 21, 63):
        ref = oracle.run_workload(A, wl, rhs=j)
        e = out["exp2"][:, j]
        for d in range(16):
            err = parity.rel_err_series(out["det"][:, d, j], e, ref["det"][:, d], ref["det_exp"][:, d])
            assert err <= 1e-5, (j, d, err)
        for c in range(3):
            err = parity.rel_err_series(out["tot"][:, c, j], e, ref["tot"][:, c], ref["tot_exp"][:, c])
            assert err <= 1e-5, (j, c, err)
        assert parity.rel_l1(out["x"][:A.n_states, j], out["x_exp"][j], ref["x"], ref["x_exp"]) <= 1e-5


def test_exact_mode_rejects_dithered_values():
    wl = W.c3(n=12, k=4, n_steps=5, rounding="dither")
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(A, 4, wl.detectors, max_steps=5)
    with pytest.raises(drts.DrtsError):
        S.set_options(kernel=drts.KERNEL_STRUCTURED)
