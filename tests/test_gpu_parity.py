"""HIP path against the FP64 oracle, element by element, on seeded inputs.

Every test calls the library through its C ABI (the ctypes binding).  Bars:
  - assembly (row pointers, columns, FP64 values, FP32 values under both
    rounding modes): bit-exact;
  - FP64 runs: relative error <= 1e-12 (sum orders differ);
  - FP32 runs: <= 1e-5 against the FP64 oracle (the stated tolerance);
  - the same kernel under different launch shapes, eager / graph / step-by-
    step, resume, and the rescale: bit-exact where the arithmetic is the same.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity
from tests.test_oracle_pins import TINY

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _oracle_csr(med, value_type, rounding):
    A = oracle.Matrix(med)
    rp, col = A.row_ptr.copy(), A.col.copy()
    val = A.val.copy() if value_type == "f64" else A.round_f32(rounding)
    return A, rp, col, val


def _assert_same_csr(med, value_type, rounding, n_ref=1.4):
    A_o, rp, col, val = _oracle_csr(med, value_type, rounding)
    M = drts.Matrix(med, value_type, rounding, n_ref)
    assert (M.n_states, M.n_escape, M.nnz) == (A_o.n_states, A_o.n_escape, A_o.nnz)
    grp, gcol, gval = M.export_rows()
    assert np.array_equal(grp, rp)
    assert np.array_equal(gcol, col)
    assert gval.dtype == val.dtype
    assert np.array_equal(gval.view(np.uint8), val.view(np.uint8))
    return M, A_o


# ---- assembly -----------------------------------------------------------------

@pytest.mark.parametrize("name,med", TINY, ids=[t[0] for t in TINY])
@pytest.mark.parametrize("vt,rnd", [("f64", "nearest"), ("f32", "nearest"), ("f32", "dither")])
def test_assembly_bitexact_tiny(name, med, vt, rnd):
    _assert_same_csr(med, vt, rnd)


@pytest.mark.parametrize("vt,rnd", [("f64", "nearest"), ("f32", "dither")])
def test_assembly_bitexact_layers_and_sphere(vt, rnd):
    _assert_same_csr(W.c2(n=24).medium, vt, rnd)
    req = W.c5(n_req=3, edge=(20, 26))
    for q in req:
        _assert_same_csr(q.workload.medium, vt, rnd)


def test_assembly_bitexact_tied_interface_directions():
    """A sphere centred on the middle column of an odd grid: many crossings
    snap to tied lattice directions, whose parts are split evenly."""
    bg, inc = W.Material(10.0, 0.05, 0.8, 1.0), W.Material(6.0, 0.2, 0.5, 1.6)
    med = W.sphere_inclusion(9, bg, inc, (4.5, 4.5, 4.0), 2.6)
    for vt, rnd in (("f64", "nearest"), ("f32", "dither")):
        _assert_same_csr(med, vt, rnd)


def test_assembly_from_geometry_equals_map():
    """mat_of_voxel = NULL: the library derives the same map from the geometry."""
    for med in (W.c2(n=20).medium, W.c5(n_req=1, edge=(18, 18))[0].workload.medium):
        a = drts.Matrix(med, "f32", "dither", use_map=True)
        b = drts.Matrix(med, "f32", "dither", use_map=False)
        for x, y in zip(a.export_rows(), b.export_rows()):
            assert np.array_equal(x, y)


def test_assembly_c1_full():
    _assert_same_csr(W.c1().medium, "f64", "nearest")


# ---- FP64 parity ---------------------------------------------------------------

def test_c1_fp64_parity():
    """C1: 16^3, mu_s 10, FP64, 200 steps, impulse at the centre in +z."""
    wl = W.c1()
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl)
    tot, e = out["tot"][:, :, 0], out["exp2"][:, 0]
    for j in range(3):
        err = parity.rel_err_series(tot[:, j], e, ref["tot"][:, j], ref["tot_exp"][:, j])
        assert err <= 1e-12, (j, err)
    D = A.n_states
    assert parity.rel_l1(out["x"][:D, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-12
    # the totals underflow FP32 by the end: the exponent carries them
    assert (e[-1] + np.log2(tot[-1, 0])) < -120


# ---- FP32 parity ---------------------------------------------------------------

def _fp32_parity(wl, n_steps, tol=1e-5):
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl, n_steps=n_steps)
    out = solve.run(wl, n_steps=n_steps)
    tot, e = out["tot"][:, :, 0], out["exp2"][:, 0]
    errs = {}
    for j, name in enumerate(("N", "escaped", "absorbed")):
        errs[name] = parity.rel_err_series(tot[:, j], e, ref["tot"][:, j], ref["tot_exp"][:, j])
    for d in range(len(wl.detectors)):
        errs["det%d" % d] = parity.rel_err_series(out["det"][:, d, 0], e, ref["det"][:, d], ref["det_exp"][:, d])
    D = A.n_states
    errs["state_l1"] = parity.rel_l1(out["x"][:D, 0], out["x_exp"][0], ref["x"], ref["x_exp"])
    # same-matrix oracle: FP64 arithmetic on the library's FP32 values
    same = oracle.run_workload(A, wl, n_steps=n_steps, vals32=A.round_f32(wl.rounding))
    errs["state_l1_same_matrix"] = parity.rel_l1(out["x"][:D, 0], out["x_exp"][0], same["x"], same["x_exp"])
    print(wl.name, n_steps, errs)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    return errs


def test_c2_layers_fp32_parity():
    """Three Fresnel layers, Gaussian 100 fs top-face source, two face detectors."""
    _fp32_parity(W.c2(n=24), 300)


def test_c5_sphere_fp32_parity():
    """Spherical inclusion with index mismatch (reflection, refraction, TIR)."""
    wl = W.c5(n_req=1, edge=(22, 22))[0].workload
    _fp32_parity(wl, 250)


def test_fp32_nearest_rounding_parity():
    _fp32_parity(W.c2(n=18, rounding="nearest"), 200)


# ---- same kernel, different schedules --------------------------------------------

def _state_and_series(wl, n, **kw):
    out = solve.run(wl, n_steps=n, **kw)
    return out["x"], out["x_exp"], out["tot"], out["exp2"], out["det"]


@pytest.mark.parametrize("kernel", [0, 2], ids=["csr", "struct_f64sum"])
def test_step_run_and_graph_replay_identical(kernel):
    """Eager steps, drts_run and replays of a captured 8-step graph (the
    matrix-free step forks its second kernel onto another stream inside the
    capture) give the same state and series bit for bit."""
    wl = W.c2(n=16)
    a = _state_and_series(wl, 50, use_run=False, options={"kernel": kernel})
    b = _state_and_series(wl, 50, options={"kernel": kernel})
    c = _state_and_series(wl, 50, options={"graph_steps": 8, "kernel": kernel})
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(y, z)


@pytest.mark.parametrize("opts", [
    {"rows_per_tile": 64, "tiles_per_chunk": 1, "grid": 8, "xcd_remap": 0},
    {"rows_per_tile": 128, "tiles_per_chunk": 7, "grid": 24, "xcd_remap": 1},
    {"rows_per_tile": 256, "tiles_per_chunk": 64, "grid": 2048, "xcd_remap": 1},
    {"rows_per_tile": 64, "tiles_per_chunk": 3, "grid": 9, "xcd_remap": 1},
    {"rows_per_tile": 256, "tiles_per_chunk": 2, "grid": 64, "xcd_remap": 2},
    {"rows_per_tile": 128, "tiles_per_chunk": 5, "grid": 13, "xcd_remap": 2},
])
def test_launch_shapes_give_identical_states(opts):
    """Row sums do not depend on tiling (bit-exact); FP64 totals only change order."""
    wl = W.c2(n=16)
    ref = _state_and_series(wl, 40)
    got = _state_and_series(wl, 40, options=opts)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    assert np.array_equal(ref[3], got[3])
    assert np.allclose(ref[2], got[2], rtol=1e-13, atol=0)
    assert np.allclose(ref[4], got[4], rtol=1e-13, atol=0)


@pytest.mark.parametrize("rpt", [64, 128, 256])
def test_spmv_variants_give_identical_states(rpt):
    """Every SpMV variant forms the same products and adds them per row in
    column order: states bit for bit; FP64 totals differ at most in the order
    of the per-wave partial sums."""
    wl = W.c2(n=18)
    ref = _state_and_series(wl, 30, options={"rows_per_tile": rpt, "variant": drts.SPMV_ROW})
    for v in (drts.SPMV_LDS, drts.SPMV_GROUPED):
        got = _state_and_series(wl, 30, options={"rows_per_tile": rpt, "variant": v})
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]), v
        assert np.array_equal(ref[3], got[3]), v
        assert np.allclose(ref[2], got[2], rtol=1e-13, atol=0), v
        assert np.allclose(ref[4], got[4], rtol=1e-13, atol=0), v


@pytest.mark.parametrize("kernel", [0, 1, 2], ids=["csr", "struct", "struct_f64sum"])
def test_work_order_changes_nothing(kernel):
    """The XCD walk and the slab order of the chunks only move work between
    workgroups: state and FP64 series are identical bit for bit."""
    wl = W.c2(n=20)
    base = {"kernel": kernel, "rows_per_tile": 256, "tiles_per_chunk": 2, "grid": 256}
    ref = _state_and_series(wl, 30, options=dict(base, xcd_remap=0))
    for x in (1, 2):
        got = _state_and_series(wl, 30, options=dict(base, xcd_remap=x))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), x


def test_runs_are_deterministic():
    wl = W.c2(n=16)
    a = _state_and_series(wl, 60)
    b = _state_and_series(wl, 60)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_resume_from_state_is_bitexact():
    wl = W.c2(n=16)
    full = solve.run(wl, n_steps=50)
    part = solve.run(wl, n_steps=20)
    x, e, t = part["solver"].state()
    M = part["matrix"]
    S = drts.Solver(M, 1, wl.detectors, max_steps=50)
    S.set_state(x, e, t)
    S.run(solve.source_table(M, wl), 30)
    x2, e2, t2 = S.state()
    assert t2 == 50
    assert np.array_equal(x2, full["x"]) and np.array_equal(e2, full["x_exp"])
    r = S.readout(20, 30)
    assert np.array_equal(r["exp2"], full["exp2"][20:])
    assert np.array_equal(r["tot"][:, :2], full["tot"][20:, :2])


def test_rescale_is_exact_scaling():
    """With and without the power-of-two rescale the FP32 states agree exactly
    after undoing the exponent (as long as nothing underflows)."""
    wl = W.c2(n=16)
    a = solve.run(wl, n_steps=12)
    b = solve.run(wl, n_steps=12, options={"rescale": 0})
    assert b["x_exp"][0] == 0 and a["x_exp"][0] != 0
    xa = np.ldexp(a["x"].astype(np.float64), int(a["x_exp"][0]))
    assert np.array_equal(xa.astype(np.float32), b["x"])


# ---- edge cases -------------------------------------------------------------------

def test_single_voxel_grid():
    """1x1x1: 26 states, every move leaves; everything escapes in one step."""
    med = W.homogeneous(1, W.Material(10.0, 0.1, 0.9, 1.4))
    wl = W.Workload("one", med, [W.point_source(0, 0, 0)], [], 3, 1, "f64", "nearest", 1.4)
    out = solve.run(wl)
    A = oracle.Matrix(med)
    ref = oracle.run_workload(A, wl)
    assert A.n_escape == 26 and out["matrix"].n_escape == 26
    for j in range(3):
        assert parity.rel_err_series(out["tot"][:, j, 0], out["exp2"][:, 0], ref["tot"][:, j],
                                     ref["tot_exp"][:, j]) <= 1e-14


def test_ballistic_shift_on_gpu():
    """mu_s = mu_a = 0: one entry per column, the state moves exactly."""
    med = W.homogeneous(9, W.Material(0.0, 0.0, 0.5, 1.4), ny=7, nz=5)
    wl = W.Workload("ballistic", med, [W.point_source(4, 3, 2, d=(1, 1, 0))], [], 3, 1, "f32", "dither", 1.4)
    out = solve.run(wl)
    x = out["x"][:26 * 9 * 7 * 5, 0]
    nz = np.flatnonzero(x)
    d = {tuple(v): i for i, v in enumerate(W.lattice_vectors())}[(1, 1, 0)]
    assert list(nz) == [26 * (6 + 9 * (5 + 7 * 2)) + d]   # (4,3,2) + 2 (1,1,0)
    assert np.ldexp(np.float64(x[nz[0]]), int(out["x_exp"][0])) == 1.0


def test_reflecting_walls_conserve_in_fp64():
    med = W.homogeneous(7, W.Material(10.0, 0.0, 0.8, 1.4), bc="reflect")
    wl = W.Workload("box", med, [W.point_source(3, 3, 3)], [], 120, 1, "f64", "nearest", 1.4)
    out = solve.run(wl)
    N = np.ldexp(out["tot"][:, 0, 0], out["exp2"][:, 0])
    assert np.allclose(N, 1.0, rtol=1e-12)
    assert np.all(out["tot"][:, 1, 0] == 0.0)


@pytest.mark.parametrize("variant", [0, 1, 2], ids=["row", "lds", "grouped"])
def test_ragged_tail_and_tiny_tiles(variant):
    """Row counts that are not a multiple of the tile, the smallest tile."""
    med = W.homogeneous(5, W.Material(3.0, 0.05, 0.6, 1.4), ny=3, nz=7)
    wl = W.Workload("ragged", med, [W.point_source(2, 1, 3)], [W.face_escape_detector(med, "top")], 40, 1,
                    "f32", "dither", 1.4)
    A = oracle.Matrix(med)
    assert A.n_rows % 64 != 0
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl, options={"rows_per_tile": 64, "tiles_per_chunk": 1, "grid": 8, "variant": variant})
    assert parity.rel_err_series(out["det"][:, 0, 0], out["exp2"][:, 0], ref["det"][:, 0],
                                 ref["det_exp"][:, 0]) <= 1e-5
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-5


@pytest.mark.parametrize("rpt,tpc", [(64, 1), (64, 4), (256, 2)])
def test_multi_pass_tiles_between_fitting_tiles(rpt, tpc):
    """Refractive index alternating every z-plane: rows crossing a plane hold
    the transmitted and the reflected group (about 45 entries), so many tiles
    exceed the stage (28 entries per row) and take the multi-pass path between
    tiles that fit.  The LDS layout (whose y stores wait for the next tile)
    equals the plain layout bit for bit, and the oracle within 1e-5."""
    n = 6
    mp = np.zeros((n, n, n), dtype=np.uint8)
    mp[1::2] = 1
    med = W.Medium(n, n, n, 0.1, [W.Material(5.0, 0.02, 0.8, 1.33), W.Material(8.0, 0.03, 0.85, 1.45)], mp,
                   "voxels", "vacuum")
    wl = W.Workload("alternating", med, [W.point_source(3, 3, 0)], [W.face_escape_detector(med, "bottom")], 40, 1,
                    "f32", "nearest", 1.33)
    A = oracle.Matrix(med)
    rp = A.row_ptr
    per_tile = [(rp[min((k + 1) * rpt, A.n_rows)] - rp[k * rpt]) / rpt for k in range((A.n_rows + rpt - 1) // rpt)]
    assert any(a > 28 for a in per_tile) and any(a <= 27 for a in per_tile)
    got = {}
    for v in (drts.SPMV_ROW, drts.SPMV_LDS):
        got[v] = solve.run(wl, options={"rows_per_tile": rpt, "tiles_per_chunk": tpc, "grid": 16, "variant": v})
    for k in ("x", "x_exp", "tot", "exp2", "det"):
        assert np.array_equal(got[drts.SPMV_ROW][k], got[drts.SPMV_LDS][k]), k
    ref = oracle.run_workload(A, wl)
    out = got[drts.SPMV_LDS]
    assert parity.rel_err_series(out["det"][:, 0, 0], out["exp2"][:, 0], ref["det"][:, 0],
                                 ref["det_exp"][:, 0]) <= 1e-5
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-5


def test_errors_are_reported():
    wl = W.c2(n=8)
    M = drts.Matrix(wl.medium, "f32")
    S = drts.Solver(M, 1, wl.detectors, max_steps=5)
    with pytest.raises(drts.DrtsError) as ei:
        S.run(solve.source_table(M, wl), 6)
    assert ei.value.rc == -4
    with pytest.raises(drts.DrtsError):
        S.set_options(rows_per_tile=1000)
    M64 = drts.Matrix(wl.medium, "f64")
    S64 = drts.Solver(M64, 1, wl.detectors, max_steps=5)
    with pytest.raises(drts.DrtsError):
        S64.set_options(variant=drts.SPMV_LDS)       # the LDS and grouped layouts take FP32 values
    with pytest.raises(drts.DrtsError):
        S64.set_options(variant=drts.SPMV_GROUPED)
    with pytest.raises(drts.DrtsError):
        S64.set_options(variant=3)                   # no such variant
    bad = W.homogeneous(4, W.Material(1.0, 0.1, 1.5, 1.4))
    with pytest.raises(drts.DrtsError) as ei:
        drts.Matrix(bad)
    assert ei.value.rc == -1


# ---- structured (matrix-free) step -------------------------------------------------

def _struct_workload(name):
    if name == "c2_dither":
        return W.c2(n=20)
    if name == "c2_nearest":
        return W.c2(n=18, rounding="nearest")
    if name.startswith("c5_sphere"):
        wl = W.c5(n_req=1, edge=(21, 21))[0].workload
        if name.endswith("nearest"):
            wl.rounding = "nearest"
        return wl
    if name == "c1_f64":
        return W.c1(n=12)
    if name == "long_lines_nearest":
        # x-lines of 70 voxels: a full 64-voxel tile and a ragged 6-voxel one
        med = W.Medium(70, 6, 5, 0.1, [W.Material(5, 0.1, 0.8, 1.33), W.Material(15, 0.2, 0.9, 1.45)],
                       np.repeat(np.array([0, 0, 1, 1, 0], dtype=np.uint8)[:, None, None], 6, 1).repeat(70, 2),
                       "voxels", "vacuum")
        return W.Workload("long_lines", med, [W.point_source(66, 3, 0), W.point_source(5, 2, 0)],
                          [W.face_escape_detector(med, "top")], 60, 1, "f32", "nearest", 1.33)
    med = W.layered(9, [W.Material(5, 0.1, 0.8, 1.33), W.Material(15, 0.2, 0.9, 1.45),
                        W.Material(10, 0.1, 0.3, 1.4)], bc="reflect")
    rnd = "nearest" if name.endswith("nearest") else "dither"
    return W.Workload("reflect", med, [W.point_source(4, 4, 0)], [], 150, 1, "f32", rnd, 1.33)


@pytest.mark.parametrize("wl_name", ["c2_dither", "c2_nearest", "c5_sphere", "c5_sphere_nearest", "c1_f64",
                                     "reflect", "reflect_nearest", "long_lines_nearest"])
def test_structured_equals_csr(wl_name):
    """The matrix-free kernel re-derives every entry exactly as assembled:
    states and step exponents equal the CSR run bit for bit (nearest values go
    through the direction-major kernel, FP64 and dithered values through the
    gather kernel)."""
    wl = _struct_workload(wl_name)
    n = 45
    a = solve.run(wl, n_steps=n)
    b = solve.run(wl, n_steps=n, options={"kernel": 1, "tiles_per_chunk": 3}, matrix=a["matrix"])
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["x_exp"], b["x_exp"])
    assert np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["tot"], b["tot"], rtol=1e-13, atol=0)
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("wl_name", ["c2_dither", "c5_sphere", "reflect"])
def test_structured_f64sum_against_oracle(wl_name):
    """FP64 row sums: against the FP64 oracle at the FP32 tolerance, and closer
    to it than the stored-value (dithered) CSR run."""
    wl = _struct_workload(wl_name)
    n = 150
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl, n_steps=n)
    csr = solve.run(wl, n_steps=n)
    spl = solve.run(wl, n_steps=n, options={"kernel": 2}, matrix=csr["matrix"])
    D = A.n_states
    e_csr = parity.rel_l1(csr["x"][:D, 0], csr["x_exp"][0], ref["x"], ref["x_exp"])
    e_spl = parity.rel_l1(spl["x"][:D, 0], spl["x_exp"][0], ref["x"], ref["x_exp"])
    print(wl_name, "state rel L1: csr", e_csr, "f64sum", e_spl)
    assert e_spl <= 1e-5 and e_spl <= e_csr * 1.5
    for j in range(3):
        err = parity.rel_err_series(spl["tot"][:, j, 0], spl["exp2"][:, 0], ref["tot"][:, j], ref["tot_exp"][:, j])
        assert err <= 1e-5, (j, err)
    for d in range(len(wl.detectors)):
        err = parity.rel_err_series(spl["det"][:, d, 0], spl["exp2"][:, 0], ref["det"][:, d], ref["det_exp"][:, d])
        assert err <= 1e-5, (d, err)
