"""The CSR step by row groups (rows with equal column lists share one read of
their columns and one gather of x) against the tiled and row-by-row steps,
for many right-hand sides and for one.

Bar: bit-exact state, exponents and exponent series, FP64 series to 1e-13
(the chunk partials are summed in another order), on media whose rows group
in different ways: the homogeneous slab (whole groups of 26 rows), Fresnel
layers and a sphere (interface rows that split off their voxel's group),
reflecting walls, scattering order 3 (rows wider than one voxel), crossing
within the step, and a Lebedev-86 medium (rows that do not group: the
library takes its other step); with one, few and 64 right-hand sides,
sources in several rows of a group and detectors on escape and state rows.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _mat():
    return W.Material(10.0, 0.05, 0.85, 1.4)


def _layers(n):
    return W.layered(n, [W.Material(5.0, 0.02, 0.8, 1.33), W.Material(15.0, 0.1, 0.9, 1.45),
                         W.Material(10.0, 0.05, 0.85, 1.40)])


def _sphere(n):
    return W.sphere_inclusion(n, W.Material(10.0, 0.01, 0.9, 1.33), W.Material(10.0, 0.08, 0.9, 1.45),
                              (n / 2 - 0.7, n / 2 + 0.1, n / 2 - 0.3), n / 3.5)


def _order3(n):
    m = W.homogeneous(n, _mat())
    m.scatter_order = 3
    return m


def _substep(n):
    m = _layers(n)
    m.interface = "substep"
    return m


def _leb(n):
    m = W.homogeneous(n, _mat())
    m.directions = "lebedev86"
    return m


def _layers17(n):
    # more materials than the value-indexed step has dictionaries: the fast
    # groups' values stream as FP32
    return W.layered(n, [W.Material(5.0 + i, 0.01 * (i + 1), 0.8, 1.4) for i in range(17)])


MEDIA = [("slab", lambda n: W.homogeneous(n, _mat(), nz=n - 3)),
         ("layers", _layers),
         ("sphere", _sphere),
         ("reflect", lambda n: W.homogeneous(n, _mat(), bc="reflect")),
         ("order3", _order3),
         ("substep", _substep),
         ("layers17", _layers17),
         ("lebedev", _leb)]


def _workload(med, k, steps, seed):
    r = np.random.default_rng([161108536, seed])
    srcs = []
    for j in range(k):
        x, y = (int(v) for v in r.integers(1, med.nx - 1, size=2))
        kind = "gaussian" if j % 2 else "impulse"
        srcs.append(W.point_source(x, y, 0, kind=kind, fwhm_fs=float(r.uniform(50, 300)), rhs=j))
        if j % 3 == 0:
            # a second source row of the same voxel (another direction) feeds the same rhs
            srcs.append(W.point_source(x, y, 0, d=(1, 0, 1), rhs=j, w=0.5))
        # an interior source: its row is a member of a full lattice group
        # (the face rows above are empty rows, taken one by one)
        srcs.append(W.point_source(x, y, med.nz // 2, d=(0, 1, 1), rhs=j, w=0.25))
    dets = []
    if med.directions == "lattice26" and med.bc == "vacuum":
        dets = [W.face_escape_detector(med, "top"), W.face_escape_detector(med, "bottom", 1, med.nx - 2)]
        c = med.nx // 2
        lv = W.lattice_vectors()
        dets.append(W.Detector(np.array([[c, c, 1]] * 3), lv[[0, 12, 25]], np.zeros(3, dtype=bool),
                               np.array([1.0, 2.0, 0.5]), "state"))
    return W.Workload("grouped", med, srcs, dets, steps, k, "f32", "dither", 1.4)


@pytest.mark.parametrize("k", [5, 64])
@pytest.mark.parametrize("name,make", MEDIA, ids=[m[0] for m in MEDIA])
def test_grouped_equals_row_by_row(name, make, k):
    n = 7 if name == "lebedev" else 12
    wl = _workload(make(n), k, 40, 7 + k)
    print("%s %d^3, %d rhs" % (name, n, k), flush=True)
    a = solve.run(wl, options={"variant": drts.SPMM_GROUPED})
    b = solve.run(wl, matrix=a["matrix"], options={"variant": drts.SPMM_ROWS})
    assert np.array_equal(a["x"].view(np.uint32), b["x"].view(np.uint32))
    assert np.array_equal(a["x_exp"], b["x_exp"]) and np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["tot"], b["tot"], rtol=1e-13, atol=0)
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)
    assert (a["tot"][:, 0, :] > 0).any()
    a["solver"].close()
    b["solver"].close()


@pytest.mark.parametrize("opts", [{"rows_per_tile": 16, "tiles_per_chunk": 1, "grid": 24, "xcd_remap": 1},
                                  {"rows_per_tile": 256, "tiles_per_chunk": 1000, "grid": 3, "xcd_remap": 0}])
def test_grouped_launch_shapes(opts):
    """Many small work items (fewer groups than some items hold) and one item
    holding every group."""
    wl = _workload(_sphere(10), 9, 25, 3)
    a = solve.run(wl, options={"variant": drts.SPMM_ROWS})
    b = solve.run(wl, matrix=a["matrix"], options=dict(opts, variant=drts.SPMM_GROUPED))
    assert np.array_equal(a["x"].view(np.uint32), b["x"].view(np.uint32))
    assert np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)


def _single(wl):
    import copy
    w = copy.copy(wl)
    w.sources = [copy.copy(x) for x in wl.sources if x.rhs == 0]
    w.n_rhs = 1
    return w


@pytest.mark.parametrize("name,make", MEDIA, ids=[m[0] for m in MEDIA])
def test_grouped_spmv_equals_tiled(name, make):
    n = 7 if name == "lebedev" else 13
    wl = _single(_workload(make(n), 1, 40, 5))
    print("%s %d^3, one rhs" % (name, n), flush=True)
    a = solve.run(wl, options={"variant": drts.SPMV_GROUPED})
    b = solve.run(wl, matrix=a["matrix"], options={"variant": drts.SPMV_LDS})
    c = solve.run(wl, matrix=a["matrix"], options={"variant": drts.SPMV_ROW})
    for o in (b, c):
        assert np.array_equal(a["x"].view(np.uint32), o["x"].view(np.uint32))
        assert np.array_equal(a["x_exp"], o["x_exp"]) and np.array_equal(a["exp2"], o["exp2"])
        assert np.allclose(a["tot"], o["tot"], rtol=1e-13, atol=0)
        assert np.allclose(a["det"], o["det"], rtol=1e-13, atol=0)
    assert (a["tot"][:, 0, :] > 0).any()
    # the group counts: every row is a member of one group; a fast group's
    # members hold 26 entries, the other rows' entries are counted apart
    M = a["matrix"]
    if name == "lebedev":
        # rows of hundreds of entries take the wave-per-row step: no groups are built
        assert M.groups() is None
    else:
        g = M.groups()
        assert 0 < g["n_groups"] <= M.n_rows and 0 <= g["n_fast"] <= g["n_groups"]
        n_fast_rows = M.n_rows - g["n_vox2_rows"] - g["n_list_rows"]
        assert n_fast_rows >= 0
        assert M.nnz == 26 * n_fast_rows + 52 * g["n_vox2_rows"] + g["n_list_entries"]
        if name in ("layers", "sphere"):
            # Fresnel interfaces: rows with a transmitted and a reflected part
            assert g["n_vox2_rows"] > 0
        # value-indexed fast groups: a dictionary per material, unless there
        # are more than 16 materials; on the sphere the crossing rows' Fresnel
        # factors vary with the normal, more than 256 values a material, and
        # the values stream as FP32 (both paths equal the tiled step above)
        n_mat = len(a["matrix"].medium.materials)
        if name != "sphere":
            assert g["value_tables"] == (0 if name == "layers17" or g["n_fast"] == 0 else n_mat), g
    if name == "slab":
        # one medium, no interfaces: each voxel's 26 rows (state or escape)
        # form one fast group; the other rows are the empty rows of face
        # states that cannot be entered, as many as the escape rows
        assert g["n_fast"] == M.n_states // 26 and g["n_vox2_rows"] == 0
        assert g["n_list_entries"] == 0 and g["n_list_rows"] == M.n_escape
    for o in (a, b, c):
        o["solver"].close()


@pytest.mark.parametrize("opts", [{"rows_per_tile": 64, "tiles_per_chunk": 1, "grid": 24, "xcd_remap": 1},
                                  {"rows_per_tile": 256, "tiles_per_chunk": 64, "grid": 3, "xcd_remap": 0},
                                  {"rows_per_tile": 128, "tiles_per_chunk": 2, "graph_steps": 7}])
def test_grouped_spmv_launch_shapes(opts):
    """Work items of a group or two, a handful of workgroups holding every
    group, and graph replay."""
    wl = _single(_workload(_sphere(11), 1, 25, 4))
    a = solve.run(wl, options={"variant": drts.SPMV_LDS})
    b = solve.run(wl, matrix=a["matrix"], options=dict(opts, variant=drts.SPMV_GROUPED))
    assert np.array_equal(a["x"].view(np.uint32), b["x"].view(np.uint32))
    assert np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)


def test_grouped_spmv_wide_planes_keep_group_order():
    """Planes too wide for the brick order (400 x 400 voxels: consecutive
    fast groups of a brick would lie beyond the FP32 step's 32-bit value
    offsets): no bricks, so no value indexing; the FP32 grouped step in group
    order equals the tiled step bit for bit."""
    med = W.homogeneous(400, _mat(), nz=3)
    wl = W.Workload("wide", med, [W.point_source(200, 200, 1, d=(0, 1, 1))], [], 6, 1, "f32", "dither", 1.4)
    a = solve.run(wl, options={"variant": drts.SPMV_GROUPED})
    g = a["matrix"].groups()
    print("400 x 400 x 3:", g, flush=True)
    assert g["n_fast"] > 0 and g["value_tables"] == 0
    b = solve.run(wl, matrix=a["matrix"], options={"variant": drts.SPMV_LDS})
    assert np.array_equal(a["x"].view(np.uint32), b["x"].view(np.uint32))
    assert np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["tot"], b["tot"], rtol=1e-13, atol=0)
    for o in (a, b):
        o["solver"].close()
