"""Many right-hand sides (SpMM), uneven batches and the autotuner, through the C ABI.

Bars: each right-hand side against the FP64 oracle run of its own sources
(1e-5), with FP32 and with FP64 row sums; each SpMM column against the
single-rhs SpMV run of the same source (bit-exact state: the per-row sums are
the same operations in the same order); one step of either sum bit-exact
against its sum written out over the oracle's FP32 values;
each batch member against the same solver run alone (bit-exact state and
series), with the CSR step (small members in the shared tiled launch, a large
one on its own grouped step) and with the matrix-free step; autotuned launch
shapes against the defaults (bit-exact state).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _single(wl, j):
    """The workload restricted to the sources of rhs j, as one rhs."""
    import copy
    w = copy.copy(wl)
    w.sources = [copy.copy(s) for s in wl.sources if s.rhs == j]
    for s in w.sources:
        s.rhs = 0
    w.n_rhs = 1
    return w


def test_spmm_columns_equal_spmv_runs():
    wl = W.c3(n=20, k=8, n_steps=80)
    out = solve.run(wl)
    for j in (0, 3, 7):
        one = solve.run(_single(wl, j), matrix=out["matrix"])
        assert np.array_equal(out["x"][:, j], one["x"][:, 0]), j
        assert out["x_exp"][j] == one["x_exp"][0]
        assert np.array_equal(out["exp2"][:, j], one["exp2"][:, 0])
        assert np.allclose(out["tot"][:, :, j], one["tot"][:, :, 0], rtol=1e-13, atol=0)
        assert np.allclose(out["det"][:, :, j], one["det"][:, :, 0], rtol=1e-13, atol=0)


def _rows_summed(A, v32, x, f64):
    """[A; L] x with each row summed in column order from the oracle's FP32
    values: in FP32 (every product and every sum rounded) or in FP64 (the
    products of two FP32 numbers are exact there) and rounded once to FP32."""
    rp, col = A.row_ptr, A.col
    lens = np.diff(rp)
    dt = np.float64 if f64 else np.float32
    acc = np.zeros((A.n_rows, x.shape[1]), dtype=dt)
    for j in range(int(lens.max())):
        rows = np.flatnonzero(lens > j)
        e = rp[rows] + j
        acc[rows] = acc[rows] + v32[e].astype(dt)[:, None] * x[col[e]].astype(dt)
    return acc.astype(np.float32)


@pytest.mark.parametrize("variant", [drts.SPMM_GROUPED, drts.SPMM_GROUPED_F64SUM], ids=["f32sum", "f64sum"])
def test_spmm_one_step_rows_bitexact(variant):
    """A three-layer medium (fast groups, two-voxel Fresnel rows, face and
    escape rows), 8 seeded right-hand sides, one step."""
    wl = W.c2(n=14, n_steps=2)
    A = oracle.Matrix(wl.medium)
    v32 = A.round_f32(wl.rounding)
    k = 8
    x = np.stack([W.seeded_state(A.n_rows, 40 + j) for j in range(k)], axis=1).astype(np.float32)
    M = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(M, k, [], max_steps=2)
    S.set_options(variant=variant)
    assert S.options["variant"] == variant
    e0 = np.zeros(k, dtype=np.int32)
    S.set_state(x, e0, 0)
    S.step(None)
    y, e1, t = S.state()
    assert t == 1
    want = _rows_summed(A, v32, x, variant == drts.SPMM_GROUPED_F64SUM).astype(np.float64)
    got = np.ldexp(y.astype(np.float64), (e1 - e0)[None, :])
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad.shape[0], bad[:5].tolist())
    S.close()
    M.close()


def test_spmm_f64sum_needs_rows_that_group():
    """Rows of several hundred entries (Lebedev-86) take no FP64-sum SpMM; the
    options stay as they were."""
    med = W.homogeneous(5, W.Material(10.0, 0.02, 0.85, 1.4))
    med.directions = "lebedev86"
    M = drts.Matrix(med, "f32", "dither", 1.4)
    S = drts.Solver(M, 2, [], max_steps=2)
    with pytest.raises(drts.DrtsError):
        S.set_options(variant=drts.SPMM_GROUPED_F64SUM)
    assert S.options["variant"] == drts.SPMM_GROUPED
    S.close()
    M.close()


@pytest.mark.parametrize("variant", [drts.SPMM_GROUPED, drts.SPMM_GROUPED_F64SUM], ids=["f32sum", "f64sum"])
def test_spmm_64_rhs_against_oracle(variant):
    wl = W.c3(n=24, k=64, n_steps=60)
    out = solve.run(wl, options={"variant": variant})
    A = oracle.Matrix(wl.medium)
    for j in (0, 17, 40, 63):
        ref = oracle.run_workload(A, wl, rhs=j)
        e = out["exp2"][:, j]
        for d in range(16):
            err = parity.rel_err_series(out["det"][:, d, j], e, ref["det"][:, d], ref["det_exp"][:, d])
            assert err <= 1e-5, (j, d, err)
        for c in range(3):
            err = parity.rel_err_series(out["tot"][:, c, j], e, ref["tot"][:, c], ref["tot_exp"][:, c])
            assert err <= 1e-5, (j, c, err)
        assert parity.rel_l1(out["x"][:A.n_states, j], out["x_exp"][j], ref["x"], ref["x_exp"]) <= 1e-5


@pytest.mark.parametrize("opts", [{"rows_per_tile": 16, "tiles_per_chunk": 5, "grid": 40, "xcd_remap": 1},
                                  {"rows_per_tile": 200, "tiles_per_chunk": 300, "grid": 7, "xcd_remap": 0}])
def test_spmm_launch_shapes(opts):
    wl = W.c3(n=16, k=5, n_steps=30)
    a = solve.run(wl)
    b = solve.run(wl, options=opts)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["exp2"], b["exp2"])
    assert np.allclose(a["det"], b["det"], rtol=1e-13, atol=0)


def _c4_small(n_inst=9, edge=(6, 15)):
    return W.c4(n_inst=n_inst, n_steps=60, edge=edge)


def test_batch_members_equal_solo_runs():
    wls = _c4_small()
    steps = [60, 45, 60, 10, 33, 60, 1, 59, 20]
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, w.detectors, max_steps=60) for m, w in zip(mats, wls)]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    B.run(tabs, steps)
    for i, (w, m, S) in enumerate(zip(wls, mats, solvers)):
        solo = solve.run(w, n_steps=steps[i], matrix=m, options={"variant": drts.SPMV_LDS})
        x, e, t = S.state()
        assert t == steps[i]
        assert np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"]), i
        r = S.readout(0, steps[i])
        assert np.array_equal(r["tot"], solo["tot"]) and np.array_equal(r["exp2"], solo["exp2"]), i


def test_batch_large_member_takes_its_own_grouped_step():
    """A member of at least BATCH_OWN_ROWS rows (a 40^3 cube) keeps the step by
    row groups inside the batch while the small members share the tiled
    launch: after the batch autotuner, through graph-replayed segments (more
    than 50 steps) and members dropping out on both sides, every member equals
    its solo run with the same step, bit for bit (state, exponent, series)."""
    big = W.c4(n_inst=1, n_steps=80, edge=(40, 40))[0]
    small = _c4_small(n_inst=3)
    wls = [small[0], big, small[1], small[2]]
    steps = [80, 60, 7, 80]
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    assert mats[1].n_rows >= drts.BATCH_OWN_ROWS
    assert all(mats[i].n_rows < drts.BATCH_OWN_ROWS for i in (0, 2, 3))
    solvers = [drts.Solver(m, 1, w.detectors, max_steps=80) for m, w in zip(mats, wls)]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    chosen = B.autotune()
    keys = ("rows_per_tile", "tiles_per_chunk", "variant")
    assert solvers[1].options["variant"] == drts.SPMV_GROUPED
    for i in (0, 2, 3):
        assert {k: solvers[i].options[k] for k in keys} == {k: chosen[k] for k in keys}
    B.run(tabs, steps)
    B.close()
    assert mats[1].groups() is not None
    for i, (w, m, S) in enumerate(zip(wls, mats, solvers)):
        opts = None if i == 1 else {k: chosen[k] for k in keys}
        solo = solve.run(w, n_steps=steps[i], matrix=m, options=opts)
        x, e, t = S.state()
        assert t == steps[i]
        assert np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"]), i
        r = S.readout(0, steps[i])
        assert np.array_equal(r["tot"], solo["tot"]) and np.array_equal(r["exp2"], solo["exp2"]), i
        solo["solver"].close()
    for S in solvers:
        S.close()
    for m in mats:
        m.close()


def test_batch_autotune_keeps_results():
    """drts_batch_autotune before the first step: every member gets the one
    chosen shape, the tuning steps leave no trace in state or series, and each
    member then equals its solo run with the chosen options, bit for bit."""
    wls = _c4_small(n_inst=7, edge=(6, 14))
    steps = [40, 25, 40, 7, 33, 40, 1]
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, w.detectors, max_steps=40) for m, w in zip(mats, wls)]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    chosen = B.autotune()
    assert chosen["rows_per_tile"] in (64, 128, 256) and chosen["grid"] > 0
    keys = ("rows_per_tile", "tiles_per_chunk", "variant")
    for S in solvers:
        assert {k: S.options[k] for k in keys} == {k: chosen[k] for k in keys}
    B.run(tabs, steps)
    for i, (w, m, S) in enumerate(zip(wls, mats, solvers)):
        solo = solve.run(w, n_steps=steps[i], matrix=m, options={k: chosen[k] for k in keys})
        x, e, t = S.state()
        assert t == steps[i]
        assert np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"]), i
        r = S.readout(0, steps[i])
        assert np.array_equal(r["tot"], solo["tot"]) and np.array_equal(r["exp2"], solo["exp2"]), i
    with pytest.raises(drts.DrtsError):
        B.autotune()          # members have stepped


def _mf_batch(kernel, n=6):
    """Sphere-inclusion media (Fresnel interfaces, detectors), nearest-rounded
    values, as matrix-free solvers with the given kernel."""
    import dataclasses
    reqs = W.c5(n_req=n, rate=1e6, edge=(10, 16), steps=(30, 60))
    wls = [dataclasses.replace(q.workload, rounding="nearest") for q in reqs]
    opts = {"kernel": kernel, "tiles_per_chunk": 2}
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, w.detectors, max_steps=w.n_steps) for m, w in zip(mats, wls)]
    for S in solvers:
        S.set_options(**opts)
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    return wls, mats, solvers, tabs, opts


@pytest.mark.parametrize("kernel", [1, 2], ids=["exact", "f64sum"])
def test_matrix_free_batch_members_equal_solo_runs(kernel):
    """Matrix-free members advanced together (one launch per kernel and step)
    equal the same solvers run alone: states, exponents, totals and detector
    series bit for bit."""
    wls, mats, solvers, tabs, opts = _mf_batch(kernel)
    steps = [w.n_steps for w in wls]
    B = drts.Batch(solvers)
    B.run(tabs, steps)
    for i, (w, m, S) in enumerate(zip(wls, mats, solvers)):
        solo = solve.run(w, n_steps=steps[i], matrix=m, options=opts)
        x, e, t = S.state()
        assert t == steps[i]
        assert np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"]), i
        r = S.readout(0, steps[i])
        for k in ("tot", "exp2", "det"):
            assert np.array_equal(r[k], solo[k]), (i, k)


def test_matrix_free_batch_against_oracle():
    wls, mats, solvers, tabs, _ = _mf_batch(2, n=4)
    B = drts.Batch(solvers)
    B.run(tabs, [w.n_steps for w in wls])
    for i, w in enumerate(wls):
        ref = oracle.run_workload(oracle.Matrix(w.medium), w)
        r = solvers[i].readout(0, w.n_steps)
        err = parity.rel_err_series(r["tot"][:, 0, 0], r["exp2"][:, 0], ref["tot"][:, 0], ref["tot_exp"][:, 0])
        assert err <= 1e-5, (i, err)
        err = parity.rel_err_series(r["det"][:, 0, 0], r["exp2"][:, 0], ref["det"][:, 0], ref["det_exp"][:, 0])
        assert err <= 1e-5, (i, "det", err)


def test_batch_against_oracle_and_continues():
    wls = _c4_small(n_inst=5, edge=(8, 12))
    mats = [drts.Matrix(w.medium, w.value_type, w.rounding, w.n_ref) for w in wls]
    solvers = [drts.Solver(m, 1, w.detectors, max_steps=60) for m, w in zip(mats, wls)]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    B.run(tabs, [30] * 5)
    B.run(tabs, [30, 0, 30, 30, 30])      # solver 1 idles, the others continue
    for i, w in enumerate(wls):
        A = oracle.Matrix(w.medium)
        n = 30 if i == 1 else 60
        ref = oracle.run_workload(A, w, n_steps=n)
        x, e, t = solvers[i].state()
        assert t == n
        r = solvers[i].readout(0, n)
        err = parity.rel_err_series(r["tot"][:, 0, 0], r["exp2"][:, 0], ref["tot"][:, 0], ref["tot_exp"][:, 0])
        assert err <= 1e-5, (i, err)
        assert parity.rel_l1(x[:A.n_states, 0], e[0], ref["x"], ref["x_exp"]) <= 1e-5


def test_batch_rejects_mixed_inputs():
    w32 = W.c4(n_inst=1, n_steps=5, edge=(6, 6))[0]
    m32 = drts.Matrix(w32.medium, "f32")
    m64 = drts.Matrix(w32.medium, "f64")
    s32 = drts.Solver(m32, 1, [], max_steps=5)
    s64 = drts.Solver(m64, 1, [], max_steps=5)
    with pytest.raises(drts.DrtsError):
        drts.Batch([s32, s64])
    with pytest.raises(drts.DrtsError):
        drts.Batch([s32, s32])
    # every member needs the same step: CSR with matrix-free (the exact
    # matrix-free step of dithered values, mode 0, or FP64 row sums) is refused,
    # and so is a batch of mode-0 members (the gather kernel has no batch form)
    m_mf = drts.Matrix(w32.medium, "f32")
    s_mf = drts.Solver(m_mf, 1, [], max_steps=5)
    B = drts.Batch([s32, s_mf])
    for k in (drts.KERNEL_STRUCTURED, drts.KERNEL_STRUCTURED_F64SUM):
        s_mf.set_options(kernel=k)
        with pytest.raises(drts.DrtsError):
            B.autotune()
        with pytest.raises(drts.DrtsError):
            B.run([None, None], [2, 2])
    s32.set_options(kernel=drts.KERNEL_STRUCTURED)
    s_mf.set_options(kernel=drts.KERNEL_STRUCTURED)
    with pytest.raises(drts.DrtsError):
        B.run([None, None], [2, 2])
    s32.set_options(kernel=drts.KERNEL_CSR)
    s_mf.set_options(kernel=drts.KERNEL_CSR)
    B.run([None, None], [2, 2])
    assert s32.state()[2] == 2 and s_mf.state()[2] == 2


def test_autotune_keeps_results_and_caches(tmp_path):
    wl = W.c2(n=20, n_steps=30)
    ref = solve.run(wl)
    M = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(M, 1, wl.detectors, max_steps=30)
    cache = str(tmp_path / "tune.txt")
    chosen = S.autotune(cache)
    assert chosen["rows_per_tile"] in (64, 128, 256)
    S.run(solve.source_table(M, wl), 30)
    x, e, t = S.state()
    assert np.array_equal(x, ref["x"]) and np.array_equal(e, ref["x_exp"])
    assert open(cache).read().strip()
    S2 = drts.Solver(M, 1, wl.detectors, max_steps=30)
    again = S2.autotune(cache)
    assert again == chosen
