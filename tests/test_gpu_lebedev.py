"""Lebedev-86 directions with the multi-voxel weights of Eq. (18)-(19) on the
GPU: the paper's own discretisation, whose rows hold several hundred entries.

Bars:
  - device assembly bit-exact against the oracle (row pointers, columns, FP64
    values, FP32 values under both roundings) on small media: homogeneous and
    layered, light paths of one and of 0.6 voxels per step;
  - FP64 steps within 1e-12 and FP32 steps within 1e-5 of the FP64 oracle
    (totals and state), with the same-matrix error printed beside it;
  - the 64^3 medium (22.5M states, about 14 billion entries, int64 row
    pointers) in the launch configuration the benchmark times: sampled rows
    (random, first and last, escape) bit-exact against the oracle's single-row
    function, one product at the sampled rows within the FP32 summation
    bound, and the energy balance of the first steps;
  - a batch of Lebedev members equals their solo runs bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _leb(med, c_dt=1.0):
    med.directions = "lebedev86"
    med.c_dt = c_dt
    return med


def _media():
    lay = [W.Material(5.0, 0.05, 0.8, 1.4), W.Material(15.0, 0.2, 0.9, 1.4), W.Material(10.0, 0.1, 0.6, 1.4)]
    return [("homog6", _leb(W.homogeneous(6, W.Material(10.0, 0.01, 0.9, 1.4)))),
            ("layers7", _leb(W.layered(7, lay))),
            ("slab_c06", _leb(W.homogeneous(5, W.Material(20.0, 0.1, 0.7, 1.4), ny=6, nz=4), 0.6))]


MEDIA = _media()


@pytest.mark.parametrize("name,med", MEDIA, ids=[m[0] for m in MEDIA])
@pytest.mark.parametrize("vt,rnd", [("f64", "nearest"), ("f32", "nearest"), ("f32", "dither")])
def test_lebedev_assembly_bitexact(name, med, vt, rnd):
    A = oracle.Matrix(med)
    M = drts.Matrix(med, vt, rnd, 1.4)
    assert (M.n_states, M.n_escape, M.nnz) == (A.n_states, A.n_escape, A.nnz)
    rp, col, val = M.export_rows()
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(col, A.col)
    want = A.val if vt == "f64" else A.round_f32(rnd)
    assert np.array_equal(val.view(np.uint8), want.view(np.uint8))
    M.close()


def _impulse(med, n_steps, vt="f64"):
    c = med.nx // 2
    return W.Workload("leb", med, [W.point_source(c, c, 1)], [], n_steps, 1, vt, "dither", 1.4)


def test_lebedev_fp64_parity():
    wl = _impulse(_leb(W.homogeneous(8, W.Material(10.0, 0.01, 0.9, 1.4))), 40)
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl)
    out = solve.run(wl)
    e = out["exp2"][:, 0]
    for j in range(3):
        assert parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j]) <= 1e-12
    assert parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"]) <= 1e-12


@pytest.mark.parametrize("c_dt", [1.0, 0.6])
def test_lebedev_fp32_parity(c_dt):
    """Three layers, a Gaussian top-face source in +z (the nearest rule
    direction), FP32 dithered values."""
    lay = [W.Material(5.0, 0.05, 0.8, 1.4), W.Material(15.0, 0.2, 0.9, 1.4), W.Material(10.0, 0.1, 0.6, 1.4)]
    base = W.c2(n=12, n_steps=60)
    med = _leb(W.layered(12, lay), c_dt)
    wl = W.Workload("leb_layers", med, base.sources, [], 60, 1, "f32", "dither", 1.4)
    A = oracle.Matrix(med)
    ref = oracle.run_workload(A, wl)
    same = oracle.run_workload(A, wl, vals32=A.round_f32("dither"))
    out = solve.run(wl)
    e = out["exp2"][:, 0]
    errs, errs_same = [], []
    for j in range(3):
        errs.append(parity.rel_err_series(out["tot"][:, j, 0], e, ref["tot"][:, j], ref["tot_exp"][:, j]))
        errs_same.append(parity.rel_err_series(out["tot"][:, j, 0], e, same["tot"][:, j], same["tot_exp"][:, j]))
    l1 = parity.rel_l1(out["x"][:A.n_states, 0], out["x_exp"][0], ref["x"], ref["x_exp"])
    print("lebedev c_dt %.1f: series %.3g (same-matrix %.3g), state L1 %.3g" % (c_dt, max(errs), max(errs_same), l1))
    assert max(errs) <= 1e-5 and l1 <= 1e-5


def test_lebedev_batch_members_equal_solo_runs():
    meds = [_leb(W.homogeneous(n, W.Material(10.0, 0.02, 0.85, 1.4))) for n in (5, 7, 6)]
    wls = [_impulse(m, 20, "f32") for m in meds]
    mats = [drts.Matrix(w.medium, "f32", "dither", 1.4) for w in wls]
    solvers = [drts.Solver(m, 1, [], max_steps=20) for m in mats]
    tabs = [solve.source_table(m, w) for m, w in zip(mats, wls)]
    B = drts.Batch(solvers)
    B.run(tabs, [20, 12, 20])
    B.close()
    for i, n in enumerate((20, 12, 20)):
        solo = solve.run(wls[i], n_steps=n, matrix=mats[i])
        x, e, t = solvers[i].state()
        assert t == n and np.array_equal(x, solo["x"]) and np.array_equal(e, solo["x_exp"])
        solo["solver"].close()


def test_lebedev_64_full_size_sampled():
    med = _leb(W.homogeneous(64, W.Material(10.0, 0.01, 0.9, 1.4)))
    print("lebedev 64^3: assembling", flush=True)
    M = drts.Matrix(med, "f32", "dither", 1.4)
    R = oracle.LebedevRows(med)
    assert (M.n_states, M.n_rows) == (R.n_states, R.n_rows)
    print("lebedev 64^3: %d rows, %d entries (%.0f per row)" % (M.n_rows, M.nnz, M.nnz / M.n_rows), flush=True)
    assert M.nnz > 2 ** 31
    rng = np.random.default_rng([161108536, 86])
    rows = np.unique(np.concatenate([rng.integers(0, M.n_states, 300), [0, M.n_states - 1],
                                     rng.integers(M.n_states, M.n_rows, 40)]))
    x = np.zeros(M.n_rows, dtype=np.float32)
    x[:M.n_states] = W.seeded_state(M.n_states, 86).astype(np.float32)
    for r in rows:
        rp, col, val = M.export_rows(int(r), 1)
        c_o, v_o = R.row(int(r))
        assert np.array_equal(col, c_o), r
        v32 = np.array([oracle_round(v, r, c) for v, c in zip(v_o, c_o)], dtype=np.float32)
        assert np.array_equal(val, v32), r
    # one product at the sampled rows
    S = drts.Solver(M, 1, [], max_steps=4)
    S.set_state(x, [0], 0)
    S.step(None)
    y, e, t = S.state()
    for r in rows:
        _, col, val = M.export_rows(int(r), 1)
        terms = val.astype(np.float64) * x[col].astype(np.float64)
        got = np.ldexp(float(y[r, 0]), int(e[0]))
        assert abs(got - terms.sum()) <= 64 * 2.0 ** -24 * np.abs(terms).sum() + 1e-300, r
    # energy balance of the next steps: N(t+1) = N(t) - absorbed - escaped
    S.run(None, 3)
    out = S.readout(0, 4)
    tot = np.ldexp(out["tot"][:, :, 0], out["exp2"][:, :1])
    for k in range(1, 4):
        assert abs(tot[k, 0] - (tot[k - 1, 0] - tot[k, 2] - tot[k, 1])) <= 1e-5 * tot[k - 1, 0]
    S.close()
    R.close()
    M.close()


_splitmix = []


def oracle_round(a, row, col):
    """The FP32 value the dithered rounding gives the FP64 entry a at (row,
    col): the oracle's rule for one entry, with the oracle's splitmix64
    (pinned against its published sequence)."""
    import ctypes
    if not _splitmix:
        f = oracle._load().or_splitmix64_value
        f.restype = ctypes.c_uint64
        f.argtypes = [ctypes.c_uint64]
        _splitmix.append(f)
    f = np.float32(a)
    if float(f) == a:
        return f
    g = np.nextafter(f, np.float32(np.inf) if float(f) < a else np.float32(-np.inf))
    p = abs(float(f) - a) / abs(float(g) - float(f))
    u = (_splitmix[0](((int(row) << 32) ^ int(col)) & (2 ** 64 - 1)) >> 11) * 2.0 ** -53
    return g if u < p else f
