"""Windowed measurement and sensors outside the volume (Eq. (27), Sec. 4.2)
on the GPU.

  - drts_detector_window (the FIR of a solver's FP64 detector series by each
    sensor's impulse response, on the device) equals the oracle's plain FIR
    of the same series within 1e-13, and the oracle's FIR of its own series
    within the FP32 gate 1e-5; for a causal and a symmetric window, one and
    several right-hand sides;
  - a medium extended by free space above its surface, with the sensor on
    the extension's top face: assembly bit-exact against the oracle, the
    sensor's series within 1e-5 of the oracle, and equal to the original's
    visible top-face escape flux delayed by the gap.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402


def _response(n, width):
    t = np.arange(n)
    return np.exp(-0.5 * ((t - n // 2) / width) ** 2)


@pytest.mark.parametrize("tap0", [0, -7])
def test_window_kernel_against_oracle_fir(tap0):
    wl = W.c2(n=20, n_steps=150)
    out = solve.run(wl)
    S = out["solver"]
    taps = np.stack([_response(15, 2.0), _response(15, 4.0)])
    val, e = S.window(taps, tap0=tap0)
    got = np.ldexp(val[:, :, 0], e[:, :, 0])
    # the oracle's FIR of the library's own series: the FIR alone
    own = oracle.window(out["det"][:, :, 0], np.repeat(out["exp2"][:, :1], 2, axis=1), taps, tap0)
    assert np.allclose(got, own, rtol=1e-13, atol=0)
    # against the FP64 oracle end to end
    A = oracle.Matrix(wl.medium)
    ref = oracle.run_workload(A, wl)
    want = oracle.window(ref["det"], ref["det_exp"], taps, tap0)
    keep = want > 1e-30 * want.max()
    err = float(np.max(np.abs(got[keep] - want[keep]) / want[keep]))
    print("window tap0 %d: FP32 run vs FP64 oracle %.3g" % (tap0, err))
    assert err <= 1e-5
    S.close()


def test_window_kernel_many_rhs():
    wl = W.c3(n=16, k=5, n_steps=60)
    out = solve.run(wl)
    S = out["solver"]
    taps = _response(9, 1.5)[None, :]
    val, e = S.window(taps, tap0=-2)
    for k in range(5):
        own = oracle.window(out["det"][:, :, k], np.repeat(out["exp2"][:, k:k + 1], S.n_det, axis=1),
                            np.repeat(taps, S.n_det, axis=0), -2)
        assert np.allclose(np.ldexp(val[:, :, k], e[:, :, k]), own, rtol=1e-13, atol=0), k
    S.close()


def test_outside_sensor_on_free_space_extension():
    gap, T = 4, 120
    base = W.c2(n=16, n_steps=T)
    ext = W.extend_top(base.medium, gap)
    sensor = W.face_escape_detector(ext, "top")
    we = W.Workload("ext", ext, [W.shifted_z(s, gap) for s in base.sources], [sensor], T,
                    n_ref=base.n_ref)
    A = oracle.Matrix(ext)
    M = drts.Matrix(ext, "f32", "dither", base.n_ref)
    rp, col, val = M.export_rows()
    assert np.array_equal(rp, A.row_ptr) and np.array_equal(col, A.col)
    assert np.array_equal(val.view(np.uint8), A.round_f32("dither").view(np.uint8))
    out = solve.run(we, matrix=M)
    ref = oracle.run_workload(A, we)
    e = out["exp2"][:, 0]
    err = parity.rel_err_series(out["det"][:, 0, 0], e, ref["det"][:, 0], ref["det_exp"][:, 0])
    assert err <= 1e-5, err
    # the same photons on the original medium, delayed by the gap
    top = W.face_escape_detector(base.medium, "top")
    end = top.vox[:, :2] + gap * top.dirs[:, :2]
    top.F = (((end >= 0) & (end < base.medium.nx)).all(axis=1)).astype(np.float64)
    wo = W.Workload("orig", base.medium, base.sources, [top], T, n_ref=base.n_ref)
    orig = solve.run(wo)
    se = np.ldexp(out["det"][:, 0, 0], e)
    so = np.ldexp(orig["det"][:, 0, 0], orig["exp2"][:, 0])
    keep = so[:T - gap] > 1e-30 * so.max()
    assert np.all(se[:gap] == 0)
    assert np.allclose(se[gap:][keep], so[:T - gap][keep], rtol=2e-5, atol=0)
    out["solver"].close()
    orig["solver"].close()
