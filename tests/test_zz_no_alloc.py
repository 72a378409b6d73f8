"""drts_step_noalloc (the step whose scratch memory is the library's fixed
device array) against drts_step (the same step with the solver's own
buffers): states, exponents and every series entry equal bit for bit, over
two media in a row, the second smaller than the first (what the first call
left in the shared array must not reach the second)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import solve  # noqa: E402

CASES = [
    ("csr", {}),
    ("csr_queue", {"queue": 1}),
    ("matrix_free_f64sum", {"kernel": 2}),
]


def _pair(wl, opts, n_steps):
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    tab = solve.source_table(A, wl)
    ref = drts.Solver(A, wl.n_rhs, wl.detectors, max_steps=n_steps)
    new = drts.Solver(A, wl.n_rhs, wl.detectors, max_steps=n_steps)
    if opts:
        ref.set_options(**opts)
        new.set_options(**opts)
    new.run(tab, 0)                    # stages the table (no step)
    for _ in range(n_steps):
        ref.step(tab)
        new.step_noalloc(tab)
    return ref, new


def _assert_same(ref, new, n_steps):
    a, b = ref.readout(0, n_steps), new.readout(0, n_steps)
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    xa, ea, ta = ref.state()
    xb, eb, tb = new.state()
    assert ta == tb == n_steps
    assert np.array_equal(ea, eb)
    assert np.array_equal(xa.view(np.uint8), xb.view(np.uint8))


@pytest.mark.parametrize("name,opts", CASES, ids=[c[0] for c in CASES])
def test_noalloc_step_equals_step_twice(name, opts):
    for n, steps in ((22, 25), (11, 18)):
        print("no-alloc step: %s, %d^3 layers, %d steps" % (name, n, steps), flush=True)
        wl = W.c2(n=n, n_steps=steps)
        ref, new = _pair(wl, opts, steps)
        _assert_same(ref, new, steps)


def test_noalloc_step_many_rhs():
    """Two right-hand sides (SpMM kernel): same bar."""
    wl = W.c3(n=14, k=2, n_steps=20)
    print("no-alloc step: 14^3 slab, 2 rhs, 20 steps", flush=True)
    ref, new = _pair(wl, {}, 20)
    _assert_same(ref, new, 20)


def test_noalloc_step_refuses_unstaged_table_and_oversize():
    wl = W.c2(n=10, n_steps=5)
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    S = drts.Solver(A, 1, wl.detectors, max_steps=5)
    tab = solve.source_table(A, wl)
    with pytest.raises(drts.DrtsError) as e:
        S.step_noalloc(tab)            # not staged yet
    assert e.value.rc == -5
    # 256 detectors over 64-row tiles, one tile per chunk: the partials need
    # 260 x (chunks + 256) doubles, beyond the 16 MiB array
    med = W.homogeneous(30, W.Material(10.0, 0.01, 0.9, 1.4))
    B = drts.Matrix(med, "f32", "dither", 1.4)
    dets = [W.Detector(np.array([[i % 30, (i // 30) % 30, 0]]), np.array([[0, 0, 1]]), np.array([False]),
                       np.array([1.0])) for i in range(256)]
    T = drts.Solver(B, 1, dets, max_steps=2)
    T.set_options(rows_per_tile=64, tiles_per_chunk=1)
    T.run(None, 0)
    with pytest.raises(drts.DrtsError) as e:
        T.step_noalloc(None)
    assert e.value.rc == -4
    T.step(None)                       # the allocating step still runs
