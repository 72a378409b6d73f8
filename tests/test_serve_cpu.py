"""Host logic of the serving loop (drts_serve_*) without a GPU: argument
checks, the footprint bound against the oracle's exact matrix size, the
budget check at submission, and the request states.  No call here reaches
the device: submission only builds the host model of the medium."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import sources  # noqa: E402

lib = drts._lib


def _server(budget, quantum=10, max_active=4, max_skips=2, policy=0):
    h = C.c_void_p()
    assert lib.drts_serve_create(None, budget, quantum, max_active, max_skips, policy, C.byref(h)) == 0
    return h


def _submit(h, wl, n_steps=None, value_type="f32"):
    m, keep = drts._medium_struct(wl.medium, value_type, wl.rounding, wl.n_ref)
    dt, arrs = drts._detectors_struct(wl.medium, wl.detectors)
    tab = drts.SourceTable(wl.medium, wl.sources, sources.amplitude)
    rid = C.c_int64()
    rc = lib.drts_serve_submit(h, C.byref(m), C.byref(tab.c), C.byref(dt) if dt is not None else None,
                               n_steps or wl.n_steps, C.byref(rid))
    return rc, rid.value, tab


def _footprint(wl, n_steps=None):
    m, keep = drts._medium_struct(wl.medium, "f32", wl.rounding, wl.n_ref)
    dt, arrs = drts._detectors_struct(wl.medium, wl.detectors)
    tab = drts.SourceTable(wl.medium, wl.sources, sources.amplitude)
    b = C.c_int64()
    assert lib.drts_serve_footprint(C.byref(m), C.byref(tab.c), C.byref(dt) if dt is not None else None,
                                    n_steps or wl.n_steps, C.byref(b)) == 0
    return b.value


def test_create_rejects_bad_arguments():
    h = C.c_void_p()
    assert lib.drts_serve_create(None, 0, 10, 4, 0, 0, C.byref(h)) == -1
    assert lib.drts_serve_create(None, 1 << 30, 0, 4, 0, 0, C.byref(h)) == -1
    assert lib.drts_serve_create(None, 1 << 30, 10, 0, 0, 0, C.byref(h)) == -1
    assert lib.drts_serve_create(None, 1 << 30, 10, 4, -1, 0, C.byref(h)) == -1
    assert lib.drts_serve_create(None, 1 << 30, 10, 4, 0, 2, C.byref(h)) == -1
    assert lib.drts_serve_create(None, 1 << 30, 10, 4, 0, 0, None) == -1


@pytest.mark.parametrize("edge", [(10, 10), (14, 14)])
def test_footprint_bounds_the_exact_matrix(edge):
    """The bound covers the exact [A; L] (oracle nnz and rows), two FP32 state
    buffers and the series, and is not far above them."""
    req = W.c5(n_req=2, edge=edge, steps=(80, 80))
    for q in req:
        wl = q.workload
        A = oracle.Matrix(wl.medium)
        exact = 8 * A.nnz + 4 * (A.n_rows + 1) + 2 * 4 * A.n_rows + wl.n_steps * 8 * (3 + len(wl.detectors))
        fp = _footprint(wl)
        assert fp >= exact
        assert fp <= 2 * exact + (8 << 20)


def test_submit_checks_budget_and_precision():
    wl = W.c5(n_req=1, edge=(12, 12), steps=(40, 40))[0].workload
    fp = _footprint(wl)
    h = _server(fp - 1)
    rc, rid, _ = _submit(h, wl)
    assert rc == -2 and b"budget" in lib.drts_last_error()
    lib.drts_serve_destroy(h)
    h = _server(fp)
    assert _submit(h, wl, value_type="f64")[0] == -1
    rc, rid, tab = _submit(h, wl)
    assert rc == 0 and rid >= 1
    # queued, not finished: no result yet, cannot be released
    ser = np.zeros(40)
    assert lib.drts_serve_result(h, rid, None, None, ser.ctypes.data) == -5
    assert lib.drts_serve_release(h, rid) == -5
    assert lib.drts_serve_result(h, rid + 100, None, None, None) == -1
    ids = (C.c_int64 * 4)()
    n = C.c_int32()
    assert lib.drts_serve_poll(h, ids, 4, C.byref(n)) == 0 and n.value == 0
    lib.drts_serve_destroy(h)


def test_tick_on_an_empty_server_does_nothing():
    h = _server(1 << 30)
    a, w, f, b = C.c_int32(-1), C.c_int32(-1), C.c_int32(-1), C.c_int64(-1)
    assert lib.drts_serve_tick(h, C.byref(a), C.byref(w), C.byref(f), C.byref(b)) == 0
    assert (a.value, w.value, f.value, b.value) == (0, 0, 0, 0)
    lib.drts_serve_destroy(h)


def test_concurrent_submissions_queue_every_request_once():
    """Submissions from several threads at once (each builds its host model
    outside the server's lock): every call gets its own id, ids are the
    consecutive range of the calls, every request is queued (known and not
    finished), and a failing submission on one thread does not disturb the
    others."""
    import threading
    reqs = W.c5(n_req=8, edge=(10, 16), steps=(20, 40))
    h = _server(1 << 34)
    out, errs = {}, []
    keep = []
    barrier = threading.Barrier(len(reqs) + 1)

    def work(i):
        barrier.wait()
        rc, rid, tab = _submit(h, reqs[i].workload)
        keep.append(tab)
        out[i] = (rc, rid)

    def bad():
        barrier.wait()
        errs.append(_submit(h, reqs[0].workload, value_type="f64")[0])

    ts = [threading.Thread(target=work, args=(i,)) for i in range(len(reqs))] + [threading.Thread(target=bad)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert errs == [-1]
    assert all(rc == 0 for rc, _ in out.values())
    ids = sorted(rid for _, rid in out.values())
    assert ids == list(range(1, len(reqs) + 1))   # the FP64 medium is refused before it takes an id
    for rid in ids:
        assert lib.drts_serve_result(h, rid, None, None, None) == -5   # queued, not finished
    n = C.c_int32()
    pid = (C.c_int64 * 16)()
    assert lib.drts_serve_poll(h, pid, 16, C.byref(n)) == 0 and n.value == 0
    lib.drts_serve_destroy(h)
