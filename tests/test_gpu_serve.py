"""The serving loop on the GPU: continuous batching of independent solves
(sphere-inclusion media with Fresnel interfaces, edges 10..16, through the
C ABI).

Bars:
  - every served result (detector series, exponents, totals) equals the same
    solve run alone with drts_run, bit for bit: the batched launch performs
    the same per-row operations and the same per-chunk FP64 partial sums;
  - served results against the FP64 oracle: relative error <= 1e-5;
  - admission keeps the admitted footprint within the budget: with a budget
    of about three requests, several requests run at once and the rest wait
    until earlier ones retire;
  - requests served with the matrix-free step (FP64 row sums) equal the same
    solves run alone with the server's options, bit for bit, and meet the
    same 1e-5 bar against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu

drts = pytest.importorskip("paper_1611_08536_amd.drts")
from paper_1611_08536_amd import serve  # noqa: E402


def _requests(n, steps=(30, 120)):
    return W.c5(n_req=n, rate=1e6, edge=(10, 16), steps=steps)


def _footprints(reqs):
    return [drts.Server.footprint(q.workload.medium, serve._table(q.workload), q.workload.detectors,
                                  q.workload.n_steps) for q in reqs]


def _same(a, b):
    return (np.array_equal(a["exp2"], b["exp2"]) and np.array_equal(a["tot"], b["tot"])
            and np.array_equal(a["det"], b["det"]))


@pytest.mark.parametrize("policy", ["arrival", "shortest"])
def test_served_results_equal_solo_runs(policy):
    reqs = _requests(8)
    fps = sorted(_footprints(reqs))
    budget = sum(fps[-3:])
    out = serve.serve(reqs, budget, quantum=16, max_active=6, max_skips=2, policy=policy, keep_results=True)
    assert 2 <= out["peak_active"] < len(reqs), out["peak_active"]
    solo = serve.fifo_plain(reqs, keep_results=True)
    for i in range(len(reqs)):
        assert _same(out["results"][i], solo["results"][i]), i


def test_strict_fifo_and_single_slot_give_the_same_results():
    reqs = _requests(5, steps=(20, 60))
    for q in reqs:
        q.arrival_s = 0.0          # all submitted before the first tick
    # submissions on the ticking thread: all five are queued before the first tick
    a = serve.serve(reqs, 1 << 34, quantum=7, max_active=1, max_skips=0, keep_results=True, submit_threads=0)
    b = serve.serve(reqs, 1 << 34, quantum=64, max_active=64, max_skips=0, keep_results=True, submit_threads=0)
    assert a["peak_active"] == 1 and b["peak_active"] == len(reqs)
    for i in range(len(reqs)):
        assert _same(a["results"][i], b["results"][i]), i


@pytest.mark.skip(reason="large CSR requests keep the shared tiled launch: a replay of the full 256-request "
                         "stream with them on their own grouped steps ended in a host segmentation fault after "
                         "70 requests, cause not found, so that path is switched off in the server")
def test_large_request_keeps_the_grouped_step():
    """A request of at least BATCH_OWN_ROWS rows (a 40^3 sphere medium) served
    beside small ones keeps its step by row groups, its groups built and
    counted at admission (its footprint bound covers them): every result
    equals the solo run with the server's options, bit for bit, and the large
    one is within 1e-5 of the oracle."""
    big = W.c5(n_req=1, rate=1e6, edge=(40, 40), steps=(40, 40))
    reqs = big + _requests(3, steps=(20, 50))
    for q in reqs:
        q.arrival_s = 0.0
    fps = _footprints(reqs)
    out = serve.serve(reqs, 2 * sum(fps), quantum=16, max_active=4, keep_results=True, submit_threads=0)
    assert out["peak_active"] == len(reqs), out["peak_active"]
    solo = serve.fifo_plain(reqs, keep_results=True)
    for i in range(len(reqs)):
        assert _same(out["results"][i], solo["results"][i]), i
    wl = reqs[0].workload
    A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
    assert A.n_rows >= drts.BATCH_OWN_ROWS
    S = drts.Solver(A, 1, wl.detectors, max_steps=1)
    S.run(serve._table(wl), 1)                # builds the groups, as admission does
    assert A.groups() is not None
    assert A.device_bytes() <= fps[0], (A.device_bytes(), fps[0])
    S.close()
    A.close()
    ref = oracle.run_workload(oracle.Matrix(wl.medium), wl)
    r = out["results"][0]
    for c in range(3):
        err = parity.rel_err_series(r["tot"][:, c], r["exp2"], ref["tot"][:, c], ref["tot_exp"][:, c])
        assert err <= 1e-5, (c, err)


def test_served_results_against_oracle():
    reqs = _requests(4)
    out = serve.serve(reqs, 1 << 34, quantum=25, keep_results=True)
    for i in (0, 3):
        wl = reqs[i].workload
        ref = oracle.run_workload(oracle.Matrix(wl.medium), wl)
        r = out["results"][i]
        for c in range(3):
            err = parity.rel_err_series(r["tot"][:, c], r["exp2"], ref["tot"][:, c], ref["tot_exp"][:, c])
            assert err <= 1e-5, (i, c, err)
        err = parity.rel_err_series(r["det"][:, 0], r["exp2"], ref["det"][:, 0], ref["det_exp"][:, 0])
        assert err <= 1e-5, (i, "det", err)


@pytest.mark.parametrize("k", [1, 2], ids=["exact_dithered_solo", "f64sum_batched"])
def test_matrix_free_served_results_equal_solo_runs_and_oracle(k):
    """Dithered values with the exact matrix-free step (the gather kernel)
    run request by request; FP64 row sums run as one matrix-free batch."""
    reqs = _requests(6)
    fps = sorted(_footprints(reqs))
    out = serve.serve(reqs, sum(fps[-3:]), quantum=16, max_active=4, max_skips=2, policy="shortest",
                      keep_results=True, kernel=k)
    assert 2 <= out["peak_active"] < len(reqs), out["peak_active"]
    solo = serve.fifo_plain(reqs, keep_results=True, kernel=k)
    for i in range(len(reqs)):
        assert _same(out["results"][i], solo["results"][i]), i
    for i in (0, 5):
        wl = reqs[i].workload
        ref = oracle.run_workload(oracle.Matrix(wl.medium), wl)
        r = out["results"][i]
        for c in range(3):
            err = parity.rel_err_series(r["tot"][:, c], r["exp2"], ref["tot"][:, c], ref["tot_exp"][:, c])
            assert err <= 1e-5, (i, c, err)
        err = parity.rel_err_series(r["det"][:, 0], r["exp2"], ref["det"][:, 0], ref["det_exp"][:, 0])
        assert err <= 1e-5, (i, "det", err)


def test_server_rejects_unknown_step():
    with pytest.raises(drts.DrtsError):
        drts.Server(1 << 30, kernel=7)

