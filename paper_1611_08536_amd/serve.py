"""Request replay over the library's serving loop (drts_serve_*).

`serve` replays a list of timed requests (workloads.Request: arrival time and
workload) against one drts.Server: every request is submitted once the wall
clock passes its arrival time, by a small pool of submitting threads (a
submission builds the request's host model, which the library does outside
the server's lock), while the main thread ticks (admit, one quantum of
batched steps, retire) until all have finished.  `fifo_plain` is the
comparison: the same requests solved one after another in arrival order, each
alone with drts_run.  Both report per-request latency (completion - arrival)
and the solves per second of the whole replay.
"""
from __future__ import annotations

import concurrent.futures as cf
import time
from typing import List, Optional

import numpy as np

from . import drts, sources


def _table(wl) -> "drts.SourceTable":
    return drts.SourceTable(wl.medium, wl.sources, sources.amplitude)


def _summary(lat: List[float], wall: float, n: int) -> dict:
    a = np.asarray(lat)
    return {"requests": n, "wall_s": wall, "solves_per_s": n / wall if wall > 0 else 0.0,
            "p50_s": float(np.percentile(a, 50)), "p99_s": float(np.percentile(a, 99)),
            "mean_s": float(a.mean())}


def serve(requests, budget_bytes: int, quantum: int = 50, max_active: int = 256, max_skips: int = 8,
          policy: str = "arrival", keep_results: bool = False, log=None, submit_threads: int = 4,
          kernel: int = drts.KERNEL_CSR) -> dict:
    """Replays `requests` through one server; returns the latency summary and,
    with keep_results, every request's series in submission order.
    submit_threads = 0 submits on the calling thread (every request that has
    arrived is queued before the next tick)."""
    S = drts.Server(budget_bytes, quantum, max_active, max_skips, policy, kernel=kernel)
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
    tables, rid_of, arrival_of = {}, {}, {}
    done_at, results = {}, {}
    pending = {}   # submission future -> request index
    k = 0
    peak_active = 0
    pool = cf.ThreadPoolExecutor(max_workers=submit_threads) if submit_threads > 0 else None

    def collect():
        for fut in [f for f in pending if f.done()]:
            i = pending.pop(fut)
            rid = fut.result()   # raises the submission's error
            rid_of[rid] = i
            arrival_of[rid] = requests[i].arrival_s

    t0 = time.perf_counter()
    try:
        while len(done_at) < len(requests):
            now = time.perf_counter() - t0
            while k < len(order) and requests[order[k]].arrival_s <= now:
                i = order[k]
                wl = requests[i].workload
                tables[i] = _table(wl)   # stays valid until the request has finished
                args = (wl.medium, tables[i], wl.detectors, wl.n_steps, wl.rounding, wl.n_ref)
                if pool is None:
                    fut = cf.Future()
                    fut.set_result(S.submit(*args))
                else:
                    fut = pool.submit(S.submit, *args)
                pending[fut] = i
                k += 1
            collect()
            info = S.tick()
            peak_active = max(peak_active, info["active"] + info["finished"])   # ran during the tick
            t = time.perf_counter() - t0
            collect()
            for rid in S.poll():
                done_at[rid] = t
                if keep_results:
                    results[rid_of[rid]] = S.result(rid)
                S.release(rid)
                tables.pop(rid_of[rid], None)
            if log and info["finished"]:
                log("serve: t=%.2fs active=%d waiting=%d done=%d/%d" %
                    (t, info["active"], info["waiting"], len(done_at), len(requests)))
            if info["active"] == 0 and info["waiting"] == 0:
                # nothing on the device: wait for a submission or the next arrival
                wait = (requests[order[k]].arrival_s - (time.perf_counter() - t0)) if k < len(order) else None
                if pending:
                    cf.wait(list(pending), timeout=wait, return_when=cf.FIRST_COMPLETED)
                elif wait is not None:
                    time.sleep(max(0.0, wait))
    finally:
        if pool is not None:
            pool.shutdown(wait=True)
        S.close()
    wall = time.perf_counter() - t0
    out = _summary([done_at[r] - arrival_of[r] for r in done_at], wall, len(requests))
    out["peak_active"] = peak_active
    if keep_results:
        out["results"] = [results[i] for i in range(len(requests))]
    return out


def solo_options(kernel: int, n_rows: int = 0) -> Optional[dict]:
    """The launch options the server gives a request of n_rows rows run with
    `kernel` (the CSR server batches every request on the tiled step: its
    large requests do not keep their grouped step)."""
    if kernel == drts.KERNEL_CSR:
        return {"variant": drts.SPMV_LDS, "tiles_per_chunk": 4}
    import torch
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    return {"kernel": kernel, "tiles_per_chunk": 8, "grid": 16 * cus}


def fifo_plain(requests, keep_results: bool = False, log=None, kernel: int = drts.KERNEL_CSR) -> dict:
    """The same requests, one at a time in arrival order, each solved alone
    (with the options the server gives a request run with `kernel`)."""
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
    lat, results = [], {}
    t0 = time.perf_counter()
    for n, i in enumerate(order):
        req = requests[i]
        wait = req.arrival_s - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        wl = req.workload
        A = drts.Matrix(wl.medium, wl.value_type, wl.rounding, wl.n_ref)
        Sv = drts.Solver(A, 1, wl.detectors, max_steps=wl.n_steps)
        opts = solo_options(kernel, A.n_rows)
        if opts:
            Sv.set_options(**opts)
        Sv.run(_table(wl), wl.n_steps)
        r = Sv.readout(0, wl.n_steps)       # synchronizes
        lat.append(time.perf_counter() - t0 - req.arrival_s)
        if keep_results:
            results[i] = {"det": r["det"][:, :, 0], "exp2": r["exp2"][:, 0], "tot": r["tot"][:, :, 0]}
        Sv.close()
        A.close()
        if log:
            log("fifo: %d/%d done" % (n + 1, len(order)))
    wall = time.perf_counter() - t0
    out = _summary(lat, wall, len(requests))
    if keep_results:
        out["results"] = [results[i] for i in range(len(requests))]
    return out


def footprint_budget(fraction: float = 0.8, device: Optional[int] = None) -> int:
    """A budget of `fraction` of the device memory torch reports free."""
    import torch
    free, _ = torch.cuda.mem_get_info(device)
    return int(free * fraction)
