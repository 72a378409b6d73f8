"""Runs a workload (workloads.Workload) through the DRTS library.

Builds [A; L] on the device, creates the solver with the workload's
detectors, feeds its sources and returns the FP64 series (value, exponent)
and the final state.  Every step runs in the library's kernels.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import drts, sources


def source_table(matrix: "drts.Matrix", workload) -> "drts.SourceTable":
    return drts.SourceTable(matrix.medium, workload.sources, sources.amplitude)


def run(workload, n_steps: Optional[int] = None, options: Optional[dict] = None, matrix=None,
        use_run: bool = True, want_state: bool = True) -> dict:
    n = workload.n_steps if n_steps is None else n_steps
    A = matrix or drts.Matrix(workload.medium, workload.value_type, workload.rounding, workload.n_ref)
    S = drts.Solver(A, workload.n_rhs, workload.detectors, max_steps=max(n, 1))
    if options:
        S.set_options(**options)
    tab = source_table(A, workload)
    if use_run:
        S.run(tab, n)
    else:
        for _ in range(n):
            S.step(tab)
    out = S.readout(0, n)
    out["matrix"] = A
    out["solver"] = S
    if want_state:
        x, e, t = S.state()
        out["x"], out["x_exp"], out["t"] = x, e, t
    return out


def physical(value, exp2) -> np.ndarray:
    """value * 2^exp2 (may underflow to 0 in FP64 for very long runs)."""
    return np.ldexp(np.asarray(value, dtype=np.float64), np.asarray(exp2))
