"""Source pulse shapes for the DRTS source table (Sec. 4.1, Eq. (26)).

The number of photons a source emits during step t is the integral of its
time profile over [t dt, (t+1) dt): the step-integrated source the paper asks
for when the source varies faster than a step.
"""
from __future__ import annotations

import math


def impulse_step(t: int) -> float:
    """All photons at the first step."""
    return 1.0 if t == 0 else 0.0


def gaussian_step(fwhm_s: float, dt_s: float, t: int) -> float:
    """Normalised Gaussian pulse (FWHM fwhm_s, peak at 3 sigma) integrated over
    step t; the first step also takes everything before t = 0, so the steps sum
    to one.  Written with erfc to avoid cancellation in the tails."""
    sigma = fwhm_s / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    peak = 3.0 * sigma
    scale = sigma * math.sqrt(2.0)
    upper = math.erfc(((t + 1) * dt_s - peak) / scale)
    lower = 2.0 if t == 0 else math.erfc((t * dt_s - peak) / scale)
    return 0.5 * (lower - upper)


def amplitude(source, t: int, dt_s: float) -> float:
    """Photons emitted during step t by a workloads.Source."""
    if source.kind == "impulse":
        return impulse_step(t)
    if source.kind == "gaussian":
        return gaussian_step(source.fwhm_fs * 1e-15, dt_s, t)
    raise ValueError("unknown source kind %r" % source.kind)
