"""Source pulse shapes for the DRTS source table (Sec. 4.1, Eq. (26)).

The number of photons a source emits during step t is the integral of its
time profile over [t dt, (t+1) dt): the step-integrated source the paper asks
for when the source varies faster than a step.  The profiles are the
library's (drts_pulse_step in include/drts.h), so C callers and this binding
use one definition.
"""
from __future__ import annotations


def _drts():
    from . import drts
    return drts


def impulse_step(t: int) -> float:
    """All photons at the first step."""
    d = _drts()
    return d.pulse_step(d.PULSE_IMPULSE, 0.0, t, 1.0)


def gaussian_step(fwhm_s: float, dt_s: float, t: int) -> float:
    """Normalised Gaussian pulse (FWHM fwhm_s, peak at 3 sigma) integrated over
    step t; the first step also takes everything before t = 0, so the steps sum
    to one."""
    d = _drts()
    return d.pulse_step(d.PULSE_GAUSSIAN, fwhm_s, t, dt_s)


def amplitude(source, t: int, dt_s: float) -> float:
    """Photons emitted during step t by a workloads.Source."""
    if source.kind == "impulse":
        return impulse_step(t)
    if source.kind == "gaussian":
        return gaussian_step(source.fwhm_fs * 1e-15, dt_s, t)
    raise ValueError("unknown source kind %r" % source.kind)
