"""The C-ABI library builds for gfx950, loads, and exports every function that
include/drts.h declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drts.h")
LIB = os.path.join(ROOT, "paper_1611_08536_amd", "libdrts.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(drts_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_t")))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (the library binds to torch's HIP runtime)
    if not os.path.exists(LIB):
        from paper_1611_08536_amd import _build
        _build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("drts_build_matrix", "drts_step", "drts_run", "drts_detector_readout"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for name in declared_functions():
        assert name in exported, name
        getattr(lib, name)


def test_binding_lists_every_symbol(lib):
    from paper_1611_08536_amd import drts
    assert sorted(drts.EXPORTED) == declared_functions()


def test_library_is_built_for_gfx950():
    """The offload bundle of the library names the gfx950 target."""
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_last_error_is_empty_string_initially(lib):
    """In a fresh process no call has failed yet (other tests here set it)."""
    code = ("import torch, ctypes; l = ctypes.CDLL(%r); l.drts_last_error.restype = ctypes.c_char_p; "
            "print(repr(l.drts_last_error()))" % LIB)
    out = subprocess.check_output(["python", "-c", code], text=True, cwd=ROOT)
    assert out.strip() == "b''"


def test_invalid_arguments_fail_without_a_gpu(lib):
    """Argument checks happen before any HIP call."""
    from paper_1611_08536_amd import drts
    h = ctypes.c_void_p()
    assert lib.drts_build_matrix(None, None, ctypes.byref(h)) == -1
    assert b"NULL" in drts._lib.drts_last_error()
    assert drts._lib.drts_solver_create(None, 1, None, 10, None, ctypes.byref(h)) == -1
    assert drts._lib.drts_step(None, None) == -1
    assert drts._lib.drts_matrix_row_of(None, 0, 0) == -1


def test_one_hip_runtime_is_mapped(lib):
    """torch's HIP runtime and the library's are the same mapped file."""
    from paper_1611_08536_amd import drts
    assert len(drts._hip_runtimes()) == 1


def test_pulse_steps_integrate_the_profile(lib):
    """drts_pulse_step (host function, no GPU): the Gaussian's steps sum to one
    and each equals the density integrated over its step (numerical
    quadrature); the impulse is one photon in step 0; bad arguments give NaN."""
    import math
    from scipy.integrate import quad
    from paper_1611_08536_amd import drts
    for fwhm, dt in ((100e-15, 467e-15), (1e-12, 0.3e-12), (50e-15, 10e-15)):
        sig = fwhm / (2 * math.sqrt(2 * math.log(2)))
        dens = lambda t: math.exp(-0.5 * ((t - 3 * sig) / sig) ** 2) / (sig * math.sqrt(2 * math.pi))
        steps = [drts.pulse_step(drts.PULSE_GAUSSIAN, fwhm, t, dt) for t in range(int(12 * sig / dt) + 3)]
        assert sum(steps) == pytest.approx(1.0, abs=1e-14)
        for t in range(1, min(len(steps), 8)):
            assert steps[t] == pytest.approx(quad(dens, t * dt, (t + 1) * dt, epsabs=1e-15, epsrel=1e-13)[0],
                                             abs=1e-13)
        assert steps[0] == pytest.approx(quad(dens, -50 * sig, dt, epsabs=1e-15, epsrel=1e-13, limit=200)[0],
                                         abs=1e-13)
    assert [drts.pulse_step(drts.PULSE_IMPULSE, 0.0, t, 1e-15) for t in range(3)] == [1.0, 0.0, 0.0]
    f = drts._lib.drts_pulse_step
    for kind, fwhm, step, dt in ((7, 1e-13, 0, 1e-15), (drts.PULSE_GAUSSIAN, 0.0, 0, 1e-15),
                                 (drts.PULSE_GAUSSIAN, 1e-13, -1, 1e-15), (drts.PULSE_IMPULSE, 0.0, 0, 0.0)):
        assert math.isnan(f(ctypes.byref(drts.PulseT(kind, fwhm)), step, dt))
    assert math.isnan(f(None, 0, 1e-15))
