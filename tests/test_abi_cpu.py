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
