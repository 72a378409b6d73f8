"""MI355X-native hot path of the Dynamic Radiative Transfer System.

J(t + dt) = A J(t) + B P(t) on gfx950: device assembly of the sparse system
matrix, a CSR SpMV / SpMM time step with fused rescale, source injection and
FP64 detector reduction, a matrix-free form of the same step built from the
per-material direction blocks, uneven persistent batches (CSR or
matrix-free members), autotuners and a continuous-batching server.  The
public ABI is include/drts.h; ``drts`` is its Python binding.
"""
from . import sources  # noqa: F401

__all__ = ["drts", "sources", "solve"]


def __getattr__(name):
    if name in ("drts", "solve"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
