"""ctypes binding of libdrts.so (the C ABI in include/drts.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory (its caching allocator, through
the drts_device_t hooks) and the stream (torch's current stream).  The module
raises ImportError when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdrts.so")

F64, F32 = 0, 1
ROUND_NEAREST, ROUND_DITHER = 0, 1
GEOM = {"voxels": 0, "homog": 0, "layers_z": 1, "sphere": 2}
DIRECTIONS = {"lattice26": 0, "lebedev86": 1}
INTERFACE = {"origin": 0, "substep": 1}
BC = {"vacuum": 0, "reflect": 1}
KERNEL_CSR, KERNEL_STRUCTURED, KERNEL_STRUCTURED_F64SUM = 0, 1, 2
SPMM_GROUPED, SPMM_ROWS, SPMM_GROUPED_F64SUM = 0, 1, 2   # variant of a many-rhs CSR solver
SPMV_ROW, SPMV_LDS, SPMV_GROUPED = 0, 1, 2   # variants of a single-rhs CSR solver
BATCH_OWN_ROWS = 512 * 1024   # a CSR batch member this large keeps its own grouped step
SERVE_ARRIVAL, SERVE_SHORTEST = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError("libdrts.so is not built (run paper_1611_08536_amd._build.build())")

# torch's HIP runtime must be the one libdrts.so binds to: torch ships it as
# libamdhip64.so with the soname libamdhip64.so.7, so once torch is loaded the
# library's dependency resolves to that same copy.  Loading libdrts.so first
# would map a second HIP runtime from /opt/rocm, and torch's streams, events
# and allocations would then belong to a different runtime than the kernels.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)


def _hip_runtimes():
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            p = line.split()[-1] if line.strip() else ""
            if "libamdhip64" in p:
                paths.add(os.path.realpath(p))
    return sorted(paths)


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped (%s); import torch before loading libdrts.so"
                      % ", ".join(_hip_runtimes()))

P = C.c_void_p
i32, i64, dbl = C.c_int32, C.c_int64, C.c_double


class Grid(C.Structure):
    _fields_ = [("nx", i32), ("ny", i32), ("nz", i32), ("h_mm", dbl)]


class MaterialT(C.Structure):
    _fields_ = [("mu_s", dbl), ("mu_a", dbl), ("g", dbl), ("n", dbl)]


class Geometry(C.Structure):
    _fields_ = [("kind", i32), ("sphere_c", dbl * 3), ("sphere_r", dbl), ("n_layers", i32),
                ("layer_z0", C.POINTER(i32))]


class MediumT(C.Structure):
    _fields_ = [("grid", Grid), ("n_mat", i32), ("mat", C.POINTER(MaterialT)),
                ("mat_of_voxel", C.POINTER(C.c_uint8)), ("geom", Geometry), ("bc", i32),
                ("value_type", i32), ("rounding", i32), ("n_ref", dbl), ("scatter_order", i32),
                ("directions", i32), ("c_dt", dbl), ("interface_model", i32)]


ALLOC_FN = C.CFUNCTYPE(P, P, C.c_size_t, P)
FREE_FN = C.CFUNCTYPE(None, P, P, P)


class DeviceT(C.Structure):
    _fields_ = [("ctx", P), ("alloc", ALLOC_FN), ("free", FREE_FN), ("stream", P)]


SUPPORT_FN = C.CFUNCTYPE(i64, P, i32, C.POINTER(i64), C.POINTER(dbl), i64)
AMP_FN = C.CFUNCTYPE(dbl, P, i32, i64, dbl, dbl)
RHS_FN = C.CFUNCTYPE(i32, P, i32)


class SourceTableT(C.Structure):
    _fields_ = [("ctx", P), ("n_src", i32), ("support", SUPPORT_FN), ("amplitude", AMP_FN),
                ("rhs_of", RHS_FN)]


PULSE_IMPULSE, PULSE_GAUSSIAN = 0, 1


class PulseT(C.Structure):
    _fields_ = [("kind", i32), ("fwhm_s", dbl)]


class GroupsInfoT(C.Structure):
    _fields_ = [("n_groups", i64), ("n_fast", i64), ("n_vox2_rows", i64), ("n_list_rows", i64),
                ("n_list_entries", i64), ("value_tables", i64)]


class DetectorsT(C.Structure):
    _fields_ = [("n_det", i32), ("det_ptr", C.POINTER(i64)), ("state", C.POINTER(i64)),
                ("escape", C.POINTER(C.c_uint8)), ("F", C.POINTER(dbl))]


class OptionsT(C.Structure):
    _fields_ = [("kernel", i32), ("rows_per_tile", i32), ("tiles_per_chunk", i32), ("grid", i32),
                ("xcd_remap", i32), ("graph_steps", i32), ("rescale", i32), ("variant", i32), ("queue", i32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("drts_last_error", C.c_char_p, [])
_sig("drts_build_matrix", C.c_int, [C.POINTER(MediumT), C.POINTER(DeviceT), C.POINTER(P)])
_sig("drts_direction_set", C.c_int, [i32, P, P])
_sig("drts_matrix_info", C.c_int, [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                   C.POINTER(dbl)])
_sig("drts_matrix_row_of", i64, [P, i64, i32])
_sig("drts_pulse_step", dbl, [C.POINTER(PulseT), i64, dbl])
_sig("drts_matrix_groups", C.c_int, [P, C.POINTER(GroupsInfoT)])
_sig("drts_matrix_export_rows", C.c_int, [P, i64, i64, P, P, P])
_sig("drts_matrix_destroy", None, [P])
_sig("drts_solver_create", C.c_int, [P, i32, C.POINTER(DetectorsT), i64, C.POINTER(DeviceT), C.POINTER(P)])
_sig("drts_solver_get_options", C.c_int, [P, C.POINTER(OptionsT)])
_sig("drts_solver_set_options", C.c_int, [P, C.POINTER(OptionsT)])
_sig("drts_step", C.c_int, [P, C.POINTER(SourceTableT)])
_sig("drts_step_noalloc", C.c_int, [P, C.POINTER(SourceTableT)])
_sig("drts_run", C.c_int, [P, C.POINTER(SourceTableT), i64])
_sig("drts_solver_time", C.c_int, [P, C.POINTER(i64)])
_sig("drts_detector_readout", C.c_int, [P, i64, i64, P, P, P])
_sig("drts_detector_window", C.c_int, [P, P, i32, i32, i64, i64, P, P])
_sig("drts_state_read", C.c_int, [P, P, P, C.POINTER(i64)])
_sig("drts_state_write", C.c_int, [P, P, P, i64])
_sig("drts_solver_profile", C.c_int, [P, i32])
_sig("drts_solver_profile_stats", C.c_int, [P, C.POINTER(i64), C.POINTER(dbl)])
_sig("drts_solver_destroy", None, [P])
_sig("drts_batch_create", C.c_int, [C.POINTER(P), i32, C.POINTER(DeviceT), C.POINTER(P)])
_sig("drts_batch_run", C.c_int, [P, C.POINTER(C.POINTER(SourceTableT)), C.POINTER(i64)])
_sig("drts_batch_destroy", None, [P])
_sig("drts_batch_autotune", C.c_int, [P, C.POINTER(OptionsT)])
_sig("drts_autotune", C.c_int, [P, C.c_char_p, C.POINTER(OptionsT)])
_sig("drts_serve_create", C.c_int, [C.POINTER(DeviceT), i64, i32, i32, i32, i32, C.POINTER(P)])
_sig("drts_serve_submit", C.c_int, [P, C.POINTER(MediumT), C.POINTER(SourceTableT), C.POINTER(DetectorsT), i64,
                                    C.POINTER(i64)])
_sig("drts_serve_footprint", C.c_int, [C.POINTER(MediumT), C.POINTER(SourceTableT), C.POINTER(DetectorsT), i64,
                                       C.POINTER(i64)])
_sig("drts_serve_tick", C.c_int, [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)])
_sig("drts_serve_poll", C.c_int, [P, C.POINTER(i64), i32, C.POINTER(i32)])
_sig("drts_serve_result", C.c_int, [P, i64, P, P, P])
_sig("drts_serve_release", C.c_int, [P, i64])
_sig("drts_serve_destroy", None, [P])
_sig("drts_serve_set_step", C.c_int, [P, i32])

EXPORTED = [
    "drts_direction_set", "drts_pulse_step", "drts_build_matrix", "drts_matrix_info", "drts_matrix_groups", "drts_matrix_row_of", "drts_matrix_export_rows",
    "drts_matrix_destroy", "drts_solver_create", "drts_solver_get_options", "drts_solver_set_options",
    "drts_step", "drts_step_noalloc", "drts_run", "drts_solver_time", "drts_detector_readout", "drts_detector_window", "drts_state_read",
    "drts_state_write", "drts_solver_profile", "drts_solver_profile_stats", "drts_solver_destroy",
    "drts_batch_create", "drts_batch_run", "drts_batch_destroy", "drts_batch_autotune", "drts_autotune", "drts_last_error",
    "drts_serve_create", "drts_serve_submit", "drts_serve_footprint", "drts_serve_tick", "drts_serve_poll", "drts_serve_result",
    "drts_serve_release", "drts_serve_destroy", "drts_serve_set_step",
]


class DrtsError(RuntimeError):
    def __init__(self, rc, where):
        msg = _lib.drts_last_error().decode(errors="replace")
        super().__init__("%s failed (%d): %s" % (where, rc, msg))
        self.rc = rc


def pulse_step(kind: int, fwhm_s: float, step: int, dt_s: float) -> float:
    """Photons a pulse of unit total emits during step `step` (the library's
    drts_pulse_step: its time profile integrated over the step)."""
    v = _lib.drts_pulse_step(C.byref(PulseT(kind, fwhm_s)), step, dt_s)
    if v != v:
        raise DrtsError(-1, "drts_pulse_step")   # DRTS_E_INVALID
    return v


def _check(rc, where):
    if rc != 0:
        raise DrtsError(rc, where)


# ---- device hooks over torch ------------------------------------------------

class TorchDevice:
    """drts_device_t backed by torch's caching allocator and current stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the DRTS library needs an MI355X")
        self._torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        sp = self.stream.cuda_stream

        def _alloc(ctx, size, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), self.device, sp)
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.c = DeviceT(None, self._alloc, self._free, sp)

    def synchronize(self):
        self.stream.synchronize()


_default_device = None


def default_device() -> TorchDevice:
    global _default_device
    if _default_device is None:
        _default_device = TorchDevice()
    return _default_device


# ---- state layout of the library ---------------------------------------------

def direction_set(name: str = "lattice26"):
    """(unit [n, 3], weight [n]) of an angular partition (drts_direction_set)."""
    code = DIRECTIONS[name]
    n = _lib.drts_direction_set(code, None, None)
    unit, w = np.zeros((n, 3)), np.zeros(n)
    _check(0 if _lib.drts_direction_set(code, unit.ctypes.data, w.ctypes.data) == n else -1, "drts_direction_set")
    return unit, w


def state_index(medium, vox, dirs) -> np.ndarray:
    """State 26 v + d of voxels (x, y, z) and lattice vectors (dx, dy, dz), with
    v = x + nx (y + ny z) and d = k - (k > 13), k = 9(dz+1) + 3(dy+1) + (dx+1);
    on Lebedev media 86 v + n, n the library's direction nearest the given
    vector (largest cosine, the lowest index on ties)."""
    vox = np.asarray(vox, dtype=np.int64).reshape(-1, 3)
    if getattr(medium, "directions", "lattice26") == "lebedev86":
        unit, _ = direction_set("lebedev86")
        dv = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
        dv = dv / np.linalg.norm(dv, axis=1, keepdims=True)
        v = vox[:, 0] + medium.nx * (vox[:, 1] + medium.ny * vox[:, 2])
        return 86 * v + np.argmax(dv @ unit.T, axis=1)
    dirs = np.asarray(dirs, dtype=np.int64).reshape(-1, 3)
    k = 9 * (dirs[:, 2] + 1) + 3 * (dirs[:, 1] + 1) + (dirs[:, 0] + 1)
    d = k - (k > 13)
    v = vox[:, 0] + medium.nx * (vox[:, 1] + medium.ny * vox[:, 2])
    return 26 * v + d


# ---- matrix ---------------------------------------------------------------------

def _medium_struct(medium, value_type="f32", rounding="dither", n_ref=None, use_map=True):
    """drts_medium_t of a workloads.Medium plus the host arrays it points to."""
    mats = (MaterialT * len(medium.materials))(
        *[MaterialT(m.mu_s, m.mu_a, m.g, m.n) for m in medium.materials])
    vmap = np.ascontiguousarray(medium.mat_of_voxel, dtype=np.uint8).reshape(-1)
    z0 = np.ascontiguousarray(medium.layer_z0 or (0,), dtype=np.int32)
    geom = Geometry()
    geom.kind = GEOM[medium.geom]
    geom.sphere_c = (dbl * 3)(*(medium.sphere_c or (0.0, 0.0, 0.0)))
    geom.sphere_r = medium.sphere_r or 0.0
    geom.n_layers = len(medium.layer_z0)
    geom.layer_z0 = z0.ctypes.data_as(C.POINTER(i32))
    m = MediumT()
    m.grid = Grid(medium.nx, medium.ny, medium.nz, medium.h_mm)
    m.n_mat = len(medium.materials)
    m.mat = mats
    m.mat_of_voxel = vmap.ctypes.data_as(C.POINTER(C.c_uint8)) if use_map else None
    m.geom = geom
    m.bc = BC[medium.bc]
    m.value_type = F64 if value_type == "f64" else F32
    m.rounding = ROUND_DITHER if rounding == "dither" else ROUND_NEAREST
    m.n_ref = n_ref if n_ref is not None else medium.materials[0].n
    m.scatter_order = getattr(medium, "scatter_order", 1)
    m.directions = DIRECTIONS[getattr(medium, "directions", "lattice26")]
    m.c_dt = getattr(medium, "c_dt", 1.0)
    m.interface_model = INTERFACE[getattr(medium, "interface", "origin")]
    return m, (mats, vmap, z0)


def _detectors_struct(medium, detectors):
    """drts_detectors_t of a list of workloads.Detector (None when empty) plus its arrays."""
    if not detectors:
        return None, None
    ptr, st, esc, F = [0], [], [], []
    for d in detectors:
        s = state_index(medium, d.vox, d.dirs)
        st.append(s)
        esc.append(np.asarray(d.escape, dtype=np.uint8).reshape(-1))
        F.append(np.asarray(d.F, dtype=np.float64).reshape(-1))
        ptr.append(ptr[-1] + s.size)
    arrs = (np.asarray(ptr, dtype=np.int64), np.concatenate(st), np.concatenate(esc), np.concatenate(F))
    dt = DetectorsT(len(detectors), arrs[0].ctypes.data_as(C.POINTER(i64)), arrs[1].ctypes.data_as(C.POINTER(i64)),
                    arrs[2].ctypes.data_as(C.POINTER(C.c_uint8)), arrs[3].ctypes.data_as(C.POINTER(dbl)))
    return dt, arrs


class Matrix:
    """[A; L] of one medium, assembled on the device (drts_build_matrix)."""

    def __init__(self, medium, value_type: str = "f32", rounding: str = "dither",
                 n_ref: Optional[float] = None, device: Optional[TorchDevice] = None,
                 use_map: bool = True):
        self.device = device or default_device()
        self.medium = medium
        m, self._keep = _medium_struct(medium, value_type, rounding, n_ref, use_map)
        self.value_type = value_type
        h = P()
        _check(_lib.drts_build_matrix(C.byref(m), C.byref(self.device.c), C.byref(h)), "drts_build_matrix")
        self._h = h
        a, b, c, d = i64(), i64(), i64(), i64()
        dt = dbl()
        _check(_lib.drts_matrix_info(h, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(dt)),
               "drts_matrix_info")
        self.n_states, self.n_escape, self.nnz, self.bytes, self.dt = a.value, b.value, c.value, d.value, dt.value
        self.n_rows = self.n_states + self.n_escape

    def device_bytes(self) -> int:
        """Device bytes the matrix holds now: the CSR arrays, and the row groups
        once a solo solver has asked for the grouped step."""
        d = i64()
        _check(_lib.drts_matrix_info(self._h, None, None, None, C.byref(d), None), "drts_matrix_info")
        return d.value

    def groups(self):
        """The matrix's row groups (drts_groups_info_t as a dict: n_groups,
        n_fast, n_vox2_rows, n_list_rows, n_list_entries, value_tables), or
        None while they are not built."""
        g = GroupsInfoT()
        rc = _lib.drts_matrix_groups(self._h, C.byref(g))
        if rc == -5:
            return None
        _check(rc, "drts_matrix_groups")
        return {f: getattr(g, f) for f, _ in GroupsInfoT._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.drts_matrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def row_of(self, state: int, escape: bool) -> int:
        return _lib.drts_matrix_row_of(self._h, int(state), 1 if escape else 0)

    def export_rows(self, row0: int = 0, n_rows: Optional[int] = None):
        n_rows = self.n_rows - row0 if n_rows is None else n_rows
        rp = np.empty(n_rows + 1, dtype=np.int64)
        _check(_lib.drts_matrix_export_rows(self._h, row0, n_rows, rp.ctypes.data, None, None), "export_rows")
        n = int(rp[-1] - rp[0])
        col = np.empty(n, dtype=np.int32)
        val = np.empty(n, dtype=np.float64 if self.value_type == "f64" else np.float32)
        _check(_lib.drts_matrix_export_rows(self._h, row0, n_rows, rp.ctypes.data, col.ctypes.data,
                                            val.ctypes.data), "export_rows")
        return rp, col, val


# ---- sources --------------------------------------------------------------------

class SourceTable:
    """drts_source_table_t over a list of workloads.Source (support and pulse shape)."""

    def __init__(self, medium, sources, amplitude_fn):
        self.medium = medium
        self.sources = list(sources)
        self._support = [(state_index(medium, s.vox, s.dirs), np.asarray(s.w, dtype=np.float64))
                         for s in self.sources]
        self._amp = amplitude_fn

        def support(ctx, src, state, w, cap):
            st, ww = self._support[src]
            n = st.size
            if n <= cap:
                C.memmove(state, st.ctypes.data, n * 8)
                C.memmove(w, ww.ctypes.data, n * 8)
            return n

        def amplitude(ctx, src, step, t0, dt):
            return float(self._amp(self.sources[src], int(step), dt))

        def rhs_of(ctx, src):
            return int(self.sources[src].rhs)

        self._cb = (SUPPORT_FN(support), AMP_FN(amplitude), RHS_FN(rhs_of))
        self.c = SourceTableT(None, len(self.sources), *self._cb)


# ---- solver ---------------------------------------------------------------------

class Solver:
    """Time stepping of one matrix for n_rhs right-hand sides (drts_solver_*)."""

    def __init__(self, matrix: Matrix, n_rhs: int = 1, detectors: Sequence = (), max_steps: int = 1000,
                 device: Optional[TorchDevice] = None):
        self.A = matrix
        self.device = device or matrix.device
        self.n_rhs = n_rhs
        self.max_steps = max_steps
        self.n_det = len(detectors)
        dt, self._det = _detectors_struct(matrix.medium, detectors)
        h = P()
        _check(_lib.drts_solver_create(matrix._h, n_rhs, C.byref(dt) if dt is not None else None, max_steps,
                                       C.byref(self.device.c), C.byref(h)), "drts_solver_create")
        self._h = h
        self._tables = []

    def close(self):
        if getattr(self, "_h", None):
            _lib.drts_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def options(self) -> dict:
        o = OptionsT()
        _check(_lib.drts_solver_get_options(self._h, C.byref(o)), "get_options")
        return {k: getattr(o, k) for k, _ in OptionsT._fields_}

    def set_options(self, **kw):
        cur = self.options
        cur.update(kw)
        o = OptionsT(**cur)
        _check(_lib.drts_solver_set_options(self._h, C.byref(o)), "set_options")

    def _table(self, sources: Optional[SourceTable]):
        if sources is None:
            return None
        if sources not in self._tables:
            self._tables.append(sources)
        return C.byref(sources.c)

    def step(self, sources: Optional[SourceTable] = None):
        _check(_lib.drts_step(self._h, self._table(sources)), "drts_step")

    def step_noalloc(self, sources: Optional[SourceTable] = None):
        """drts_step_noalloc: the same step with the library's fixed scratch
        array (the table must already be staged by step() or run())."""
        _check(_lib.drts_step_noalloc(self._h, self._table(sources)), "drts_step_noalloc")

    def run(self, sources: Optional[SourceTable], n_steps: int):
        _check(_lib.drts_run(self._h, self._table(sources), int(n_steps)), "drts_run")

    def time(self) -> int:
        t = i64()
        _check(_lib.drts_solver_time(self._h, C.byref(t)), "drts_solver_time")
        return t.value

    def readout(self, first: int = 0, count: Optional[int] = None) -> dict:
        count = self.time() - first if count is None else count
        nr, nd = self.n_rhs, self.n_det
        ser = np.zeros((count, max(nd, 1), nr))
        e = np.zeros((count, nr), dtype=np.int32)
        tot = np.zeros((count, 3, nr))
        _check(_lib.drts_detector_readout(self._h, first, count, ser.ctypes.data, e.ctypes.data, tot.ctypes.data),
               "drts_detector_readout")
        return {"det": ser[:, :nd, :], "exp2": e, "tot": tot}

    def window(self, taps, tap0: int = 0, first: int = 0, count: Optional[int] = None):
        """drts_detector_window: readings of sensors with impulse responses
        taps [n_det, n_taps] (delays tap0 ..), as (value [count, n_det, n_rhs],
        exp2 [count, n_det, n_rhs])."""
        taps = np.ascontiguousarray(np.broadcast_to(np.asarray(taps, dtype=np.float64),
                                                    (self.n_det, np.asarray(taps).shape[-1])))
        count = (self.max_steps - first) if count is None else count
        out = np.zeros((count, self.n_det, self.n_rhs))
        e = np.zeros((count, self.n_det, self.n_rhs), dtype=np.int32)
        _check(_lib.drts_detector_window(self._h, taps.ctypes.data, taps.shape[1], int(tap0), int(first), int(count),
                                         out.ctypes.data, e.ctypes.data), "drts_detector_window")
        return out, e

    def state(self):
        dtype = np.float64 if self.A.value_type == "f64" else np.float32
        x = np.empty((self.A.n_rows, self.n_rhs), dtype=dtype)
        e = np.zeros(self.n_rhs, dtype=np.int32)
        t = i64()
        _check(_lib.drts_state_read(self._h, x.ctypes.data, e.ctypes.data, C.byref(t)), "drts_state_read")
        return x, e, t.value

    def set_state(self, x, exp2, t: int):
        dtype = np.float64 if self.A.value_type == "f64" else np.float32
        x = np.ascontiguousarray(x, dtype=dtype).reshape(self.A.n_rows, self.n_rhs)
        e = np.ascontiguousarray(exp2, dtype=np.int32).reshape(self.n_rhs)
        _check(_lib.drts_state_write(self._h, x.ctypes.data, e.ctypes.data, int(t)), "drts_state_write")

    def profile(self, enable: bool = True):
        _check(_lib.drts_solver_profile(self._h, 1 if enable else 0), "drts_solver_profile")

    def profile_stats(self):
        n, ms = i64(), dbl()
        _check(_lib.drts_solver_profile_stats(self._h, C.byref(n), C.byref(ms)), "profile_stats")
        return n.value, ms.value

    def autotune(self, cache_path: Optional[str] = None) -> dict:
        o = OptionsT()
        _check(_lib.drts_autotune(self._h, cache_path.encode() if cache_path else None, C.byref(o)),
               "drts_autotune")
        return {k: getattr(o, k) for k, _ in OptionsT._fields_}


class Batch:
    """Uneven batch of single-rhs FP32 solvers advanced by one launch per step
    (per kernel): all members on the CSR step (members of BATCH_OWN_ROWS rows
    or more keep their own step by row groups, the others share one tiled
    launch), or all on the matrix-free step in a direction-major mode
    (drts_batch_*)."""

    def __init__(self, solvers: List[Solver], device: Optional[TorchDevice] = None):
        self.solvers = list(solvers)
        self.device = device or solvers[0].device
        arr = (P * len(solvers))(*[s._h for s in solvers])
        h = P()
        _check(_lib.drts_batch_create(arr, len(solvers), C.byref(self.device.c), C.byref(h)), "drts_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.drts_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, tables: Sequence[Optional[SourceTable]], n_steps: Sequence[int]):
        n = len(self.solvers)
        ptrs = (C.POINTER(SourceTableT) * n)(
            *[C.pointer(t.c) if t is not None else C.POINTER(SourceTableT)() for t in tables])
        # each member solver recognises its staged sources by the table's
        # address: keep every table it has seen alive as long as the solver
        for s, t in zip(self.solvers, tables):
            if t is not None and t not in s._tables:
                s._tables.append(t)
        steps = np.ascontiguousarray(n_steps, dtype=np.int64)
        _check(_lib.drts_batch_run(self._h, ptrs, steps.ctypes.data_as(C.POINTER(i64))), "drts_batch_run")

    def autotune(self) -> dict:
        """drts_batch_autotune: one launch shape for all CSR members, before
        their first step; returns the chosen options (grid: the batch's)."""
        o = OptionsT()
        _check(_lib.drts_batch_autotune(self._h, C.byref(o)), "drts_batch_autotune")
        return {k: getattr(o, k) for k, _ in OptionsT._fields_}


class Server:
    """Continuous batching of independent FP32 solves (drts_serve_*); kernel
    other than KERNEL_CSR selects the matrix-free step for every request
    admitted (drts_serve_set_step)."""

    def __init__(self, budget_bytes: int, quantum: int = 50, max_active: int = 256, max_skips: int = 8,
                 policy: str = "arrival", device: Optional[TorchDevice] = None, kernel: int = KERNEL_CSR):
        self.device = device or default_device()
        h = P()
        pol = {"arrival": SERVE_ARRIVAL, "shortest": SERVE_SHORTEST}[policy]
        _check(_lib.drts_serve_create(C.byref(self.device.c), int(budget_bytes), int(quantum), int(max_active),
                                      int(max_skips), pol, C.byref(h)), "drts_serve_create")
        self._h = h
        if kernel != KERNEL_CSR:
            _check(_lib.drts_serve_set_step(self._h, int(kernel)), "drts_serve_set_step")
        self._req = {}     # id -> (n_steps, n_det, source table kept alive)

    def close(self):
        if getattr(self, "_h", None):
            _lib.drts_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, medium, sources: Optional[SourceTable], detectors: Sequence, n_steps: int,
               rounding: str = "dither", n_ref: Optional[float] = None) -> int:
        m, keep = _medium_struct(medium, "f32", rounding, n_ref)
        dt, _ = _detectors_struct(medium, detectors)
        rid = i64()
        _check(_lib.drts_serve_submit(self._h, C.byref(m), C.byref(sources.c) if sources is not None else None,
                                      C.byref(dt) if dt is not None else None, int(n_steps), C.byref(rid)),
               "drts_serve_submit")
        self._req[rid.value] = (int(n_steps), len(detectors), sources)
        return rid.value

    @staticmethod
    def footprint(medium, sources: Optional[SourceTable], detectors: Sequence, n_steps: int,
                  rounding: str = "dither", n_ref: Optional[float] = None) -> int:
        m, keep = _medium_struct(medium, "f32", rounding, n_ref)
        dt, _ = _detectors_struct(medium, detectors)
        b = i64()
        _check(_lib.drts_serve_footprint(C.byref(m), C.byref(sources.c) if sources is not None else None,
                                         C.byref(dt) if dt is not None else None, int(n_steps), C.byref(b)),
               "drts_serve_footprint")
        return b.value

    def tick(self) -> dict:
        a, w, f, b = i32(), i32(), i32(), i64()
        _check(_lib.drts_serve_tick(self._h, C.byref(a), C.byref(w), C.byref(f), C.byref(b)), "drts_serve_tick")
        return {"active": a.value, "waiting": w.value, "finished": f.value, "bytes": b.value}

    def poll(self) -> List[int]:
        out = []
        buf = (i64 * 256)()
        n = i32()
        while True:
            _check(_lib.drts_serve_poll(self._h, buf, 256, C.byref(n)), "drts_serve_poll")
            out.extend(buf[:n.value])
            if n.value < 256:
                return out

    def result(self, rid: int) -> dict:
        n_steps, n_det, _ = self._req[rid]
        ser = np.zeros((n_steps, max(n_det, 1)))
        e = np.zeros(n_steps, dtype=np.int32)
        tot = np.zeros((n_steps, 3))
        _check(_lib.drts_serve_result(self._h, int(rid), ser.ctypes.data, e.ctypes.data, tot.ctypes.data),
               "drts_serve_result")
        return {"det": ser[:, :n_det], "exp2": e, "tot": tot}

    def release(self, rid: int):
        _check(_lib.drts_serve_release(self._h, int(rid)), "drts_serve_release")
        self._req.pop(rid, None)
