"""FP64 CPU oracle of the DRTS time step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  The product library (``include/drts.h``
and ``paper_1611_08536_amd``) never imports, links or executes it, and the two
share no code: the only module both sides read is ``workloads`` (seeded
inputs, none of the method's arithmetic).

The arithmetic lives in ``drts_oracle.c`` (plain C, FP64): assembly of the
system matrix of Eq. (21)/(23) plus escape rows, the evolution of Eq. (26)
and the one-step detector sums of Eq. (27).  This module compiles it with gcc
on first use and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "drts_oracle.c")
_LIB = os.path.join(_HERE, "_drts_oracle.so")
_lock = threading.Lock()
_lib = None

GEOM = {"voxels": 0, "homog": 0, "layers_z": 1, "sphere": 2}
BC = {"vacuum": 0, "reflect": 1}


def build(force: bool = False) -> str:
    """Compile the oracle library with gcc (FP contraction off, OpenMP on)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Medium(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_mat", C.c_int32),
        ("h_mm", C.c_double),
        ("mat", C.POINTER(C.c_double)),
        ("mat_of_voxel", C.POINTER(C.c_uint8)),
        ("geom", C.c_int32), ("bc", C.c_int32),
        ("sphere_c", C.c_double * 3), ("sphere_r", C.c_double),
        ("scatter_order", C.c_int32),
        ("directions", C.c_int32), ("c_dt", C.c_double),
        ("interface_model", C.c_int32),
    ]


DIRECTIONS = {"lattice26": 0, "lebedev86": 1}
INTERFACE = {"origin": 0, "substep": 1}


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        lib = C.CDLL(build())
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        lib.or_build.restype = P
        lib.or_build.argtypes = [C.POINTER(_Medium)]
        lib.or_free.argtypes = [P]
        for name in ("or_n_vox", "or_n_states", "or_n_escape", "or_n_rows", "or_nnz"):
            getattr(lib, name).restype = i64
            getattr(lib, name).argtypes = [P]
        for name in ("or_row_ptr", "or_col", "or_val", "or_absorb_of_voxel"):
            getattr(lib, name).restype = P
            getattr(lib, name).argtypes = [P]
        lib.or_row_of.restype = i64
        lib.or_row_of.argtypes = [P, i64, C.c_int]
        lib.or_round_f32.argtypes = [P, C.c_int, P]
        lib.or_spmv.argtypes = [P, P, P, P]
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_set_threads.restype = None
        lib.or_run.restype = C.c_int
        lib.or_run.argtypes = [P, P, i64, P, i32,
                               i64, P, P, P, i32, P,
                               i64, P, P, P, i32,
                               P, P, P, P, P, P]
        lib.or_n_dir.restype = C.c_int
        lib.or_n_dir.argtypes = [P]
        lib.or_lebedev86.argtypes = [P, P]
        lib.or_leb_open.restype = P
        lib.or_leb_open.argtypes = [C.POINTER(_Medium)]
        lib.or_leb_close.argtypes = [P]
        for name in ("or_leb_n_rows", "or_leb_n_escape"):
            getattr(lib, name).restype = i64
            getattr(lib, name).argtypes = [P]
        lib.or_leb_row.restype = i64
        lib.or_leb_row.argtypes = [P, i64, P, P, i64]
        lib.or_leb_stencil.restype = i64
        lib.or_leb_stencil.argtypes = [P, C.c_int, C.c_int, P, P, i64]
        lib.or_leb_block.argtypes = [P, C.c_int, P]
        lib.or_collision_block.argtypes = [dbl, dbl, dbl, dbl, P]
        lib.or_collision_block_k.argtypes = [dbl, dbl, dbl, dbl, C.c_int, P]
        lib.or_fresnel.argtypes = [C.c_int, dbl, dbl, P, P, P, P, P, P, P]
        lib.or_dt_seconds.restype = dbl
        lib.or_dt_seconds.argtypes = [dbl, dbl]
        lib.or_gaussian_step.restype = dbl
        lib.or_gaussian_step.argtypes = [dbl, dbl, i64]
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- scalar pieces, exposed for the pins ----------------------------------

def set_threads(n: int) -> None:
    """Threads of the oracle's SpMV loop from now on (timing only; n < 1 keeps
    the OpenMP default).  Results do not depend on it."""
    _load().or_set_threads(int(n))


def collision_block(mu_s, mu_a, g, h_mm, order: int = 1) -> np.ndarray:
    """26x26 direction block C[m, n] of one material (Eq. (9), (10), (19), (21));
    order K > 1 resolves up to K scatterings per step (Eq. (4))."""
    out = np.zeros(26 * 26, dtype=np.float64)
    if order == 1:
        _load().or_collision_block(mu_s, mu_a, g, h_mm, _ptr(out))
    else:
        _load().or_collision_block_k(mu_s, mu_a, g, h_mm, int(order), _ptr(out))
    return out.reshape(26, 26)


def fresnel(m: int, n1: float, n2: float, normal) -> tuple:
    """(R, T, reflected directions, transmitted directions) for lattice
    direction m crossing n1 -> n2; tied directions share their part evenly."""
    N = np.ascontiguousarray(normal, dtype=np.float64)
    R, T = C.c_double(), C.c_double()
    mr, mt = (C.c_int * 26)(), (C.c_int * 26)()
    nr, nt = C.c_int(), C.c_int()
    _load().or_fresnel(m, n1, n2, _ptr(N), C.byref(R), C.byref(T), mr, C.byref(nr), mt, C.byref(nt))
    return R.value, T.value, list(mr[:nr.value]), list(mt[:nt.value])


def lebedev86():
    """(S [86, 3], w [86]): the directions (ascending z, y, x) and normalised
    weights of Lebedev's 86-point rule."""
    S = np.zeros((86, 3))
    w = np.zeros(86)
    _load().or_lebedev86(_ptr(S), _ptr(w))
    return S, w


def dt_seconds(h_mm: float, n_ref: float) -> float:
    return _load().or_dt_seconds(h_mm, n_ref)


def gaussian_step(fwhm_s: float, dt_s: float, t: int) -> float:
    return _load().or_gaussian_step(fwhm_s, dt_s, t)


def amplitudes(sources, dt_s: float, n_steps: int) -> np.ndarray:
    """[n_steps, n_src] photons emitted per step by each source function (Eq. (26))."""
    amp = np.zeros((n_steps, len(sources)), dtype=np.float64)
    for j, s in enumerate(sources):
        if s.kind == "impulse":
            amp[0, j] = 1.0
        elif s.kind == "gaussian":
            f = s.fwhm_fs * 1e-15
            for t in range(n_steps):
                amp[t, j] = gaussian_step(f, dt_s, t)
        else:
            raise ValueError("unknown source kind %r" % s.kind)
    return amp


def dir_index(dx: int, dy: int, dz: int) -> int:
    k = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
    return k if k < 13 else k - 1


# ---- assembled matrix -------------------------------------------------------

def _medium_struct(medium):
    mat = np.ascontiguousarray(
        [[m.mu_s, m.mu_a, m.g, m.n] for m in medium.materials], dtype=np.float64).reshape(-1)
    vmap = np.ascontiguousarray(medium.mat_of_voxel, dtype=np.uint8).reshape(-1)
    assert vmap.size == medium.nx * medium.ny * medium.nz
    st = _Medium()
    st.nx, st.ny, st.nz = medium.nx, medium.ny, medium.nz
    st.n_mat = len(medium.materials)
    st.h_mm = medium.h_mm
    st.mat = mat.ctypes.data_as(C.POINTER(C.c_double))
    st.mat_of_voxel = vmap.ctypes.data_as(C.POINTER(C.c_uint8))
    st.geom = GEOM[medium.geom]
    st.bc = BC[medium.bc]
    c = medium.sphere_c if medium.sphere_c is not None else (0.0, 0.0, 0.0)
    st.sphere_c = (C.c_double * 3)(*c)
    st.sphere_r = medium.sphere_r or 0.0
    st.scatter_order = getattr(medium, "scatter_order", 1)
    st.directions = DIRECTIONS[getattr(medium, "directions", "lattice26")]
    st.c_dt = getattr(medium, "c_dt", 1.0)
    st.interface_model = INTERFACE[getattr(medium, "interface", "origin")]
    return st, (mat, vmap)


class LebedevRows:
    """Single rows of a Lebedev medium's [A; L] without assembling it (the
    same products as the assembly; for sampled checks of large media)."""

    def __init__(self, medium):
        self._st, self._keep = _medium_struct(medium)
        self._h = _load().or_leb_open(C.byref(self._st))
        if not self._h:
            raise MemoryError("oracle model failed")
        self.n_states = 86 * medium.nx * medium.ny * medium.nz
        self.n_rows = _load().or_leb_n_rows(self._h)
        self.n_escape = _load().or_leb_n_escape(self._h)

    def row(self, r: int):
        cap = 4096
        col = np.zeros(cap, dtype=np.int32)
        val = np.zeros(cap)
        k = _load().or_leb_row(self._h, int(r), _ptr(col), _ptr(val), cap)
        assert k <= cap
        return col[:k].copy(), val[:k].copy()

    def stencil(self, m: int, n: int):
        off = np.zeros((4096, 3), dtype=np.int32)
        w = np.zeros(4096)
        k = _load().or_leb_stencil(self._h, m, n, _ptr(off), _ptr(w), 4096)
        return off[:k].copy(), w[:k].copy()

    def block(self, q: int = 0) -> np.ndarray:
        C_ = np.zeros(86 * 86)
        _load().or_leb_block(self._h, q, _ptr(C_))
        return C_.reshape(86, 86)

    def close(self):
        if getattr(self, "_h", None):
            _load().or_leb_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """Oracle assembly of [A; L] for one medium (FP64, int64 row pointers)."""

    def __init__(self, medium):
        lib = _load()
        st, (self._mat, self._map) = _medium_struct(medium)
        self._st = st
        self.medium = medium
        h = lib.or_build(C.byref(st))
        if not h:
            raise MemoryError("oracle assembly failed")
        self._h = h
        self.n_vox = lib.or_n_vox(h)
        self.n_states = lib.or_n_states(h)
        self.n_escape = lib.or_n_escape(h)
        self.n_rows = lib.or_n_rows(h)
        self.nnz = lib.or_nnz(h)
        self.n_dir = lib.or_n_dir(h)

    def close(self):
        if getattr(self, "_h", None):
            _load().or_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _view(self, fn, dtype, n):
        p = getattr(_load(), fn)(self._h)
        buf = (C.c_char * (n * np.dtype(dtype).itemsize)).from_address(p)
        return np.frombuffer(buf, dtype=dtype, count=n)

    @property
    def row_ptr(self) -> np.ndarray:
        return self._view("or_row_ptr", np.int64, self.n_rows + 1)

    @property
    def col(self) -> np.ndarray:
        return self._view("or_col", np.int32, self.nnz)

    @property
    def val(self) -> np.ndarray:
        return self._view("or_val", np.float64, self.nnz)

    @property
    def absorb_of_voxel(self) -> np.ndarray:
        return self._view("or_absorb_of_voxel", np.float64, self.n_vox)

    def row_of(self, state: int, escape: bool) -> int:
        return _load().or_row_of(self._h, int(state), 1 if escape else 0)

    def rows_of(self, states, escape) -> np.ndarray:
        states = np.asarray(states, dtype=np.int64).reshape(-1)
        escape = np.broadcast_to(np.asarray(escape, dtype=bool), states.shape)
        return np.array([self.row_of(s, e) for s, e in zip(states, escape)], dtype=np.int64)

    def round_f32(self, mode: str = "dither") -> np.ndarray:
        out = np.empty(self.nnz, dtype=np.float32)
        _load().or_round_f32(self._h, {"nearest": 0, "dither": 1}[mode], _ptr(out))
        return out

    def to_scipy(self, vals=None):
        import scipy.sparse as sp
        v = self.val if vals is None else vals
        return sp.csr_matrix((np.array(v, dtype=np.float64), self.col.copy(), self.row_ptr.copy()),
                             shape=(self.n_rows, self.n_states))

    def spmv(self, x, vals32=None) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size >= self.n_states
        y = np.empty(self.n_rows, dtype=np.float64)
        _load().or_spmv(self._h, _ptr(vals32), _ptr(x), _ptr(y))
        return y

    def run(self, n_steps, src_rows=None, src_ids=None, src_w=None, amp=None,
            det_rows=None, det_ids=None, det_F=None, n_det=0, x0=None, e0=0, vals32=None):
        """FP64 evolution of Eq. (26).  Returns a dict of (value, exponent) arrays."""
        lib = _load()
        n_steps = int(n_steps)
        i64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.int64)
        i32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.int32)
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        src_rows, src_ids, src_w, amp = i64(src_rows), i32(src_ids), f64(src_w), f64(amp)
        det_rows, det_ids, det_F = i64(det_rows), i32(det_ids), f64(det_F)
        n_src_e = 0 if src_rows is None else src_rows.size
        n_src = 0 if amp is None else (amp.shape[1] if amp.ndim == 2 else 1)
        n_det_e = 0 if det_rows is None else det_rows.size
        if n_src_e:
            assert src_rows.max() < self.n_states and src_rows.min() >= 0
            assert amp.shape[0] >= n_steps
        if n_det_e:
            assert det_rows.min() >= 0 and det_rows.max() < self.n_rows
        tot = np.zeros((n_steps, 3))
        tot_e = np.zeros((n_steps, 3), dtype=np.int32)
        det = np.zeros((n_steps, max(n_det, 1)))
        det_e = np.zeros((n_steps, max(n_det, 1)), dtype=np.int32)
        x_out = np.zeros(self.n_states)
        e_out = C.c_int32()
        if vals32 is not None:
            vals32 = np.ascontiguousarray(vals32, dtype=np.float32)
            assert vals32.size == self.nnz
        x0 = f64(x0)
        rc = lib.or_run(self._h, _ptr(vals32), n_steps, _ptr(x0), int(e0),
                        n_src_e, _ptr(src_rows), _ptr(src_ids), _ptr(src_w), n_src, _ptr(amp),
                        n_det_e, _ptr(det_rows), _ptr(det_ids), _ptr(det_F), int(n_det),
                        _ptr(tot), _ptr(tot_e), _ptr(det), _ptr(det_e), _ptr(x_out),
                        C.byref(e_out))
        if rc != 0:
            raise MemoryError("oracle run failed")
        return {"tot": tot, "tot_exp": tot_e, "det": det[:, :n_det], "det_exp": det_e[:, :n_det],
                "x": x_out, "x_exp": int(e_out.value)}


# ---- windowed measurement ------------------------------------------------------

def window(det, det_exp, taps, tap0=0, t_done=None):
    """Readings of sensors with impulse responses (Eq. (27) over several steps):
    M_d(t) = sum_j taps[d][j] m_d(t - tap0 - j) for every step t of the series,
    where m_d(s) = det[s, d] * 2^det_exp[s, d] is the one-step detector sum and
    steps outside 0 .. t_done - 1 contribute nothing.  Plain FP64 loops,
    ascending j; returns physical values [T, n_det]."""
    det = np.asarray(det, dtype=np.float64)
    T, nd = det.shape
    t_done = T if t_done is None else t_done
    m = np.ldexp(det, np.asarray(det_exp))
    taps = np.broadcast_to(np.asarray(taps, dtype=np.float64), (nd, np.asarray(taps).shape[-1]))
    out = np.zeros((T, nd))
    for t in range(T):
        for d in range(nd):
            acc = 0.0
            for j in range(taps.shape[1]):
                s = t - tap0 - j
                if 0 <= s < t_done and taps[d, j] != 0.0:
                    acc += taps[d, j] * m[s, d]
            out[t, d] = acc
    return out


# ---- workload helpers (oracle side of the row mapping) ----------------------

def state_of(medium, vox, dirs) -> np.ndarray:
    """State index of voxels (x,y,z) and directions: 26 v + d for lattice
    vectors (dx,dy,dz); on Lebedev media 86 v + n with n the rule's direction
    nearest the given vector (largest cosine, the lowest index on ties)."""
    vox = np.asarray(vox, dtype=np.int64).reshape(-1, 3)
    v = vox[:, 0] + medium.nx * (vox[:, 1] + medium.ny * vox[:, 2])
    if getattr(medium, "directions", "lattice26") == "lebedev86":
        S, _ = lebedev86()
        dv = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
        dv = dv / np.linalg.norm(dv, axis=1, keepdims=True)
        d = np.argmax(dv @ S.T, axis=1)
        return 86 * v + d
    dirs = np.asarray(dirs, dtype=np.int64).reshape(-1, 3)
    k = 9 * (dirs[:, 2] + 1) + 3 * (dirs[:, 1] + 1) + (dirs[:, 0] + 1)
    d = np.where(k < 13, k, k - 1)
    return 26 * v + d


def source_arrays(A: Matrix, workload, rhs=None):
    """(rows, ids, weights, amplitudes) of the workload's sources feeding one rhs."""
    med = workload.medium
    # the step: light crosses c_dt voxels (one on the lattice)
    dt = dt_seconds(med.h_mm * getattr(med, "c_dt", 1.0), workload.n_ref)
    srcs = [s for s in workload.sources if rhs is None or s.rhs == rhs]
    rows, ids, w = [], [], []
    for j, s in enumerate(srcs):
        st = state_of(med, s.vox, s.dirs)
        rows.append(st)
        ids.append(np.full(st.size, j, dtype=np.int32))
        w.append(np.asarray(s.w, dtype=np.float64))
    amp = amplitudes(srcs, dt, workload.n_steps)
    return np.concatenate(rows), np.concatenate(ids), np.concatenate(w), amp


def detector_arrays(A: Matrix, workload):
    med = workload.medium
    rows, ids, F = [], [], []
    for j, d in enumerate(workload.detectors):
        st = state_of(med, d.vox, d.dirs)
        r = A.rows_of(st, d.escape)
        if (r < 0).any():
            raise ValueError("detector entry on a state that does not leave the grid")
        rows.append(r)
        ids.append(np.full(r.size, j, dtype=np.int32))
        F.append(np.asarray(d.F, dtype=np.float64))
    if not rows:
        return None, None, None, 0
    return np.concatenate(rows), np.concatenate(ids), np.concatenate(F), len(workload.detectors)


def run_workload(A: Matrix, workload, rhs=None, n_steps=None, vals32=None):
    """Runs one right-hand side of a workload through the oracle."""
    sr, si, sw, amp = source_arrays(A, workload, rhs)
    dr, di, dF, nd = detector_arrays(A, workload)
    return A.run(n_steps or workload.n_steps, sr, si, sw, amp, dr, di, dF, nd, vals32=vals32)
