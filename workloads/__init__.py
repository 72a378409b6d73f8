"""Seeded synthetic inputs of the DRTS workloads (no arithmetic of the method).

Both the product path and the oracle read their inputs from here and nowhere
else.  A workload is a medium (grid, materials, a voxel material map, the
surface description used for interface normals, boundary type), a list of
source functions with their spatial/directional support, detectors, a step
count and the arithmetic type.  Sources and detectors name voxels by their
integer coordinates and directions by their lattice vector (dx, dy, dz); each
side maps them to its own state indices.

Random draws use ``numpy.random.default_rng([161108536, cfg_id])``.

Workloads (lengths in mm, coefficients in 1/mm, voxel edge h = 0.1 mm):
  C1  16^3 homogeneous (mu_s 10, mu_a 0.01, g 0.9, n 1.4), vacuum faces,
      unit impulse at the centre voxel in +z, 200 steps, FP64.
  C2  128^3, three planar layers (5/0.005/0.8/1.33, 15/0.05/0.9/1.45,
      10/0.02/0.85/1.40) split at floor(N/3), floor(2N/3); vacuum faces;
      every z = 0 voxel emits a 100 fs Gaussian pulse in +z with weight
      1/N^2; detectors: everything leaving through z = 0 (reflectance) and
      z = N-1 (transmittance); 2000 steps, FP32.
  C3  96^3 homogeneous slab (10, 0.01, 0.9, 1.4), 64 right-hand sides: 64
      distinct z = 0 voxels (drawn) in +z, FWHM ~ U(50, 500) fs; 16 detectors
      = 4x4 patches of the z = 0 face; 1000 steps, FP32.
  C4  256 independent cubes, edge ~ U{16..64}, mu_s ~ logU(1, 20),
      mu_a ~ logU(0.001, 0.1), g ~ U(0.7, 0.95), n 1.4, vacuum, impulse at the
      centre voxel in +z; 500 steps each, FP32.
  C5  request stream: Poisson arrivals at 200/s; cube edge ~ U{32..128};
      background (10, 0.01, 0.9, 1.33) with a spherical inclusion of radius
      U(0.1, 0.3) N, mu_a U(2, 10) x 0.01, n 1.45; impulse at the centre of
      the z = 0 face in +z; steps ~ U{500..5000}; FP32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED = 161108536


def rng(cfg_id: int) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg_id])


@dataclasses.dataclass
class Material:
    mu_s: float   # scattering coefficient, 1/mm
    mu_a: float   # absorption coefficient, 1/mm
    g: float      # Henyey-Greenstein anisotropy
    n: float      # refractive index


@dataclasses.dataclass
class Medium:
    nx: int
    ny: int
    nz: int
    h_mm: float
    materials: List[Material]
    mat_of_voxel: np.ndarray            # uint8 [nz, ny, nx] (x fastest)
    geom: str = "voxels"                # "voxels" | "layers_z" | "sphere"
    bc: str = "vacuum"                  # "vacuum" | "reflect"
    sphere_c: Optional[Tuple[float, float, float]] = None   # voxel units, centres at i + 0.5
    sphere_r: Optional[float] = None
    layer_z0: Tuple[int, ...] = ()
    scatter_order: int = 1              # scatterings per step the direction block resolves
    directions: str = "lattice26"       # "lattice26" | "lebedev86" (Sec. 3, Eq. (18)-(19))
    c_dt: float = 1.0                   # lebedev86: light path per step, in voxels
    interface: str = "origin"           # "origin" | "substep": crossing within the step (Sec. 4.2)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_states(self) -> int:
        return 26 * self.n_vox


@dataclasses.dataclass
class Source:
    kind: str                 # "impulse" (one photon at step 0) | "gaussian"
    vox: np.ndarray           # int [k, 3] voxel coordinates
    dirs: np.ndarray          # int [k, 3] lattice vectors
    w: np.ndarray             # float [k] weights
    fwhm_fs: float = 0.0
    rhs: int = 0


@dataclasses.dataclass
class Detector:
    vox: np.ndarray           # int [k, 3]
    dirs: np.ndarray          # int [k, 3]
    escape: np.ndarray        # bool [k]: the escape row of (voxel, direction), else the state
    F: np.ndarray             # float [k]
    name: str = ""


@dataclasses.dataclass
class Workload:
    name: str
    medium: Medium
    sources: List[Source]
    detectors: List[Detector]
    n_steps: int
    n_rhs: int = 1
    value_type: str = "f32"   # "f64" | "f32"
    rounding: str = "dither"  # FP64 -> FP32 value rounding: "nearest" | "dither"
    n_ref: float = 1.4        # refractive index that sets dt (source material)


def lattice_vectors() -> np.ndarray:
    """The 26 neighbour offsets in ascending order of 9(dz+1)+3(dy+1)+(dx+1)."""
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx or dy or dz:
                    out.append((dx, dy, dz))
    return np.array(out, dtype=np.int64)


def homogeneous(n: int, mat: Material, h_mm: float = 0.1, bc: str = "vacuum",
                ny: Optional[int] = None, nz: Optional[int] = None) -> Medium:
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    return Medium(n, ny, nz, h_mm, [mat], np.zeros((nz, ny, n), dtype=np.uint8), "voxels", bc)


def layered(n: int, mats: Sequence[Material], h_mm: float = 0.1, bc: str = "vacuum") -> Medium:
    k = len(mats)
    z0 = tuple((i * n) // k for i in range(k))
    m = np.zeros((n, n, n), dtype=np.uint8)
    for i, z in enumerate(z0):
        m[z:, :, :] = i
    return Medium(n, n, n, h_mm, list(mats), m, "layers_z", bc, layer_z0=z0)


def sphere_inclusion(n: int, bg: Material, inc: Material, c, r, h_mm: float = 0.1,
                     bc: str = "vacuum") -> Medium:
    idx = np.arange(n) + 0.5
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    inside = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= r * r
    m = inside.astype(np.uint8)
    return Medium(n, n, n, h_mm, [bg, inc], m, "sphere", bc,
                  sphere_c=tuple(float(v) for v in c), sphere_r=float(r))


def extend_top(med: Medium, gap: int, n_ext: Optional[float] = None) -> Medium:
    """The medium with `gap` planes of free space (no scattering, no
    absorption) added above its z = 0 face, so that a sensor outside the
    volume can be placed in the grid (Sec. 4.2).  Voxel (x, y, z) of the
    original is voxel (x, y, z + gap) of the result.  The free space has index
    n_ext, by default the index of the original's top voxels (no interface at
    the original surface, as at its vacuum faces)."""
    top = med.materials[int(med.mat_of_voxel[0, 0, 0])]
    free = Material(0.0, 0.0, 0.0, top.n if n_ext is None else n_ext)
    m = np.empty((med.nz + gap, med.ny, med.nx), dtype=np.uint8)
    m[:gap] = 0
    m[gap:] = med.mat_of_voxel + 1
    sc = None if med.sphere_c is None else (med.sphere_c[0], med.sphere_c[1], med.sphere_c[2] + gap)
    z0 = (0,) + tuple(gap + z for z in med.layer_z0) if med.layer_z0 else ()
    return Medium(med.nx, med.ny, med.nz + gap, med.h_mm, [free] + list(med.materials), m, med.geom, med.bc,
                  sc, med.sphere_r, z0, med.scatter_order)


def shifted_z(item, gap: int):
    """A source or detector of the original medium, on the medium extended by
    extend_top(med, gap)."""
    import copy
    out = copy.copy(item)
    out.vox = np.asarray(item.vox) + np.array([0, 0, gap])
    return out


def point_source(x, y, z, d=(0, 0, 1), kind="impulse", fwhm_fs=0.0, rhs=0, w=1.0) -> Source:
    return Source(kind, np.array([[x, y, z]]), np.array([d]), np.array([w], dtype=np.float64),
                  fwhm_fs, rhs)


def face_escape_detector(med: Medium, face: str, x0=0, x1=None, y0=0, y1=None, name="") -> Detector:
    """Everything leaving through the z = 0 ("top") or z = nz-1 ("bottom") face
    inside the patch [x0, x1) x [y0, y1), one escape entry per outward direction."""
    x1 = med.nx if x1 is None else x1
    y1 = med.ny if y1 is None else y1
    z, sz = (0, -1) if face == "top" else (med.nz - 1, 1)
    lv = lattice_vectors()
    outward = lv[lv[:, 2] == sz]
    ys, xs = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    vox = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, z)], axis=1)
    vox = np.repeat(vox, len(outward), axis=0)
    dirs = np.tile(outward, (xs.size, 1))
    k = len(vox)
    return Detector(vox, dirs, np.ones(k, dtype=bool), np.ones(k, dtype=np.float64), name or face)


# ---- the five workloads -------------------------------------------------------

C1_MAT = Material(10.0, 0.01, 0.9, 1.4)
C2_MATS = (Material(5.0, 0.005, 0.8, 1.33), Material(15.0, 0.05, 0.9, 1.45),
           Material(10.0, 0.02, 0.85, 1.40))
C3_MAT = Material(10.0, 0.01, 0.9, 1.4)


def c1(n: int = 16, n_steps: int = 200, bc: str = "vacuum") -> Workload:
    med = homogeneous(n, C1_MAT, bc=bc)
    c = n // 2
    return Workload("C1", med, [point_source(c, c, c)], [], n_steps, 1, "f64", "nearest", 1.4)


def c2(n: int = 128, n_steps: int = 2000, value_type: str = "f32",
       rounding: str = "dither") -> Workload:
    med = layered(n, C2_MATS)
    ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    vox = np.stack([xs.ravel(), ys.ravel(), np.zeros(n * n, dtype=np.int64)], axis=1)
    src = Source("gaussian", vox, np.tile([[0, 0, 1]], (n * n, 1)),
                 np.full(n * n, 1.0 / (n * n)), fwhm_fs=100.0)
    dets = [face_escape_detector(med, "top", name="reflectance"),
            face_escape_detector(med, "bottom", name="transmittance")]
    return Workload("C2", med, [src], dets, n_steps, 1, value_type, rounding, C2_MATS[0].n)


def c3(n: int = 96, k: int = 64, n_steps: int = 1000, rounding: str = "dither") -> Workload:
    r = rng(3)
    med = homogeneous(n, C3_MAT)
    cells = r.choice(n * n, size=k, replace=False)
    fwhm = r.uniform(50.0, 500.0, size=k)
    srcs = [point_source(int(c % n), int(c // n), 0, kind="gaussian", fwhm_fs=float(f), rhs=j)
            for j, (c, f) in enumerate(zip(cells, fwhm))]
    p = n // 4
    dets = [face_escape_detector(med, "top", i * p, (i + 1) * p, j * p, (j + 1) * p,
                                 name="patch%d%d" % (j, i))
            for j in range(4) for i in range(4)]
    return Workload("C3", med, srcs, dets, n_steps, k, "f32", rounding, C3_MAT.n)


def c4(n_inst: int = 256, n_steps: int = 500, edge=(16, 64)) -> List[Workload]:
    r = rng(4)
    out = []
    for i in range(n_inst):
        n = int(r.integers(edge[0], edge[1] + 1))
        mu_s = float(math.exp(r.uniform(math.log(1.0), math.log(20.0))))
        mu_a = float(math.exp(r.uniform(math.log(0.001), math.log(0.1))))
        g = float(r.uniform(0.7, 0.95))
        mat = Material(mu_s, mu_a, g, 1.4)
        med = homogeneous(n, mat)
        c = n // 2
        out.append(Workload("C4.%d" % i, med, [point_source(c, c, c)], [], n_steps, 1,
                            "f32", "dither", 1.4))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    workload: Workload


def c5(n_req: int = 256, rate: float = 200.0, edge=(32, 128), steps=(500, 5000)) -> List[Request]:
    r = rng(5)
    bg = Material(10.0, 0.01, 0.9, 1.33)
    t = 0.0
    out = []
    for i in range(n_req):
        t += float(r.exponential(1.0 / rate))
        n = int(r.integers(edge[0], edge[1] + 1))
        rad = float(r.uniform(0.1, 0.3)) * n
        c = r.uniform(rad, n - rad, size=3)
        inc = Material(10.0, float(r.uniform(2.0, 10.0)) * 0.01, 0.9, 1.45)
        med = sphere_inclusion(n, bg, inc, c, rad)
        n_steps = int(r.integers(steps[0], steps[1] + 1))
        wl = Workload("C5.%d" % i, med, [point_source(n // 2, n // 2, 0)],
                      [face_escape_detector(med, "top", name="reflectance")],
                      n_steps, 1, "f32", "dither", bg.n)
        out.append(Request(t, wl))
    return out


def seeded_state(n: int, cfg_id: int, scale: float = 1.0) -> np.ndarray:
    """A nonnegative seeded state vector (for one-step comparisons)."""
    return rng(1000 + cfg_id).random(n) * scale
