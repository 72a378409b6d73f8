"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle with
itself: they use closed forms, invariants stated in Sec. 3, textbook special
cases (Henyey-Greenstein, Fresnel), a second independent construction of the
matrix (pull-style, ``brute_dense``), brute force on tiny grids, published
test vectors and numerical quadrature.
"""
import ctypes
import math
import os

import numpy as np
import pytest

import workloads as W
from tests import brute_dense

LV = W.lattice_vectors()
DIR = {tuple(v): i for i, v in enumerate(LV)}


def _mat(mu_s, mu_a, g, n=1.4):
    return W.Material(mu_s, mu_a, g, n)


def _tiny_media():
    out = []
    for n in (3, 4):
        for bc in ("vacuum", "reflect"):
            out.append(("homog%d%s" % (n, bc), W.homogeneous(n, _mat(10.0, 0.5, 0.7), bc=bc)))
    lay = [_mat(5.0, 0.2, 0.8, 1.33), _mat(15.0, 0.5, 0.9, 1.45), _mat(10.0, 0.3, 0.6, 1.40)]
    for bc in ("vacuum", "reflect"):
        out.append(("layers4" + bc, W.layered(4, lay, bc=bc)))
    # off-centre sphere, strong contrast so that total internal reflection occurs
    bg, inc = _mat(10.0, 0.1, 0.9, 1.0), _mat(8.0, 0.4, 0.5, 1.6)
    for bc in ("vacuum", "reflect"):
        out.append(("sphere5" + bc, W.sphere_inclusion(5, bg, inc, (2.3, 2.6, 2.45), 1.6, bc=bc)))
    out.append(("slab343", W.homogeneous(3, _mat(2.0, 0.1, 0.3), bc="vacuum", ny=4, nz=3)))
    return out


TINY = _tiny_media()


# ---- assembly: two independent constructions agree bit for bit (Eq. (20)-(23))

@pytest.mark.parametrize("name,med", TINY, ids=[t[0] for t in TINY])
def test_push_assembly_equals_pull_dense(orc, name, med):
    A = orc.Matrix(med)
    dense, escapes = brute_dense.build_dense(med)
    assert A.n_escape == len(escapes)
    assert dense.shape == (A.n_rows, A.n_states)
    got = A.to_scipy().toarray()
    # bitwise: the same values, summed in the same order
    assert np.array_equal(got, dense), np.abs(got - dense).max()
    # structure: no stored zeros, columns ascending within rows
    rp, col = A.row_ptr, A.col
    for r in range(A.n_rows):
        c = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0)
    assert np.all(A.val > 0.0)


def test_interfaces_present_in_tiny_media(orc):
    """The tiny media really exercise walls, Fresnel splits and total internal reflection."""
    med = [m for n, m in TINY if n == "sphere5vacuum"][0]
    A = orc.Matrix(med)
    homog = orc.Matrix(W.homogeneous(5, med.materials[0]))
    assert A.nnz > homog.nnz      # the reflected parts add entries
    R, T, mr, mt = orc.fresnel(DIR[(1, 1, 1)], 1.6, 1.0, np.array([1.0, 0.0, 0.0]))
    assert R == 1.0 and T == 0.0 and mt == []


# ---- direction block: Eq. (9)-(10), (19), (21), (24) ---------------------------

def test_block_column_sums_equal_survival(orc):
    """Columns of A_S sum to one (Sec. 3), so columns of A sum to exp(-mu_a c dt) (Eq. (24))."""
    for mu_s, mu_a, g in [(10, 0.01, 0.9), (1.0, 0.1, 0.0), (20, 0.001, 0.95), (5, 0.5, -0.3)]:
        C = orc.collision_block(mu_s, mu_a, g, 0.1)
        alpha = math.exp(-mu_a * 0.1)
        assert np.allclose(C.sum(axis=0), alpha, rtol=0, atol=26 * 2.3e-16)
        assert np.all(C >= 0) and np.all(C <= 1)


def test_block_isotropic_closed_form(orc):
    """g = 0: every direction is equally likely after a scatter (p = 1/26)."""
    mu_s, mu_a, h = 3.0, 0.2, 0.1
    C = orc.collision_block(mu_s, mu_a, 0.0, h)
    P0, alpha = math.exp(-mu_s * h), math.exp(-mu_a * h)
    off = alpha * (1 - P0) / 26
    diag = alpha * (P0 + (1 - P0) / 26)
    assert np.allclose(C[~np.eye(26, dtype=bool)], off, rtol=1e-15)
    assert np.allclose(np.diag(C), diag, rtol=1e-15)


def test_block_no_scattering_is_identity(orc):
    """mu_s = 0: nothing scatters (Eq. (9)), the block is exp(-mu_a h) I."""
    C = orc.collision_block(0.0, 0.3, 0.9, 0.1)
    assert np.array_equal(C, math.exp(-0.03) * np.eye(26))


def test_block_follows_henyey_greenstein_ratios(orc):
    """Within one column the off-diagonal entries are in the ratio of the
    Henyey-Greenstein phase function at the angle between the two lattice
    directions (textbook form, normalisation cancels).  A transposed block or
    a wrong cosine fails this."""
    g = 0.8
    C = orc.collision_block(4.0, 0.05, g, 0.1)

    def hg(theta):
        return (1 - g * g) / (1 + g * g - 2 * g * math.cos(theta)) ** 1.5

    for n in (0, 4, 12, 21, 25):
        for m1, m2 in [(1, 7), (3, 20), (10, 15), (24, 2)]:
            if n in (m1, m2):
                continue
            a1 = math.acos(np.dot(LV[m1], LV[n]) / np.linalg.norm(LV[m1]) / np.linalg.norm(LV[n]))
            a2 = math.acos(np.dot(LV[m2], LV[n]) / np.linalg.norm(LV[m2]) / np.linalg.norm(LV[n]))
            assert C[m1, n] / C[m2, n] == pytest.approx(hg(a1) / hg(a2), rel=1e-12)


def test_block_diagonal_is_forward_plus_unscattered(orc):
    """The diagonal carries the unscattered population exp(-mu_s h) exp(-mu_a h)
    of Eq. (9) on top of the zero-angle scatter (Eq. (21))."""
    mu_s, mu_a, g, h = 7.0, 0.05, 0.6, 0.1
    C = orc.collision_block(mu_s, mu_a, g, h)
    Cs = orc.collision_block(mu_s, mu_a, g, h) - np.diag(np.diag(C))
    # the scattered part of the diagonal follows the same HG ratio as m = n in any column
    P0, alpha = math.exp(-mu_s * h), math.exp(-mu_a * h)
    # off-diagonal column sum + scattered diagonal = alpha (1 - P0)
    scat_diag = alpha * (1 - P0) - Cs.sum(axis=0)
    assert np.allclose(np.diag(C) - scat_diag, alpha * P0, rtol=1e-12)


# ---- Fresnel (Sec. 4.2) ------------------------------------------------------

def test_fresnel_normal_incidence(orc):
    for n1, n2 in [(1.33, 1.45), (1.45, 1.40), (1.0, 1.5)]:
        R, T, mr, mt = orc.fresnel(DIR[(0, 0, 1)], n1, n2, np.array([0.0, 0.0, 1.0]))
        assert R == pytest.approx(((n1 - n2) / (n1 + n2)) ** 2, rel=1e-13)
        assert R + T == 1.0
        assert mr == [DIR[(0, 0, -1)]] and mt == [DIR[(0, 0, 1)]]


def test_fresnel_oblique_matches_trig_form(orc):
    """R = (Rs + Rp)/2 with Rs = sin^2(i-t)/sin^2(i+t), Rp = tan^2(i-t)/tan^2(i+t)."""
    for d, (n1, n2) in [((1, 0, 1), (1.33, 1.45)), ((1, 1, 1), (1.45, 1.40)), ((0, 1, 1), (1.0, 1.5))]:
        m = DIR[d]
        N = np.array([0.0, 0.0, 1.0])
        R, T, mr, mt = orc.fresnel(m, n1, n2, N)
        s = np.array(d, float) / np.linalg.norm(d)
        ti = math.acos(s[2])
        tt = math.asin(n1 / n2 * math.sin(ti))
        Rs = math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2
        Rp = math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2
        assert R == pytest.approx(0.5 * (Rs + Rp), rel=1e-11)
        # planar interface: the mirror direction and, at these contrasts, the same direction
        assert mr == [DIR[(d[0], d[1], -d[2])]]
        assert mt == [m]


def test_fresnel_total_internal_reflection(orc):
    """Beyond the critical angle asin(n2/n1) everything is reflected."""
    m = DIR[(1, 0, 1)]   # 45 degrees
    R, T, mr, mt = orc.fresnel(m, 1.6, 1.0, np.array([0.0, 0.0, 1.0]))   # critical 38.7 deg
    assert (R, T, mt) == (1.0, 0.0, [])
    R, T, mr, mt = orc.fresnel(m, 1.3, 1.0, np.array([0.0, 0.0, 1.0]))   # critical 50.3 deg
    assert 0 < R < 1 and T == 1 - R


def test_layer_reflectance_values(orc):
    """Reflectances at the C2 interfaces for 0, 45 and 54.7 degrees."""
    N = np.array([0.0, 0.0, 1.0])
    vals = [orc.fresnel(DIR[d], 1.33, 1.45, N)[0] for d in [(0, 0, 1), (1, 0, 1), (1, 1, 1)]]
    assert vals == pytest.approx([1.863e-3, 3.208e-3, 6.561e-3], rel=2e-3)


# ---- sources (Sec. 4.1, Eq. (26)) ---------------------------------------------

def test_dt_is_voxel_crossing_time(orc):
    assert orc.dt_seconds(0.1, 1.33) == pytest.approx(0.1e-3 * 1.33 / 299792458.0, rel=1e-15)
    assert orc.dt_seconds(0.1, 1.33) == pytest.approx(443.6e-15, rel=1e-3)


def test_gaussian_pulse_integrals(orc):
    from scipy.integrate import quad
    for fwhm_fs, dt_fs in [(100.0, 443.6), (500.0, 467.0), (50.0, 30.0)]:
        f, dt = fwhm_fs * 1e-15, dt_fs * 1e-15
        sig = f / (2 * math.sqrt(2 * math.log(2)))
        tc = 3 * sig
        dens = lambda t: math.exp(-0.5 * ((t - tc) / sig) ** 2) / (sig * math.sqrt(2 * math.pi))
        steps = [orc.gaussian_step(f, dt, t) for t in range(int(12 * sig / dt) + 3)]
        assert sum(steps) == pytest.approx(1.0, abs=1e-14)
        for t in range(1, min(len(steps), 8)):
            ref = quad(dens, t * dt, (t + 1) * dt, epsabs=1e-15, epsrel=1e-13)[0]
            assert steps[t] == pytest.approx(ref, abs=1e-13)
        ref0 = quad(dens, -50 * sig, dt, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
        assert steps[0] == pytest.approx(ref0, abs=1e-13)


# ---- FP32 rounding of the values ------------------------------------------------

def test_splitmix64_published_sequence(orc):
    """splitmix64 seeded with 0: published first outputs."""
    lib = orc._load()
    lib.or_splitmix64_value.restype = ctypes.c_uint64
    lib.or_splitmix64_value.argtypes = [ctypes.c_uint64]
    g = 0x9E3779B97F4A7C15
    seq = [lib.or_splitmix64_value((k * g) & (2 ** 64 - 1)) for k in range(3)]
    assert seq == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_round_nearest_is_ieee_cast(orc):
    A = orc.Matrix(W.layered(6, W.C2_MATS))
    assert np.array_equal(A.round_f32("nearest"), A.val.astype(np.float32))


def test_round_dither_is_unbiased(orc):
    A = orc.Matrix(W.layered(10, W.C2_MATS))
    a = A.val
    f = A.round_f32("dither").astype(np.float64)
    lo = np.nextafter(a.astype(np.float32), np.float32(-np.inf)).astype(np.float64)
    hi = np.nextafter(a.astype(np.float32), np.float32(np.inf)).astype(np.float64)
    rn = a.astype(np.float32).astype(np.float64)
    # always one of the two float neighbours of a
    below = np.where(rn <= a, rn, lo)
    above = np.where(rn >= a, rn, hi)
    assert np.all((f == below) | (f == above))
    # unbiased: the relative rounding error averages out; nearest keeps a bias
    rel_d = (f - a) / a
    rel_n = (rn - a) / a
    n = a.size
    assert abs(rel_d.mean()) < 4 * rel_d.std() / math.sqrt(n)
    assert abs(rel_n.sum()) > abs(rel_d.sum()) * 5


# ---- time stepping: closed forms and invariants (Sec. 3, Eq. (23)-(27)) --------

def _coords(med):
    V = med.n_vox
    v = np.arange(V)
    return v % med.nx, (v // med.nx) % med.ny, v // (med.nx * med.ny)


def test_ballistic_shift_is_exact(orc):
    """mu_s = mu_a = 0: every population moves exactly one voxel along its own
    direction per step (Eq. (11)), and leaves at the faces."""
    med = W.homogeneous(6, _mat(0.0, 0.0, 0.9), ny=5, nz=4)
    A = orc.Matrix(med)
    assert A.nnz == A.n_states                        # one entry per column
    x0 = W.seeded_state(A.n_states, 1) + 0.5
    x, y, z = _coords(med)
    for t in (1, 2, 3):
        r = A.run(t, x0=x0)
        got = np.ldexp(r["x"], r["x_exp"]).reshape(-1, 26)
        want = np.zeros_like(got)
        xs = x0.reshape(-1, 26)
        for d, e in enumerate(LV):
            sx, sy, sz = x - t * e[0], y - t * e[1], z - t * e[2]
            ok = (sx >= 0) & (sx < med.nx) & (sy >= 0) & (sy < med.ny) & (sz >= 0) & (sz < med.nz)
            src = sx + med.nx * (sy + med.ny * sz)
            want[ok, d] = xs[src[ok], d]
        assert np.array_equal(got, want)
        # mass that left during the last step: populations one voxel from leaving
        esc = np.ldexp(r["tot"][-1, 1], r["tot_exp"][-1, 1])
        prev = np.ldexp(A.run(t - 1, x0=x0)["x"], A.run(t - 1, x0=x0)["x_exp"]).reshape(-1, 26) if t > 1 else xs
        leaving = 0.0
        for d, e in enumerate(LV):
            out = ~((x + e[0] >= 0) & (x + e[0] < med.nx) & (y + e[1] >= 0) & (y + e[1] < med.ny)
                    & (z + e[2] >= 0) & (z + e[2] < med.nz))
            leaving += prev[out, d].sum()
        assert esc == pytest.approx(leaving, rel=1e-14)


@pytest.mark.parametrize("mu_s", [0.0, 10.0])
def test_absorption_only_decay(orc, mu_s):
    """Closed walls: N(t) = exp(-mu_a c dt)^t N(0) (Eq. (8), (24))."""
    mu_a, h = 0.7, 0.1
    med = W.homogeneous(5, _mat(mu_s, mu_a, 0.9), bc="reflect")
    A = orc.Matrix(med)
    x0 = W.seeded_state(A.n_states, 2)
    r = A.run(40, x0=x0)
    N = np.ldexp(r["tot"][:, 0], r["tot_exp"][:, 0])
    alpha = math.exp(-mu_a * h)
    want = x0.sum() * alpha ** np.arange(1, 41)
    assert np.allclose(N, want, rtol=(2e-14 if mu_s == 0 else 1e-12))


def test_conservation_without_absorption(orc):
    """mu_a = 0 with reflecting walls: columns sum to one (Sec. 3) and the
    total never changes."""
    for med in (W.homogeneous(5, _mat(10.0, 0.0, 0.9), bc="reflect"),
                W.layered(6, [_mat(5, 0, 0.8, 1.33), _mat(15, 0, 0.9, 1.45), _mat(10, 0, 0.85, 1.4)],
                          bc="reflect")):
        A = orc.Matrix(med)
        S = A.to_scipy()
        colsum = np.asarray(S.sum(axis=0)).ravel()
        assert np.allclose(colsum, 1.0, rtol=0, atol=30 * 1.2e-16)
        x0 = W.seeded_state(A.n_states, 3)
        r = A.run(60, x0=x0)
        N = np.ldexp(r["tot"][:, 0], r["tot_exp"][:, 0])
        assert np.allclose(N, x0.sum(), rtol=1e-12)


def test_entries_are_probabilities_and_states_nonnegative(orc):
    """0 <= a <= 1 (Sec. 3) and nonnegative sources give nonnegative states."""
    for _, med in TINY:
        A = orc.Matrix(med)
        assert np.all((A.val > 0) & (A.val <= 1))
    w = W.c2(n=12, n_steps=30)
    A = orc.Matrix(w.medium)
    from oracle import run_workload
    r = run_workload(A, w)
    assert np.all(r["x"] >= 0) and np.all(r["tot"] >= 0) and np.all(r["det"] >= 0)


def test_interior_diagonal_is_zero(orc):
    """No photon returns to its own (voxel, direction) in one step (Sec. 3);
    diagonal entries appear only where a wall or an interface reflects."""
    med = W.homogeneous(6, _mat(10.0, 0.1, 0.5), bc="reflect")
    A = orc.Matrix(med)
    rp, col = A.row_ptr, A.col
    x, y, z = _coords(med)
    interior = (x > 0) & (x < 5) & (y > 0) & (y < 5) & (z > 0) & (z < 5)
    for r in range(A.n_states):
        has_diag = np.any(col[rp[r]:rp[r + 1]] == r)
        if interior[r // 26]:
            assert not has_diag
    # walls reflect -x into +x in the same voxel: diagonal exists there
    v = 0 + 6 * (3 + 6 * 3)
    r = 26 * v + DIR[(1, 0, 0)]
    assert np.any(col[rp[r]:rp[r + 1]] == r)


def test_light_cone(orc):
    """Photons travel at most one voxel per step (Sec. 3, finite c dt)."""
    w = W.c1(n=11, n_steps=4)
    A = orc.Matrix(w.medium)
    from oracle import run_workload
    x, y, z = _coords(w.medium)
    for t in (1, 2, 4):
        r = run_workload(A, w, n_steps=t)
        st = r["x"].reshape(-1, 26).sum(axis=1)
        dist = np.maximum(np.maximum(abs(x - 5), abs(y - 5)), abs(z - 5))
        assert st[dist > t - 1].sum() == 0.0
        assert st[dist == t - 1].sum() > 0.0


def test_body_diagonal_front(orc):
    """Only one lattice path reaches c + t(1,1,1) in t steps: every step along
    (1,1,1).  So the population there is C[d,n] C[d,d]^(t-1) exactly (the
    light-front spike of Sec. 5.4)."""
    mat = _mat(10.0, 0.01, 0.9)
    med = W.homogeneous(12, mat)
    A = orc.Matrix(med)
    C = orc.collision_block(mat.mu_s, mat.mu_a, mat.g, med.h_mm)
    n = DIR[(0, 0, 1)]
    d = DIR[(1, 1, 1)]
    x0 = np.zeros(A.n_states)
    c = 2
    x0[26 * (c + 12 * (c + 12 * c)) + n] = 1.0
    for t in range(1, 9):
        r = A.run(t, x0=x0)
        p = c + t
        got = math.ldexp(r["x"][26 * (p + 12 * (p + 12 * p)) + d], r["x_exp"])
        want = C[d, n]
        for _ in range(t - 1):
            want = want * C[d, d]
        assert got == pytest.approx(want, rel=1e-15)


def test_angular_marginal_is_block_power(orc):
    """Before anything reaches a face, summing over voxels leaves the pure
    direction dynamics: sum_v J_t[v, :] = C^t J_0[v0, :]."""
    mat = _mat(10.0, 0.05, 0.7)
    med = W.homogeneous(11, mat)
    A = orc.Matrix(med)
    C = orc.collision_block(mat.mu_s, mat.mu_a, mat.g, med.h_mm)
    x0 = np.zeros(A.n_states)
    v0 = 5 + 11 * (5 + 11 * 5)
    j0 = W.seeded_state(26, 4)
    x0[26 * v0: 26 * v0 + 26] = j0
    for t in (1, 3, 5):
        r = A.run(t, x0=x0)
        marg = np.ldexp(r["x"], r["x_exp"]).reshape(-1, 26).sum(axis=0)
        want = np.linalg.matrix_power(C, t) @ j0
        assert np.allclose(marg, want, rtol=1e-13, atol=0)
        assert r["tot"][-1, 1] == 0.0


def test_energy_balance(orc):
    """N(t+1) = N(t) - absorbed(t) - escaped(t) + source(t), every step."""
    w = W.c2(n=15, n_steps=40)
    A = orc.Matrix(w.medium)
    from oracle import run_workload, source_arrays
    r = run_workload(A, w)
    tot = np.ldexp(r["tot"], r["tot_exp"])
    _, _, sw, amp = source_arrays(A, w)
    S = amp[:, 0] * sw.sum()
    Nprev = np.concatenate([[0.0], tot[:-1, 0]])
    bal = Nprev - tot[:, 2] - tot[:, 1] + S
    assert np.allclose(tot[:, 0], bal, rtol=1e-12, atol=1e-16)
    assert tot[-1, 1] > 0 and tot[-1, 2] > 0


def test_square_symmetry(orc):
    """Odd grid, centred +z source, homogeneous: the state is invariant under
    the 8 symmetries of the square in the xy plane."""
    n = 7
    med = W.homogeneous(n, _mat(10.0, 0.05, 0.8))
    A = orc.Matrix(med)
    x0 = np.zeros(A.n_states)
    c = 3
    x0[26 * (c + n * (c + n * 1)) + DIR[(0, 0, 1)]] = 1.0
    r = A.run(6, x0=x0)
    J = np.ldexp(r["x"], r["x_exp"]).reshape(n, n, n, 26)   # [z, y, x, d]
    maps = [lambda a, b: (a, b), lambda a, b: (-a, b), lambda a, b: (a, -b), lambda a, b: (-a, -b),
            lambda a, b: (b, a), lambda a, b: (-b, a), lambda a, b: (b, -a), lambda a, b: (-b, -a)]
    for f in maps:
        perm = [DIR[(*f(e[0], e[1]), e[2])] for e in LV]
        K = np.empty_like(J)
        for yy in range(n):
            for xx in range(n):
                ax, ay = f(xx - c, yy - c)
                K[:, ay + c, ax + c, :][:, perm] = J[:, yy, xx, :]
        assert np.allclose(K, J, rtol=1e-12, atol=1e-300)


def test_superposition(orc):
    """The step is linear in the source (Eq. (26)): run(s1 + s2) = run(s1) + run(s2)."""
    med = W.layered(9, W.C2_MATS)
    A = orc.Matrix(med)
    r1 = [int(s) for s in (26 * 40 + 21, 26 * 300 + 5)]
    amp = np.zeros((25, 2))
    amp[0, 0], amp[3, 1], amp[7, 1] = 1.0, 0.5, 0.25
    a = A.run(25, [r1[0]], [0], [1.0], amp)
    b = A.run(25, [r1[1]], [1], [1.0], amp)
    ab = A.run(25, r1, [0, 1], [1.0, 1.0], amp)
    X = lambda r: np.ldexp(r["x"], r["x_exp"])
    assert np.allclose(X(ab), X(a) + X(b), rtol=1e-12, atol=1e-300)
    T = lambda r: np.ldexp(r["tot"], r["tot_exp"])
    assert np.allclose(T(ab), T(a) + T(b), rtol=1e-12, atol=1e-300)


def test_irreducible(orc):
    """A is irreducible on a connected volume (Sec. 3, Eq. (25)) over the
    states that photons can enter.  On the lattice a face voxel's state whose
    upstream voxel lies outside the grid can be entered only by a wall
    reflection; with vacuum faces, or where no reflected direction equals it
    (edges and corners), its row is empty and only a source can fill it."""
    from scipy.sparse.csgraph import connected_components
    cases = [(W.homogeneous(3, _mat(10.0, 0.1, 0.9), bc="reflect"), False),
             (W.layered(4, [_mat(5, 0.1, 0.8, 1.33), _mat(15, 0.2, 0.9, 1.45),
                            _mat(10, 0.1, 0.0, 1.4)], bc="reflect"), False),
             (W.homogeneous(4, _mat(2.0, 0.1, 0.0), bc="vacuum"), True)]
    for med, vacuum in cases:
        A = orc.Matrix(med)
        x, y, z = _coords(med)
        empty = np.diff(A.row_ptr[: A.n_states + 1]) == 0
        for d, e in enumerate(LV):
            ux, uy, uz = x - e[0], y - e[1], z - e[2]
            outside = ((ux < 0) | (ux >= med.nx) | (uy < 0) | (uy >= med.ny)
                       | (uz < 0) | (uz >= med.nz))
            col = empty.reshape(-1, 26)[:, d]
            assert not np.any(col & ~outside)
            if vacuum:
                assert np.array_equal(col, outside)
        S = A.to_scipy()[: A.n_states]
        live = np.flatnonzero(~empty)
        k, _ = connected_components(S[live][:, live], directed=True, connection="strong")
        assert k == 1


# ---- sizes --------------------------------------------------------------------

def _escape_count(n):
    return 6 * (n ** 3 - (n - 1) * n * n) + 12 * (n ** 3 - (n - 1) ** 2 * n) + 8 * (n ** 3 - (n - 1) ** 3)


@pytest.mark.parametrize("n", [5, 16])
def test_sizes_of_homogeneous_vacuum_cube(orc, n):
    """Every column has 26 entries (one per collision direction, all to different
    rows), and escape rows count the (voxel, direction) pairs that leave."""
    A = orc.Matrix(W.homogeneous(n, _mat(10.0, 0.01, 0.9)))
    assert A.n_escape == _escape_count(n)
    assert A.nnz == 26 * A.n_states
    if n == 16:
        assert (A.n_states, A.nnz, A.n_escape) == (106496, 2768896, 13256)


def test_thread_count_does_not_change_results(orc):
    """The oracle's thread count (used only to time it on one core) leaves every
    row's sequential sum, and so every state and series value, unchanged."""
    wl = W.c2(n=10, n_steps=12)
    A = orc.Matrix(wl.medium)
    try:
        orc.set_threads(1)
        one = orc.run_workload(A, wl)
        orc.set_threads(4)
        four = orc.run_workload(A, wl)
    finally:
        orc.set_threads(os.cpu_count() or 1)
    for k in ("x", "x_exp", "tot", "tot_exp", "det", "det_exp"):
        assert np.array_equal(one[k], four[k]), k


# ---- detectors, Eq. (27) with a one-step window ---------------------------------

def _face_partition_detectors(med):
    """Six detectors that split the escape rows: each (voxel, direction) that
    leaves the grid belongs to the first face it crosses in the order
    -x, +x, -y, +y, -z, +z."""
    x, y, z = _coords(med)
    vox = np.stack([x, y, z], axis=1)
    dims = (med.nx, med.ny, med.nz)
    parts = [[] for _ in range(6)]
    for d, e in enumerate(LV):
        out_lo = [(vox[:, a] + e[a] < 0) for a in range(3)]
        out_hi = [(vox[:, a] + e[a] >= dims[a]) for a in range(3)]
        taken = np.zeros(len(vox), dtype=bool)
        for a in range(3):
            for k, out in ((2 * a, out_lo[a]), (2 * a + 1, out_hi[a])):
                sel = out & ~taken
                for v in np.flatnonzero(sel):
                    parts[k].append((v, d))
                taken |= out
    dets = []
    for k in range(6):
        vs = np.array([p[0] for p in parts[k]], dtype=np.int64)
        ds = np.array([p[1] for p in parts[k]], dtype=np.int64)
        dets.append(W.Detector(vox[vs], LV[ds], np.ones(len(vs), dtype=bool), np.ones(len(vs)), "face%d" % k))
    return dets


def test_face_detectors_partition_escaped(orc):
    """Detectors over a partition of the escape rows add up to the escaped
    total of every step (the detector sums are linear in J, Eq. (27)); a
    layered scattering medium with Fresnel interfaces and a Gaussian source."""
    base = W.c2(n=9, n_steps=30)
    dets = _face_partition_detectors(base.medium)
    wl = W.Workload("parts", base.medium, base.sources, dets, 30)
    A = orc.Matrix(wl.medium)
    assert sum(len(d.F) for d in dets) == A.n_escape
    r = orc.run_workload(A, wl)
    det = np.ldexp(r["det"], r["det_exp"])
    esc = np.ldexp(r["tot"][:, 1], r["tot_exp"][:, 1])
    assert np.all(esc[3:] > 0)
    assert np.allclose(det.sum(axis=1), esc, rtol=1e-13, atol=0)
    assert np.all(det[-1] > 0)


def _ballistic_states(med, x0, t):
    """Closed form of the state after t steps with mu_s = mu_a = 0 (Eq. (11)):
    every population moves one voxel per step along its own direction."""
    x, y, z = _coords(med)
    xs = x0.reshape(-1, 26)
    out = np.zeros_like(xs)
    for d, e in enumerate(LV):
        sx, sy, sz = x - t * e[0], y - t * e[1], z - t * e[2]
        ok = (sx >= 0) & (sx < med.nx) & (sy >= 0) & (sy < med.ny) & (sz >= 0) & (sz < med.nz)
        src = sx + med.nx * (sy + med.ny * sz)
        out[ok, d] = xs[src[ok], d]
    return out


def test_detectors_ballistic_closed_form(orc):
    """mu_s = mu_a = 0: a detector on the escape rows of the z = 0 face reads,
    during step t, the weighted populations of the plane z = 0 that move
    towards -z in the state entering the step; a detector on states reads the
    state after the step.  Weights are drawn per entry, so a dropped or
    misplaced weight fails, and doubling every weight doubles the reading."""
    med = W.homogeneous(6, _mat(0.0, 0.0, 0.9), ny=5, nz=7)
    A = orc.Matrix(med)
    rng = np.random.default_rng(27)
    x0 = W.seeded_state(A.n_states, 5) + 0.25
    top = W.face_escape_detector(med, "top")
    top.F = rng.uniform(0.5, 2.0, size=len(top.F))
    sv = rng.integers(1, [med.nx - 1, med.ny - 1, med.nz - 1], size=(40, 3))
    sd = LV[rng.integers(0, 26, size=40)]
    state_det = W.Detector(sv, sd, np.zeros(40, dtype=bool), rng.uniform(0.5, 2.0, size=40), "states")
    wl = W.Workload("ballistic", med, [], [top, state_det], 3)
    dr, di, dF, nd = orc.detector_arrays(A, wl)
    T = 3
    r = A.run(T, det_rows=dr, det_ids=di, det_F=dF, n_det=nd, x0=x0)
    r2 = A.run(T, det_rows=dr, det_ids=di, det_F=2.0 * dF, n_det=nd, x0=x0)
    det = np.ldexp(r["det"], r["det_exp"])
    assert np.array_equal(np.ldexp(r2["det"], r2["det_exp"]), 2.0 * det)
    tv = top.vox[:, 0] + med.nx * (top.vox[:, 1] + med.ny * top.vox[:, 2])
    td = np.array([DIR[tuple(e)] for e in top.dirs])
    svi = sv[:, 0] + med.nx * (sv[:, 1] + med.ny * sv[:, 2])
    sdi = np.array([DIR[tuple(e)] for e in sd])
    for t in range(T):
        xt = _ballistic_states(med, x0, t)
        xt1 = _ballistic_states(med, x0, t + 1)
        want_top = float(np.sum(top.F * xt[tv, td]))
        want_st = float(np.sum(state_det.F * xt1[svi, sdi]))
        assert want_top > 0 and want_st > 0
        assert det[t, 0] == pytest.approx(want_top, rel=1e-14)
        assert det[t, 1] == pytest.approx(want_st, rel=1e-14)


# ---- sphere interfaces: the normal of a crossing (Sec. 4.2) --------------------

def test_sphere_normal_at_step_midpoint(orc):
    """The normal of a crossing is the sphere's radial direction at the midpoint
    of the two voxel centres.  The sphere is placed so that this direction is
    (1,1,0)/sqrt(2) for the +x move out of voxel (3,3,3): the incidence is
    45 degrees, the specular direction is exactly -y, and the reflected
    fraction is the textbook Fresnel value at 45 degrees (at the voxel centre
    the radial direction would be far more oblique, beyond the critical angle)."""
    inc, bg = _mat(0.0, 0.0, 0.9, 1.45), _mat(0.0, 0.0, 0.9, 1.33)
    c = (4.0 - 0.8, 3.5 - 0.8, 3.5)
    med = W.sphere_inclusion(7, bg, inc, c, 1.2)
    v = 3 + 7 * (3 + 7 * 3)
    u = 4 + 7 * (3 + 7 * 3)
    assert med.mat_of_voxel.reshape(-1)[v] == 1 and med.mat_of_voxel.reshape(-1)[u] == 0
    A = orc.Matrix(med)
    S = A.to_scipy().tocsc()
    col = 26 * v + DIR[(1, 0, 0)]
    rows = S.indices[S.indptr[col]:S.indptr[col + 1]]
    vals = S.data[S.indptr[col]:S.indptr[col + 1]]
    entry = dict(zip(rows.tolist(), vals.tolist()))
    ti = math.pi / 4
    tt = math.asin(1.45 / 1.33 * math.sin(ti))
    Rs = math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2
    Rp = math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2
    R = 0.5 * (Rs + Rp)
    assert entry[26 * v + DIR[(0, -1, 0)]] == pytest.approx(R, rel=1e-12)
    assert len(entry) == 2
    (rt, T), = [(k, w) for k, w in entry.items() if k != 26 * v + DIR[(0, -1, 0)]]
    assert rt // 26 == u and T == pytest.approx(1.0 - R, rel=1e-14)


def test_square_symmetry_centred_sphere(orc):
    """A sphere centred on the middle voxel's column of an odd grid, with a
    centred +z source and a contrast that reaches total internal reflection:
    the state is invariant under the 8 symmetries of the square in the xy
    plane (a normal rule that did not commute with them would break it)."""
    n, c = 9, 4
    bg, inc = _mat(10.0, 0.05, 0.8, 1.0), _mat(6.0, 0.2, 0.5, 1.6)
    med = W.sphere_inclusion(n, bg, inc, (4.5, 4.5, 4.0), 2.6)
    A = orc.Matrix(med)
    x0 = np.zeros(A.n_states)
    x0[26 * (c + n * (c + n * 1)) + DIR[(0, 0, 1)]] = 1.0
    r = A.run(7, x0=x0)
    J = np.ldexp(r["x"], r["x_exp"]).reshape(n, n, n, 26)
    maps = [lambda a, b: (a, b), lambda a, b: (-a, b), lambda a, b: (a, -b), lambda a, b: (-a, -b),
            lambda a, b: (b, a), lambda a, b: (-b, a), lambda a, b: (b, -a), lambda a, b: (-b, -a)]
    R, _, _, _ = orc.fresnel(DIR[(1, 1, 1)], 1.6, 1.0, np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0))
    assert R < 1.0
    for f in maps:
        perm = [DIR[(*f(e[0], e[1]), e[2])] for e in LV]
        K = np.empty_like(J)
        for yy in range(n):
            for xx in range(n):
                ax, ay = f(xx - c, yy - c)
                K[:, ay + c, ax + c, :][:, perm] = J[:, yy, xx, :]
        assert np.allclose(K, J, rtol=1e-12, atol=1e-300)


# ---- the dither rounding's key, written out from its definition -----------------

def _splitmix64(x):
    m = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def test_dither_decisions_follow_the_row_column_key(orc):
    """Every FP32 value of the dithered matrix, derived here from the rounding
    rule: r = RN32(a), r' = the other float neighbour of a, p = |r - a|/|r' - r|,
    u = (splitmix64((row << 32) xor col) >> 11) 2^-53, take r' iff u < p."""
    A = orc.Matrix(W.layered(4, W.C2_MATS))
    got = A.round_f32("dither")
    rp, col, val = A.row_ptr, A.col, A.val
    n_taken = 0
    for row in range(A.n_rows):
        for j in range(rp[row], rp[row + 1]):
            a = float(val[j])
            r = np.float32(a)
            want = r
            if float(r) != a:
                r2 = np.nextafter(r, np.float32(np.inf) if float(r) < a else np.float32(-np.inf))
                p = abs(float(r) - a) / abs(float(r2) - float(r))
                u = (_splitmix64((row << 32) ^ int(col[j])) >> 11) * 2.0 ** -53
                if u < p:
                    want = r2
                    n_taken += 1
            assert got[j] == want, (row, int(col[j]))
    assert n_taken > 100


# ---- several scatterings within one step (Eq. (4)-(5)) ---------------------------

def _single_scatter_kernel(orc, mu_s, g, h):
    """The discrete scattering kernel G recovered from the single-scatter block
    (pinned above against the Henyey-Greenstein form): C1 = P0 I + (1 - P0) G
    without absorption."""
    C1 = orc.collision_block(mu_s, 0.0, g, h)
    P0 = math.exp(-mu_s * h)
    return (C1 - P0 * np.eye(26)) / (1.0 - P0)


@pytest.mark.parametrize("K", [2, 3, 5, 9])
def test_higher_order_block_columns_sum_to_survival(orc, K):
    """Every order keeps the column sums at exp(-mu_a c dt) (Eq. (24))."""
    for mu_s, mu_a, g in [(10, 0.01, 0.9), (20, 0.1, 0.7), (3, 0.5, 0.0)]:
        C = orc.collision_block(mu_s, mu_a, g, 0.1, order=K)
        assert np.allclose(C.sum(axis=0), math.exp(-mu_a * 0.1), rtol=0, atol=40 * 2.3e-16)
        assert np.all(C >= 0)


def test_higher_order_isotropic_equals_single_scatter(orc):
    """g = 0: one scatter already spreads uniformly (G^i = G), so every order
    gives the single-scatter block."""
    C1 = orc.collision_block(15.0, 0.2, 0.0, 0.1)
    for K in (2, 4, 7):
        assert np.allclose(orc.collision_block(15.0, 0.2, 0.0, 0.1, order=K), C1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("mu_s,g", [(10.0, 0.9), (20.0, 0.7), (5.0, 0.3)])
def test_high_order_limit_is_the_matrix_exponential(orc, mu_s, g):
    """Poisson-weighted powers of the kernel sum to exp(lambda (G - I)) with
    lambda = mu_s c dt (a continuous-time Markov chain over directions,
    scatterings at rate mu_s c): at order 16 the omitted tail is below 1e-13."""
    from scipy.linalg import expm
    h, mu_a = 0.1, 0.03
    G = _single_scatter_kernel(orc, mu_s, g, h)
    lam = mu_s * h
    want = math.exp(-mu_a * h) * expm(lam * (G - np.eye(26)))
    got = orc.collision_block(mu_s, mu_a, g, h, order=16)
    assert np.allclose(got, want, rtol=0, atol=2e-13)
    # order 2 is the two-scatter truncation: P0 I + P1 G + (1 - P0 - P1) G^2
    P0, P1 = math.exp(-lam), math.exp(-lam) * lam
    want2 = math.exp(-mu_a * h) * (P0 * np.eye(26) + P1 * G + (1 - P0 - P1) * (G @ G))
    assert np.allclose(orc.collision_block(mu_s, mu_a, g, h, order=2), want2, rtol=0, atol=1e-14)


def test_higher_order_medium_steps_with_its_block(orc):
    """A medium of scatter order 3: before anything reaches a face, the angular
    marginal follows the order-3 block, sum_v J_t = C3^t J_0."""
    mat = _mat(20.0, 0.05, 0.8)
    med = W.homogeneous(11, mat)
    med.scatter_order = 3
    A = orc.Matrix(med)
    C3 = orc.collision_block(mat.mu_s, mat.mu_a, mat.g, med.h_mm, order=3)
    assert not np.allclose(C3, orc.collision_block(mat.mu_s, mat.mu_a, mat.g, med.h_mm), rtol=1e-6)
    x0 = np.zeros(A.n_states)
    v0 = 5 + 11 * (5 + 11 * 5)
    j0 = W.seeded_state(26, 6)
    x0[26 * v0: 26 * v0 + 26] = j0
    for t in (1, 4):
        r = A.run(t, x0=x0)
        marg = np.ldexp(r["x"], r["x_exp"]).reshape(-1, 26).sum(axis=0)
        assert np.allclose(marg, np.linalg.matrix_power(C3, t) @ j0, rtol=1e-13, atol=0)


# ---- windowed measurement and outside sensors (Eq. (27), Sec. 4.2) ---------------

def test_window_of_a_ballistic_impulse_is_the_sensor_response(orc):
    """mu_s = mu_a = 0: one photon moving -z from depth z0 leaves through the
    z = 0 face during step z0 exactly, so the one-step detector is a unit
    impulse at z0 and a sensor reading is its impulse response, delayed:
    M(t) = h(t - z0 - tap0)."""
    med = W.homogeneous(5, _mat(0.0, 0.0, 0.9), nz=9)
    A = orc.Matrix(med)
    z0 = 6
    x0 = np.zeros(A.n_states)
    x0[26 * (2 + 5 * (2 + 5 * z0)) + DIR[(0, 0, -1)]] = 1.0
    top = W.face_escape_detector(med, "top")
    wl = W.Workload("imp", med, [], [top], 20)
    dr, di, dF, nd = orc.detector_arrays(A, wl)
    r = A.run(20, det_rows=dr, det_ids=di, det_F=dF, n_det=nd, x0=x0)
    m = np.ldexp(r["det"][:, 0], r["det_exp"][:, 0])
    assert m[z0] == 1.0 and np.count_nonzero(m) == 1
    h = np.array([0.1, 0.5, 0.25, 0.125, 0.0625])
    for tap0 in (0, 2, -3):
        M = orc.window(r["det"], r["det_exp"], h[None, :], tap0)[:, 0]
        want = np.zeros(20)
        for j, hj in enumerate(h):
            if 0 <= z0 + tap0 + j < 20:
                want[z0 + tap0 + j] = hj
        assert np.array_equal(M, want), tap0


def test_window_over_the_whole_run_balances_energy(orc):
    """A sensor that integrates every step (all-ones response) over all escape
    rows reads the photons that have left by step t; with those absorbed and
    those still inside it accounts for everything emitted (Eq. (24), Sec. 3)."""
    base = W.c2(n=8, n_steps=40)
    dets = _face_partition_detectors(base.medium)
    wl = W.Workload("parts", base.medium, base.sources, dets, 40)
    A = orc.Matrix(wl.medium)
    r = orc.run_workload(A, wl)
    T = 40
    M = orc.window(r["det"], r["det_exp"], np.ones((6, T)), 0)
    escaped_by_t = M.sum(axis=1)
    tot = np.ldexp(r["tot"], r["tot_exp"])
    absorbed_by_t = np.cumsum(tot[:, 2])
    _, _, sw, amp = orc.source_arrays(A, wl)
    emitted_by_t = np.cumsum(amp[:T, 0]) * sw.sum()
    assert np.allclose(escaped_by_t + absorbed_by_t + tot[:, 0], emitted_by_t, rtol=1e-12, atol=0)


def test_outside_sensor_reads_the_delayed_escape_flux(orc):
    """Free space added above the surface (Sec. 4.2: no scattering or
    absorption, photons keep their direction): a sensor on the top face of
    the extension reads, gap steps later, the photons that left the original
    surface in directions that keep them over the sensor for gap steps."""
    gap, T = 3, 30
    base = W.c2(n=9, n_steps=T)
    med = base.medium
    ext = W.extend_top(med, gap)
    assert ext.mat_of_voxel[gap:].min() >= 1 and (ext.mat_of_voxel[:gap] == 0).all()
    # the sensor: escape rows of the extension's top face
    sensor = W.face_escape_detector(ext, "top")
    we = W.Workload("ext", ext, [W.shifted_z(s, gap) for s in base.sources], [sensor], T)
    # on the original: its top-face escapes weighted by whether the photon stays
    # over the sensor for gap steps
    top = W.face_escape_detector(med, "top")
    end = top.vox[:, :2] + gap * top.dirs[:, :2]
    top.F = (((end >= 0) & (end < np.array([med.nx, med.ny]))).all(axis=1)).astype(np.float64)
    wo = W.Workload("orig", med, base.sources, [top], T)
    re = orc.run_workload(orc.Matrix(ext), we)
    ro = orc.run_workload(orc.Matrix(med), wo)
    se = np.ldexp(re["det"][:, 0], re["det_exp"][:, 0])
    so = np.ldexp(ro["det"][:, 0], ro["det_exp"][:, 0])
    assert np.all(se[:gap] == 0)
    assert so[3:].max() > 0
    assert np.allclose(se[gap:], so[:T - gap], rtol=1e-12, atol=1e-300)


# ---- crossing an interface within the step (Sec. 4.2) ------------------------------

def test_substep_layers_path_absorption_and_tangential_landing(orc):
    """Planar interface, mu_s = 0: a population in direction (1, 0, 1) meets
    the interface half way through the step.  The transmitted part is absorbed
    over half a step in each medium, exp(-mu_a1 h/2 - mu_a2 h/2) T; the
    reflected part returns for the other half step along (1, 0, -1) and lands
    in the voxel one over along the surface, (x + 1, y, z), with R (textbook
    Fresnel at 45 degrees, the specular direction exact)."""
    h = 0.1
    m1, m2 = _mat(0.0, 0.3, 0.5, 1.33), _mat(0.0, 2.0, 0.5, 1.45)
    med = W.layered(6, [m1, m2])
    med.interface = "substep"
    A = orc.Matrix(med).to_scipy().tocsc()
    x, y, z = 2, 2, 2                      # layer 0 is z < 3
    v = x + 6 * (y + 6 * z)
    col = 26 * v + DIR[(1, 0, 1)]
    ent = dict(zip(A.indices[A.indptr[col]:A.indptr[col + 1]].tolist(), A.data[A.indptr[col]:A.indptr[col + 1]].tolist()))
    ti = math.pi / 4
    tt = math.asin(1.33 / 1.45 * math.sin(ti))
    R = 0.5 * (math.sin(ti - tt) ** 2 / math.sin(ti + tt) ** 2 + math.tan(ti - tt) ** 2 / math.tan(ti + tt) ** 2)
    a1 = math.exp(-0.3 * h)
    vr = (x + 1) + 6 * (y + 6 * z)
    u = (x + 1) + 6 * (y + 6 * (z + 1))
    assert ent[26 * vr + DIR[(1, 0, -1)]] == pytest.approx(a1 * R, rel=1e-12)
    assert ent[26 * u + DIR[(1, 0, 1)]] == pytest.approx(math.exp(-0.3 * h / 2 - 2.0 * h / 2) * (1 - R), rel=1e-12)
    assert len(ent) == 2
    # normal incidence: no tangential move
    col = 26 * v + DIR[(0, 0, 1)]
    rows = A.indices[A.indptr[col]:A.indptr[col + 1]].tolist()
    assert 26 * v + DIR[(0, 0, -1)] in rows


def test_substep_sphere_crossing_point(orc):
    """Sphere: the crossing lies where the segment between the voxel centres
    meets the surface.  Centre and radius put it 0.3 of the way along +x from
    voxel (3,3,3), at normal incidence: the transmitted entry is
    exp(-0.3 mu_a1 h - 0.7 mu_a2 h) (1 - R0), R0 = ((n1 - n2)/(n1 + n2))^2."""
    h = 0.1
    inc, bg = _mat(0.0, 0.5, 0.5, 1.45), _mat(0.0, 0.05, 0.5, 1.33)
    d = 1.2
    med = W.sphere_inclusion(7, bg, inc, (3.5 - d, 3.5, 3.5), d + 0.3)
    med.interface = "substep"
    v = 3 + 7 * (3 + 7 * 3)
    u = 4 + 7 * (3 + 7 * 3)
    assert med.mat_of_voxel.reshape(-1)[v] == 1 and med.mat_of_voxel.reshape(-1)[u] == 0
    A = orc.Matrix(med).to_scipy().tocsc()
    col = 26 * v + DIR[(1, 0, 0)]
    ent = dict(zip(A.indices[A.indptr[col]:A.indptr[col + 1]].tolist(), A.data[A.indptr[col]:A.indptr[col + 1]].tolist()))
    R0 = ((1.45 - 1.33) / (1.45 + 1.33)) ** 2
    assert ent[26 * u + DIR[(1, 0, 0)]] == pytest.approx(math.exp(-0.5 * 0.3 * h - 0.05 * 0.7 * h) * (1 - R0),
                                                         rel=1e-12)
    assert ent[26 * v + DIR[(-1, 0, 0)]] == pytest.approx(math.exp(-0.5 * h) * R0, rel=1e-12)


def test_substep_conserves_without_absorption(orc):
    """mu_a = 0 with reflecting walls: the sub-step crossing moves photons, it
    neither creates nor destroys them (columns sum to one, the total stays)."""
    mats = [_mat(5, 0, 0.8, 1.33), _mat(15, 0, 0.9, 1.45), _mat(10, 0, 0.85, 1.4)]
    med = W.layered(6, mats, bc="reflect")
    med.interface = "substep"
    A = orc.Matrix(med)
    colsum = np.asarray(A.to_scipy().sum(axis=0)).ravel()
    assert np.allclose(colsum, 1.0, rtol=0, atol=30 * 1.2e-16)
    x0 = W.seeded_state(A.n_states, 7)
    r = A.run(40, x0=x0)
    assert np.allclose(np.ldexp(r["tot"][:, 0], r["tot_exp"][:, 0]), x0.sum(), rtol=1e-12)


def test_substep_equals_origin_model_without_absorption_contrast(orc):
    """Equal absorption on both sides and normal incidence only (a 1-voxel-wide
    column along z): the sub-step model changes nothing."""
    m1, m2 = _mat(5.0, 0.2, 0.8, 1.33), _mat(5.0, 0.2, 0.8, 1.45)
    med = W.layered(4, [m1, m2])
    med = W.Medium(1, 1, 4, 0.1, med.materials, med.mat_of_voxel[:, :1, :1].copy(), "layers_z", "vacuum",
                   layer_z0=med.layer_z0)
    a = orc.Matrix(med).to_scipy().toarray()
    med.interface = "substep"
    b = orc.Matrix(med).to_scipy().toarray()
    assert np.array_equal(a, b)
