"""Pins of the oracle's Lebedev-86 discretisation (Sec. 3, Eq. (18)-(21))
against what the quadrature rule, geometry and the mathematics fix: exact
integration of spherical monomials, the octahedral symmetry of the rule,
weights that are normalised distance ramps over the voxels near each arrival
segment, an exact one-voxel shift for the axis directions, column sums,
the Henyey-Greenstein ratios of the discrete kernel, the xy-square symmetry
of a centred source, energy balance, and a second construction of the whole
matrix in numpy (pull-style, per direction pair, vectorised over voxels)."""
import math

import numpy as np
import pytest

import workloads as W

N_DIR = 86


def _lebedev_medium(n, mat, c_dt=1.0, **kw):
    med = W.homogeneous(n, mat, **kw)
    med.directions = "lebedev86"
    med.c_dt = c_dt
    return med


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


def test_rule_integrates_monomials_to_degree_15(orc):
    """Average of x^a y^b z^c over the sphere: (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!!
    for even exponents, 0 otherwise; exact up to degree 15, not at 16."""
    S, w = orc.lebedev86()
    assert S.shape == (86, 3) and np.all(w > 0)
    assert np.allclose(np.linalg.norm(S, axis=1), 1.0, rtol=0, atol=1e-15)
    assert len(set(map(tuple, np.round(S, 12)))) == 86
    worst = 0.0
    for a in range(16):
        for b in range(16 - a):
            for c in range(16 - a - b):
                q = float((w * S[:, 0] ** a * S[:, 1] ** b * S[:, 2] ** c).sum())
                ex = 0.0 if (a % 2 or b % 2 or c % 2) else _dfact(a - 1) * _dfact(b - 1) * _dfact(c - 1) / _dfact(a + b + c + 1)
                worst = max(worst, abs(q - ex))
    assert worst < 5e-15
    assert abs(float((w * S[:, 0] ** 16).sum()) - _dfact(15) / _dfact(17)) > 1e-6
    # ordered by ascending z, then y, then x
    keys = [tuple(s[::-1]) for s in S]
    assert keys == sorted(keys)


def test_rule_has_octahedral_symmetry(orc):
    """Coordinate permutations and sign changes map the rule onto itself,
    weights included."""
    S, w = orc.lebedev86()
    lookup = {tuple(np.round(s, 12)): wi for s, wi in zip(S, w)}
    for perm in ((0, 1, 2), (1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)):
        for sg in ((1, 1, 1), (-1, 1, 1), (1, -1, -1), (-1, -1, 1)):
            for s, wi in zip(S, w):
                t = tuple(np.round(np.array(sg) * s[list(perm)], 12) + 0.0)
                assert t in lookup and abs(lookup[t] - wi) < 1e-17


def _seg_dist(P, a, b):
    """Textbook distance from points P [k, 3] to the segment ab."""
    ab = b - a
    L2 = ab @ ab
    t = np.zeros(len(P)) if L2 == 0 else np.clip((P - a) @ ab / L2, 0.0, 1.0)
    return np.linalg.norm(P - (a + t[:, None] * ab), axis=1)


def test_stencils_are_normalised_ramps_over_nearby_voxels(orc):
    """Eq. (18)-(19) with 2 dr = one voxel: for each direction pair the
    offsets are exactly the lattice points closer than one voxel to the
    segment from c dt S_m to c dt S_n, their weights are proportional to
    1 - distance and sum to one."""
    S, _ = orc.lebedev86()
    for c in (1.0, 0.6):
        R = orc.LebedevRows(_lebedev_medium(4, W.Material(5.0, 0.1, 0.8, 1.4), c_dt=c))
        box = np.array([(x, y, z) for z in range(-3, 4) for y in range(-3, 4) for x in range(-3, 4)], float)
        rng = np.random.default_rng(18)
        pairs = [(m, m) for m in range(0, 86, 7)] + [tuple(p) for p in rng.integers(0, 86, size=(60, 2))]
        for m, n in pairs:
            off, w = R.stencil(m, n)
            d = _seg_dist(box, c * S[m], c * S[n])
            want = box[d < 1.0]
            assert sorted(map(tuple, off.astype(float))) == sorted(map(tuple, want)), (m, n)
            dd = _seg_dist(off.astype(float), c * S[m], c * S[n])
            assert np.allclose(w, (1 - dd) / (1 - dd).sum(), rtol=1e-13, atol=0)
            assert abs(w.sum() - 1.0) < 1e-14 and np.all(w > 0)
        R.close()


def test_axis_directions_shift_one_voxel(orc):
    """mu_s = mu_a = 0, c dt = one voxel: B = X_i + h S_n is a voxel centre for
    the six axis directions, and no other centre is closer than one voxel, so
    those populations move exactly one voxel per step (Eq. (11), (18))."""
    med = _lebedev_medium(5, W.Material(0.0, 0.0, 0.5, 1.4))
    A = orc.Matrix(med)
    S, _ = orc.lebedev86()
    axis = [int(np.argmax(S @ np.array(e, float))) for e in
            ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
    x0 = np.zeros(A.n_states)
    rng = np.random.default_rng(11)
    for d in axis:
        x0[N_DIR * np.arange(125) + d] = rng.random(125) + 0.5
    for t in (1, 2):
        r = A.run(t, x0=x0)
        got = np.ldexp(r["x"], r["x_exp"]).reshape(5, 5, 5, N_DIR)
        J0 = x0.reshape(5, 5, 5, N_DIR)
        for d, e in zip(axis, ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))):
            want = np.zeros((5, 5, 5))
            ex, ey, ez = e[0] * t, e[1] * t, e[2] * t
            src = J0[max(0, -ez):5 - max(0, ez), max(0, -ey):5 - max(0, ey), max(0, -ex):5 - max(0, ex), d]
            want[max(0, ez):5 - max(0, -ez), max(0, ey):5 - max(0, -ey), max(0, ex):5 - max(0, -ex)] = src
            assert np.array_equal(got[..., d], want), (d, t)


def test_columns_sum_to_survival(orc):
    """Every column of [A; L] sums to exp(-mu_a c dt) (Eq. (24)): the weights of
    a direction pair sum to one and the direction block's columns to alpha."""
    for mat, c in ((W.Material(10.0, 0.01, 0.9, 1.4), 1.0), (W.Material(3.0, 0.5, 0.3, 1.4), 0.7)):
        med = _lebedev_medium(4, mat, c_dt=c, ny=3, nz=5)
        A = orc.Matrix(med)
        cs = np.asarray(A.to_scipy().sum(axis=0)).ravel()
        alpha = math.exp(-mat.mu_a * c * med.h_mm)
        assert np.allclose(cs, alpha, rtol=0, atol=2e-14)
        assert np.all(A.val > 0) and np.all(A.val <= 1)


def test_kernel_isotropic_and_henyey_greenstein_ratios(orc):
    """g = 0: a scatter picks direction m with probability w_m (the rule's
    weight of its solid angle).  g != 0: within a column, entries are in the
    ratio w_m1 p(cos_1) / (w_m2 p(cos_2)) of the Henyey-Greenstein form."""
    S, w = orc.lebedev86()
    h = 0.1
    R = orc.LebedevRows(_lebedev_medium(3, W.Material(4.0, 0.2, 0.0, 1.4)))
    C = R.block(0)
    P0, alpha = math.exp(-4.0 * h), math.exp(-0.2 * h)
    off = ~np.eye(86, dtype=bool)
    assert np.allclose(C[off], (alpha * (1 - P0) * np.repeat(w[:, None], 86, axis=1))[off], rtol=1e-13)
    assert np.allclose(np.diag(C), alpha * (P0 + (1 - P0) * w), rtol=1e-13)
    g = 0.8
    R = orc.LebedevRows(_lebedev_medium(3, W.Material(4.0, 0.2, g, 1.4)))
    C = R.block(0)
    hg = lambda cs: (1 - g * g) / (1 + g * g - 2 * g * cs) ** 1.5
    rng = np.random.default_rng(19)
    for n, m1, m2 in rng.integers(0, 86, size=(40, 3)):
        if len({n, m1, m2}) < 3:
            continue
        want = w[m1] * hg(S[m1] @ S[n]) / (w[m2] * hg(S[m2] @ S[n]))
        assert C[m1, n] / C[m2, n] == pytest.approx(want, rel=1e-12)


def test_square_symmetry_of_centred_source(orc):
    """Odd grid, homogeneous, source at the centre column in +z: the state is
    invariant under the 8 symmetries of the square in the xy plane (the rule
    and the lattice share them)."""
    n, c = 7, 3
    med = _lebedev_medium(n, W.Material(8.0, 0.05, 0.7, 1.4))
    A = orc.Matrix(med)
    S, _ = orc.lebedev86()
    x0 = np.zeros(A.n_states)
    x0[N_DIR * (c + n * (c + n * 1)) + int(np.argmax(S[:, 2]))] = 1.0
    r = A.run(3, x0=x0)
    J = np.ldexp(r["x"], r["x_exp"]).reshape(n, n, n, N_DIR)
    maps = [lambda a, b: (a, b), lambda a, b: (-a, b), lambda a, b: (a, -b), lambda a, b: (-a, -b),
            lambda a, b: (b, a), lambda a, b: (-b, a), lambda a, b: (b, -a), lambda a, b: (-b, -a)]
    for f in maps:
        img = np.array([[*f(s[0], s[1]), s[2]] for s in S])
        perm = [int(np.argmax(S @ t)) for t in img]
        assert sorted(perm) == list(range(86))
        K = np.empty_like(J)
        for yy in range(n):
            for xx in range(n):
                ax, ay = f(xx - c, yy - c)
                K[:, ay + c, ax + c, :][:, perm] = J[:, yy, xx, :]
        assert np.allclose(K, J, rtol=1e-11, atol=1e-18)


def test_energy_balance(orc):
    """N(t+1) = N(t) - absorbed(t) - escaped(t) + source(t) with the 86
    directions (absorbed from the state entering the step)."""
    med = _lebedev_medium(6, W.Material(12.0, 0.3, 0.85, 1.4))
    A = orc.Matrix(med)
    S, _ = orc.lebedev86()
    src = [A.n_dir * (3 + 6 * (3 + 6 * 0)) + int(np.argmax(S[:, 2]))]
    amp = np.zeros((15, 1))
    amp[0, 0], amp[2, 0] = 1.0, 0.5
    r = A.run(15, src, [0], [1.0], amp)
    tot = np.ldexp(r["tot"], r["tot_exp"])
    Nprev = np.concatenate([[0.0], tot[:-1, 0]])
    assert np.allclose(tot[:, 0], Nprev - tot[:, 2] - tot[:, 1] + amp[:, 0], rtol=1e-12, atol=1e-16)
    assert tot[-1, 1] > 0 and tot[-1, 2] > 0


def _pull_numpy(orc, med):
    """[A; L] of a Lebedev medium built pull-style in numpy: for every pair
    (m, n) the stencil from the textbook point-segment distance (offsets in
    ascending (dz, dy, dx), weights 1 - d normalised by their sequential sum),
    then for every voxel i and offset the entry w C[m][n] at row
    (i + offset, m), column (i, n), or the summed outside weights times
    C[m][n] in escape row (i, m)."""
    S, _ = orc.lebedev86()
    C = orc.LebedevRows(med).block(0)
    c = med.c_dt
    R = int(math.ceil(c + 1))
    box = np.array([(x, y, z) for z in range(-R, R + 1) for y in range(-R, R + 1) for x in range(-R, R + 1)],
                   dtype=np.int64)
    nx, ny, nz = med.nx, med.ny, med.nz
    V = nx * ny * nz
    vx, vy, vz = np.arange(V) % nx, (np.arange(V) // nx) % ny, np.arange(V) // (nx * ny)
    rows, cols, vals = [], [], []
    esc = {}
    for m in range(86):
        for n in range(86):
            a, b = c * S[m], c * S[n]
            ab = b - a
            L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]
            P = box.astype(float)
            ap = P - a
            if L2 > 0.0:
                t = (ap[:, 0] * ab[0] + ap[:, 1] * ab[1] + ap[:, 2] * ab[2]) / L2
                t = np.minimum(np.maximum(t, 0.0), 1.0)
            else:
                t = np.zeros(len(P))
            q = a + t[:, None] * ab
            dv = P - q
            d = np.sqrt(dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1] + dv[:, 2] * dv[:, 2])
            keep = np.flatnonzero(d < 1.0)
            raw = 1.0 - d[keep]
            tot = 0.0
            for x in raw:
                tot += x
            w = raw / tot
            cmn = C[m, n]
            for k, o in enumerate(box[keep]):
                ux, uy, uz = vx + o[0], vy + o[1], vz + o[2]
                ins = (ux >= 0) & (ux < nx) & (uy >= 0) & (uy < ny) & (uz >= 0) & (uz < nz)
                u = ux + nx * (uy + ny * uz)
                rows.append(86 * u[ins] + m)
                cols.append(86 * np.arange(V)[ins] + n)
                vals.append(np.full(ins.sum(), w[k] * cmn))
                for i in np.flatnonzero(~ins):
                    esc.setdefault((i, m, n), []).append(w[k])
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), esc, C


def test_push_assembly_equals_numpy_pull(orc):
    """The oracle's push assembly equals an independent pull-style numpy
    construction bit for bit (state rows), and every escape entry equals the
    sequential sum of its outside weights times the block entry."""
    med = _lebedev_medium(3, W.Material(6.0, 0.2, 0.7, 1.4), ny=4, nz=3)
    A = orc.Matrix(med)
    rows, cols, vals, esc, C = _pull_numpy(orc, med)
    S = A.to_scipy().tocoo()
    D = A.n_states
    got = {(int(r), int(c)): v for r, c, v in zip(S.row, S.col, S.data) if r < D}
    want = {(int(r), int(c)): v for r, c, v in zip(rows, cols, vals)}
    assert got.keys() == want.keys()
    assert all(got[k] == want[k] for k in want)
    # escape rows: (v, m) in ascending order, entry per column (v, n)
    pairs = sorted({(i, m) for (i, m, n) in esc})
    assert A.n_escape == len(pairs)
    Sd = A.to_scipy()
    for e, (i, m) in enumerate(pairs):
        row = Sd[D + e]
        for n in range(86):
            ws = esc.get((i, m, n))
            if not ws:
                continue
            acc = 0.0
            for x in ws:
                acc += x
            assert row[0, 86 * i + n] == acc * C[m, n], (i, m, n)


def test_source_steps_follow_the_light_path(orc):
    """A step lasts the time light takes for c dt: with half a voxel per step
    the pulse integrals of Sec. 4.1 are taken over steps half as long, so their
    running sum is the Gaussian's distribution function at (k + 1) dt."""
    from scipy.stats import norm
    med = _lebedev_medium(4, W.Material(10.0, 0.01, 0.9, 1.4), c_dt=0.5)
    src = W.point_source(1, 1, 0, kind="gaussian", fwhm_fs=300.0)
    wl = W.Workload("pulse", med, [src], [], 12, 1, "f32", "dither", 1.4)
    A = orc.Matrix(med)
    _, _, _, amp = orc.source_arrays(A, wl)
    dt = 0.5 * med.h_mm * 1e-3 * 1.4 / 299792458.0
    sig = 300e-15 / (2 * math.sqrt(2 * math.log(2)))
    want = norm.cdf(((np.arange(12) + 1) * dt - 3 * sig) / sig)
    assert np.allclose(np.cumsum(amp[:, 0]), want, rtol=0, atol=1e-13)
