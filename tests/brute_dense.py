"""Pull-style dense construction of the DRTS matrix on tiny grids.

A second, independent construction used only to pin the oracle: the oracle
pushes every column (v, n) to its targets; this module pulls, for every row,
the list of moves (source voxel u, collision direction m, factor f) that
deliver into it, and writes the dense entry
    a[row, 26 u + n] = sum over those moves (ascending u, then m) of f * C_q(u)[m, n]
(Eq. (20)-(21) on the 26-neighbour lattice).  Scalar coefficients use Python's
``math`` (FP64), in the same evaluation order as stated for the method, so
the two constructions must agree bit for bit.
"""
from __future__ import annotations

import math

import numpy as np

LV = []
for _dz in (-1, 0, 1):
    for _dy in (-1, 0, 1):
        for _dx in (-1, 0, 1):
            if _dx or _dy or _dz:
                LV.append((_dx, _dy, _dz))


def unit(d):
    e = LV[d]
    ln = math.sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2])
    return (e[0] / ln, e[1] / ln, e[2] / ln)


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def block(mat, h):
    mu_s, mu_a, g = mat.mu_s, mat.mu_a, mat.g
    P0 = math.exp(-mu_s * h)
    Ps = 1.0 - P0
    alpha = math.exp(-mu_a * h)

    def hg(cs):
        q = 1.0 + g * g - 2.0 * g * cs
        return (1.0 - g * g) / (q * math.sqrt(q))

    p = [[0.0] * 26 for _ in range(26)]
    for m in range(26):
        for n in range(26):
            em, en = LV[m], LV[n]
            d = em[0] * en[0] + em[1] * en[1] + em[2] * en[2]
            nm = em[0] ** 2 + em[1] ** 2 + em[2] ** 2
            nn = en[0] ** 2 + en[1] ** 2 + en[2] ** 2
            p[m][n] = hg(d / math.sqrt(nm * nn))
    C = [[0.0] * 26 for _ in range(26)]
    for n in range(26):
        Z = 0.0
        for k in range(26):
            Z += p[k][n]
        for m in range(26):
            G = p[m][n] / Z
            C[m][n] = alpha * (Ps * G) if m != n else alpha * (P0 + Ps * G)
    return C


def snap(target, N, side):
    """All directions on the requested side whose s_d . target is within 1e-12
    of the largest (tied directions share the population evenly)."""
    vals = {}
    for d in range(26):
        s = unit(d)
        sn = dot(s, N)
        if (side < 0 and sn < 0.0) or (side > 0 and sn > 0.0):
            vals[d] = dot(s, target)
    if not vals:
        return []
    top = max(vals.values())
    return [d for d in sorted(vals) if vals[d] >= top - 1e-12]


def fresnel(m, n1, n2, N):
    s = unit(m)
    ci = dot(s, N)
    eta = n1 / n2
    s2t = eta * eta * (1.0 - ci * ci)
    if s2t >= 1.0:
        R, T, ct = 1.0, 0.0, 0.0
    else:
        ct = math.sqrt(1.0 - s2t)
        rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct)
        rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct)
        R = 0.5 * (rs * rs + rp * rp)
        T = 1.0 - R
    r = [s[i] - (2.0 * ci) * N[i] for i in range(3)]
    t = [eta * s[i] + (ct - eta * ci) * N[i] for i in range(3)]
    return R, T, snap(r, N, -1), (snap(t, N, +1) if T > 0.0 else [])


def normal(med, x, y, z, e, s):
    if med.geom == "layers_z" and e[2] != 0:
        return (0.0, 0.0, 1.0 if e[2] > 0 else -1.0)
    if med.geom == "sphere":
        P = (x + 0.5 + 0.5 * e[0], y + 0.5 + 0.5 * e[1], z + 0.5 + 0.5 * e[2])
        w = [P[i] - med.sphere_c[i] for i in range(3)]
        ln = math.sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2])
        if ln > 0.0:
            N = [w[0] / ln, w[1] / ln, w[2] / ln]
            if dot(s, N) < 0.0:
                N = [-N[0], -N[1], -N[2]]
            return tuple(N)
    return s


def build_dense(med):
    """Dense [n_rows, n_states] matrix, with escape rows after the states."""
    nx, ny, nz = med.nx, med.ny, med.nz
    V = nx * ny * nz
    D = 26 * V
    mat = med.mat_of_voxel.reshape(-1)
    nidx = [m.n for m in med.materials]
    blocks = [block(m, med.h_mm) for m in med.materials]

    def coords(v):
        return v % nx, (v // nx) % ny, v // (nx * ny)

    def inside(x, y, z):
        return 0 <= x < nx and 0 <= y < ny and 0 <= z < nz

    def vid(x, y, z):
        return x + nx * (y + ny * z)

    # escape rows, in ascending state order
    escapes = []
    if med.bc == "vacuum":
        for v in range(V):
            x, y, z = coords(v)
            for m in range(26):
                e = LV[m]
                if not inside(x + e[0], y + e[1], z + e[2]):
                    escapes.append((v, m))
    R = D + len(escapes)
    A = np.zeros((R, D))

    def incoming(w, mp):
        """moves (u, m, f) delivering into state (w, mp)."""
        x, y, z = coords(w)
        out = []
        # ballistic / scattered arrival from the neighbour behind
        for m in range(26):
            e = LV[m]
            ux, uy, uz = x - e[0], y - e[1], z - e[2]
            if not inside(ux, uy, uz):
                continue
            u = vid(ux, uy, uz)
            n1, n2 = nidx[mat[u]], nidx[mat[w]]
            if n1 == n2:
                if m == mp:
                    out.append((u, m, 1.0))
            else:
                s = unit(m)
                N = normal(med, ux, uy, uz, e, s)
                Rf, Tf, mr, mt = fresnel(m, n1, n2, N)
                if Tf > 0.0 and mp in mt:
                    out.append((u, m, Tf / len(mt)))
        # populations of w itself turned back: walls and interface reflection
        for m in range(26):
            e = LV[m]
            tx, ty, tz = x + e[0], y + e[1], z + e[2]
            if not inside(tx, ty, tz):
                if med.bc == "reflect":
                    r = [e[0] if 0 <= tx < nx else -e[0],
                         e[1] if 0 <= ty < ny else -e[1],
                         e[2] if 0 <= tz < nz else -e[2]]
                    if LV.index(tuple(r)) == mp:
                        out.append((w, m, 1.0))
                continue
            t = vid(tx, ty, tz)
            n1, n2 = nidx[mat[w]], nidx[mat[t]]
            if n1 != n2:
                s = unit(m)
                N = normal(med, x, y, z, e, s)
                Rf, Tf, mr, mt = fresnel(m, n1, n2, N)
                if mp in mr:
                    out.append((w, m, Rf / len(mr)))
        return sorted(out)

    def fill(row, moves):
        for u, m, f in moves:
            C = blocks[mat[u]]
            for n in range(26):
                A[row, 26 * u + n] += f * C[m][n]

    for w in range(V):
        for mp in range(26):
            fill(26 * w + mp, incoming(w, mp))
    for i, (v, m) in enumerate(escapes):
        fill(D + i, [(v, m, 1.0)])
    return A, escapes
