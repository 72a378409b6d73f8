// Host-side coefficient model of a DRTS medium: per-material direction blocks
// (FP64), the Fresnel split of every move that crosses an interface, the list
// of (voxel, direction) pairs leaving through vacuum faces, and the list of
// moves whose target is not the plain neighbour state.
//
// Arithmetic is FP64 with the evaluation order written out in each formula;
// the device assembly only copies, multiplies by split factors and sums in a
// fixed order, so the assembled values are reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "drts_internal.h"

namespace drts {
namespace {

constexpr double kC0 = 299792458.0;  // speed of light in vacuum, m/s

struct Unit {
    double s[kDirs][3];  // unit vector of every lattice direction
    Unit()
    {
        for (int d = 0; d < kDirs; ++d) {
            int e0 = dir_dx(d), e1 = dir_dy(d), e2 = dir_dz(d);
            double len = std::sqrt((double)(e0 * e0 + e1 * e1 + e2 * e2));
            s[d][0] = (double)e0 / len;
            s[d][1] = (double)e1 / len;
            s[d][2] = (double)e2 / len;
        }
    }
};
const Unit &units()
{
    static const Unit u;
    return u;
}

inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Henyey-Greenstein phase value without its 1/(4 pi) (it cancels when normalised).
inline double phase_hg(double g, double cs)
{
    double q = 1.0 + g * g - 2.0 * g * cs;
    return (1.0 - g * g) / (q * std::sqrt(q));
}

// C[m][n] = alpha (S[m][n]) off the diagonal, alpha (P0 + S[n][n]) on it, with
// P0 = exp(-mu_s h), alpha = exp(-mu_a h), G[m][n] = p(cos_mn) / sum_k p(cos_kn)
// (Eq. (9)-(10), (19), (21)) and S the scattered part.  With at most one
// scattering per step (K = 1, Eq. (6)-(7)) S = Ps G, Ps = 1 - P0.  With K > 1
// the photons scattered i times in the step (Poisson weight P_i of Eq. (4),
// P_i = P_{i-1} (mu_s h) / i) end in the direction of i successive single
// scatterings, G^i = G G^{i-1}:
//   S = P_1 G + P_2 G^2 + ... + P_{K-1} G^{K-1} + (1 - P_0 - ... - P_{K-1}) G^K,
// summed in that order (the last weight takes every larger count).
void direction_block(const drts_material_t &q, double h, int K, double *C)
{
    const double P0 = std::exp(-q.mu_s * h);
    const double alpha = std::exp(-q.mu_a * h);
    double phase[kDirs][kDirs];
    for (int a = 0; a < kDirs; ++a) {
        const int ax = dir_dx(a), ay = dir_dy(a), az = dir_dz(a);
        for (int b = 0; b < kDirs; ++b) {
            const int bx = dir_dx(b), by = dir_dy(b), bz = dir_dz(b);
            const int ip = ax * bx + ay * by + az * bz;
            const int la = ax * ax + ay * ay + az * az, lb = bx * bx + by * by + bz * bz;
            phase[a][b] = phase_hg(q.g, (double)ip / std::sqrt((double)(la * lb)));
        }
    }
    std::vector<double> G((size_t)kDirs * kDirs), Gi, next((size_t)kDirs * kDirs), S((size_t)kDirs * kDirs, 0.0);
    for (int n = 0; n < kDirs; ++n) {
        double Z = 0.0;
        for (int k = 0; k < kDirs; ++k) Z += phase[k][n];
        for (int m = 0; m < kDirs; ++m) G[(size_t)m * kDirs + n] = phase[m][n] / Z;
    }
    // Poisson weights and the remaining probability
    double Pi = P0, cum = P0;
    const double lam = q.mu_s * h;
    Gi = G;   // G^1
    for (int i = 1; i <= K; ++i) {
        double w;
        if (i < K) {
            Pi = (Pi * lam) / (double)i;
            w = Pi;
            cum = cum + Pi;
        } else {
            w = 1.0 - cum;
        }
        for (size_t e = 0; e < S.size(); ++e) S[e] = (i == 1) ? w * Gi[e] : S[e] + w * Gi[e];
        if (i < K) {
            // G^{i+1}[m][n] = sum_k G[m][k] G^i[k][n], ascending k
            for (int m = 0; m < kDirs; ++m)
                for (int n = 0; n < kDirs; ++n) {
                    double acc = 0.0;
                    for (int k = 0; k < kDirs; ++k) acc += G[(size_t)m * kDirs + k] * Gi[(size_t)k * kDirs + n];
                    next[(size_t)m * kDirs + n] = acc;
                }
            Gi.swap(next);
        }
    }
    for (int n = 0; n < kDirs; ++n)
        for (int m = 0; m < kDirs; ++m) {
            const double s = S[(size_t)m * kDirs + n];
            C[m * kDirs + n] = (m == n) ? alpha * (P0 + s) : alpha * s;
        }
}

// Lattice directions on side `side` of the surface (sign of s_d . N) whose unit
// vectors are closest to `want`: every one whose s_d . want lies within 1e-12
// of the largest value, written in ascending order; returns their count.  A
// population snapped to k of them is split evenly (no direction index is
// preferred, so the split keeps the medium's symmetries).
int nearest_directions(const double *want, const double *N, int side, int *out)
{
    const Unit &U = units();
    double best = -INFINITY;
    bool any = false;
    for (int d = 0; d < kDirs; ++d) {
        const double sn = dot3(U.s[d], N);
        if (!(side < 0 ? sn < 0.0 : sn > 0.0)) continue;
        const double v = dot3(U.s[d], want);
        if (!any || v > best) best = v;
        any = true;
    }
    int k = 0;
    for (int d = 0; any && d < kDirs; ++d) {
        const double sn = dot3(U.s[d], N);
        if (!(side < 0 ? sn < 0.0 : sn > 0.0)) continue;
        if (dot3(U.s[d], want) >= best - 1e-12) out[k++] = d;
    }
    return k;
}

struct Split {
    double R, T;
    int n_refl = 0, n_trans = 0;
    int m_refl[kDirs], m_trans[kDirs];
};

// Unpolarised Fresnel split (Sec. 4.2) of direction m going from index n1 to n2
// through a surface of unit normal N (s_m . N > 0).
Split fresnel_split(int m, double n1, double n2, const double *N)
{
    const double *s = units().s[m];
    const double ci = dot3(s, N);
    const double eta = n1 / n2;
    const double s2t = eta * eta * (1.0 - ci * ci);
    Split out;
    double ct;
    if (s2t >= 1.0) {  // total internal reflection
        out.R = 1.0;
        out.T = 0.0;
        ct = 0.0;
    } else {
        ct = std::sqrt(1.0 - s2t);
        const double rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
        const double rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct);
        out.R = 0.5 * (rs * rs + rp * rp);
        out.T = 1.0 - out.R;
    }
    double r[3], t[3];
    for (int i = 0; i < 3; ++i) {
        r[i] = s[i] - (2.0 * ci) * N[i];
        t[i] = eta * s[i] + (ct - eta * ci) * N[i];
    }
    out.n_refl = nearest_directions(r, N, -1, out.m_refl);
    out.n_trans = out.T > 0.0 ? nearest_directions(t, N, +1, out.m_trans) : 0;
    return out;
}

// Unit normal of the crossing from voxel (x,y,z) along direction d, pointing
// from the first voxel into the second.
void crossing_normal(const drts_geometry_t &g, int x, int y, int z, int d, double *N)
{
    const double *s = units().s[d];
    const int ex = dir_dx(d), ey = dir_dy(d), ez = dir_dz(d);
    if (g.kind == DRTS_GEOM_LAYERS_Z && ez != 0) {
        N[0] = 0.0;
        N[1] = 0.0;
        N[2] = ez > 0 ? 1.0 : -1.0;
        return;
    }
    if (g.kind == DRTS_GEOM_SPHERE) {
        // radial direction at the midpoint of the two voxel centres
        const double px = (double)x + 0.5 + 0.5 * (double)ex;
        const double py = (double)y + 0.5 + 0.5 * (double)ey;
        const double pz = (double)z + 0.5 + 0.5 * (double)ez;
        const double w[3] = {px - g.sphere_c[0], py - g.sphere_c[1], pz - g.sphere_c[2]};
        const double len = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (len > 0.0) {
            N[0] = w[0] / len;
            N[1] = w[1] / len;
            N[2] = w[2] / len;
            if (dot3(s, N) < 0.0) {
                N[0] = -N[0];
                N[1] = -N[1];
                N[2] = -N[2];
            }
            return;
        }
    }
    N[0] = s[0];
    N[1] = s[1];
    N[2] = s[2];
}

// Fraction of the centre-to-centre segment from voxel (x,y,z) along lattice
// direction d lying in the first voxel's medium: 1/2 at a planar layer or a
// voxel face; for a sphere, where |X + s e - c| = r for s in [0, 1] (leaving
// the sphere when X lies inside it, entering otherwise).
double crossing_fraction(const drts_geometry_t &g, int x, int y, int z, int d)
{
    if (g.kind != DRTS_GEOM_SPHERE) return 0.5;
    const int e[3] = {dir_dx(d), dir_dy(d), dir_dz(d)};
    const double X[3] = {(double)x + 0.5 - g.sphere_c[0], (double)y + 0.5 - g.sphere_c[1],
                         (double)z + 0.5 - g.sphere_c[2]};
    const double a = (double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double b = 2.0 * ((double)e[0] * X[0] + (double)e[1] * X[1] + (double)e[2] * X[2]);
    const double c = X[0] * X[0] + X[1] * X[1] + X[2] * X[2] - g.sphere_r * g.sphere_r;
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) disc = 0.0;
    const double q = std::sqrt(disc);
    double s = (c <= 0.0) ? (-b + q) / (2.0 * a) : (-b - q) / (2.0 * a);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    return s;
}

struct IrrMove {
    int64_t row, vox;
    int32_t dir;
    double f;
    bool operator<(const IrrMove &o) const
    {
        if (row != o.row) return row < o.row;
        if (vox != o.vox) return vox < o.vox;
        return dir < o.dir;
    }
};

// ---- Lebedev-86 directions with multi-voxel weights (Sec. 3, Eq. (18)-(21)) ----

// Published generators of the 86-point rule (degree 15): the octahedron
// vertices (a1), the cube vertices (a3), two orbits (+-l, +-l, +-m) (b_k) and
// one orbit (+-p, +-q, 0) (c_1), with their weights.
constexpr double kLebA1 = 0.1154401154401154e-1;
constexpr double kLebA3 = 0.1194390908585628e-1;
constexpr double kLebBL[2] = {0.3696028464541502, 0.6943540066026664};
constexpr double kLebBW[2] = {0.1111055571060340e-1, 0.1187650129453714e-1};
constexpr double kLebCP = 0.3742430390903412;
constexpr double kLebCW = 0.1181230374690448e-1;
constexpr int kLeb = 86;

struct LebPoint {
    double x, y, z, w;
};

// every sign combination of (a, b, c), a zero component taking only +0
void leb_orbit(std::vector<LebPoint> &out, double a, double b, double c, double w)
{
    for (int sa = -1; sa <= 1; sa += 2)
        for (int sb = -1; sb <= 1; sb += 2)
            for (int sc = -1; sc <= 1; sc += 2) {
                if ((a == 0.0 && sa < 0) || (b == 0.0 && sb < 0) || (c == 0.0 && sc < 0)) continue;
                out.push_back({sa * a, sb * b, sc * c, w});
            }
}

// distance from P to the segment a -> b (the point a when a == b)
double segment_distance(const double *P, const double *a, const double *b)
{
    const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double ap[3] = {P[0] - a[0], P[1] - a[1], P[2] - a[2]};
    const double L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
    double t = 0.0;
    if (L2 > 0.0) {
        t = (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / L2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    const double q[3] = {a[0] + t * ab[0], a[1] + t * ab[1], a[2] + t * ab[2]};
    const double d[3] = {P[0] - q[0], P[1] - q[1], P[2] - q[2]};
    return std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

inline uint32_t pack_off(int dx, int dy, int dz)
{
    return (uint32_t)(dx + 16) | ((uint32_t)(dy + 16) << 5) | ((uint32_t)(dz + 16) << 10);
}

// Direction block over the 86 directions for a step of light path L (mm):
// C[m][n] = alpha (Ps G[m][n]) off the diagonal, alpha (P0 + Ps G[n][n]) on it,
// G[m][n] = w_m p(S_m . S_n) / sum_k w_k p(S_k . S_n) (each direction weighted
// by its solid angle, the rule's weight).
void lebedev_block(const drts_material_t &q, double L, const double *S, const double *w, double *C)
{
    const double P0 = std::exp(-q.mu_s * L);
    const double Ps = 1.0 - P0;
    const double alpha = std::exp(-q.mu_a * L);
    double p[kLeb];
    for (int n = 0; n < kLeb; ++n) {
        for (int m = 0; m < kLeb; ++m) {
            const double cs = S[3 * m] * S[3 * n] + S[3 * m + 1] * S[3 * n + 1] + S[3 * m + 2] * S[3 * n + 2];
            p[m] = w[m] * phase_hg(q.g, cs);
        }
        double Z = 0.0;
        for (int k = 0; k < kLeb; ++k) Z += p[k];
        for (int m = 0; m < kLeb; ++m) {
            const double G = p[m] / Z;
            C[m * kLeb + n] = (m == n) ? alpha * (P0 + Ps * G) : alpha * (Ps * G);
        }
    }
}

// The host model of a Lebedev medium: blocks, stencils of every direction
// pair (voxels within 2 dr = one voxel of the arrival segment, weights the
// normalised ramp 1 - d summed in scan order), the per-direction pull lists
// and the escape states.
int build_lebedev_model(const drts_medium_t *m, Model *M)
{
    const double c = m->c_dt > 0.0 ? m->c_dt : 1.0;
    if (!(c <= 8.0)) return set_error(DRTS_E_INVALID, "c_dt must be in (0, 8] voxels");
    if (m->bc != DRTS_BC_VACUUM) return set_error(DRTS_E_INVALID, "Lebedev directions take vacuum faces");
    if (m->scatter_order > 1) return set_error(DRTS_E_INVALID, "Lebedev directions take scatter_order 0 or 1");
    for (int q = 1; q < m->n_mat; ++q)
        if (m->mat[q].n != m->mat[0].n)
            return set_error(DRTS_E_INVALID, "Lebedev directions take one refractive index (no interfaces)");
    if (M->n_vox * kLeb > (int64_t)INT32_MAX - 1)
        return set_error(DRTS_E_RANGE, "%lld states exceed the int32 column range", (long long)(M->n_vox * kLeb));
    M->n_dir = kLeb;
    M->c_dt = c;
    M->n_states = M->n_vox * kLeb;
    M->dt_s = c * m->grid.h_mm * 1e-3 * m->n_ref / kC0;
    M->dir_unit.resize(3 * kLeb);
    M->dir_w.resize(kLeb);
    lebedev86(M->dir_unit.data(), M->dir_w.data());
    const double *S = M->dir_unit.data();
    const double L = c * m->grid.h_mm;
    M->blocks.resize((size_t)m->n_mat * kLeb * kLeb);
    for (int q = 0; q < m->n_mat; ++q) {
        lebedev_block(m->mat[q], L, S, M->dir_w.data(), &M->blocks[(size_t)q * kLeb * kLeb]);
        M->absorb[q] = -std::expm1(-m->mat[q].mu_a * L);
    }
    // stencils of the pairs, offsets in scan order (ascending dz, dy, dx)
    const int R = (int)std::ceil(c + 1.0);
    M->pair_ptr.assign((size_t)kLeb * kLeb + 1, 0);
    M->pair_key.clear();
    M->pair_w.clear();
    std::vector<double> raw;
    std::vector<uint32_t> keys;
    for (int mm = 0; mm < kLeb; ++mm)
        for (int n = 0; n < kLeb; ++n) {
            const double a[3] = {c * S[3 * mm], c * S[3 * mm + 1], c * S[3 * mm + 2]};
            const double b[3] = {c * S[3 * n], c * S[3 * n + 1], c * S[3 * n + 2]};
            M->pair_ptr[(size_t)mm * kLeb + n] = (int64_t)M->pair_key.size();
            raw.clear();
            keys.clear();
            double sum = 0.0;
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        const double P[3] = {(double)dx, (double)dy, (double)dz};
                        const double d = segment_distance(P, a, b);
                        if (d < 1.0) {
                            keys.push_back(pack_off(dx, dy, dz));
                            raw.push_back(1.0 - d);
                            sum += raw.back();
                        }
                    }
            for (size_t i = 0; i < raw.size(); ++i) {
                M->pair_key.push_back(keys[i]);
                M->pair_w.push_back(raw[i] / sum);
            }
        }
    M->pair_ptr[(size_t)kLeb * kLeb] = (int64_t)M->pair_key.size();
    // per arrival direction: (offset, n) in descending offset order, ascending n
    M->arr_ptr.assign(kLeb + 1, 0);
    M->arr_key.clear();
    M->arr_w.clear();
    struct E {
        int dz, dy, dx, n;
        double w;
    };
    std::vector<E> es;
    for (int mm = 0; mm < kLeb; ++mm) {
        es.clear();
        for (int n = 0; n < kLeb; ++n)
            for (int64_t e = M->pair_ptr[(size_t)mm * kLeb + n]; e < M->pair_ptr[(size_t)mm * kLeb + n + 1]; ++e) {
                const uint32_t k = M->pair_key[(size_t)e];
                es.push_back({off_dz(k), off_dy(k), off_dx(k), n, M->pair_w[(size_t)e]});
            }
        std::sort(es.begin(), es.end(), [](const E &u, const E &v) {
            if (u.dz != v.dz) return u.dz > v.dz;
            if (u.dy != v.dy) return u.dy > v.dy;
            if (u.dx != v.dx) return u.dx > v.dx;
            return u.n < v.n;
        });
        M->arr_ptr[(size_t)mm] = (int64_t)M->arr_key.size();
        for (const E &e : es) {
            M->arr_key.push_back(pack_off(e.dx, e.dy, e.dz) | ((uint32_t)e.n << 15));
            M->arr_w.push_back(e.w);
        }
    }
    M->arr_ptr[kLeb] = (int64_t)M->arr_key.size();
    // escape states: (v, m) with some offset of direction m outside the grid
    std::vector<int> lo(3 * kLeb, 0), hi(3 * kLeb, 0);   // extent of every direction's offsets
    for (int mm = 0; mm < kLeb; ++mm)
        for (int64_t e = M->arr_ptr[(size_t)mm]; e < M->arr_ptr[(size_t)mm + 1]; ++e) {
            const uint32_t k = M->arr_key[(size_t)e];
            const int o[3] = {off_dx(k), off_dy(k), off_dz(k)};
            for (int i = 0; i < 3; ++i) {
                if (e == M->arr_ptr[(size_t)mm] || o[i] < lo[3 * mm + i]) lo[3 * mm + i] = o[i];
                if (e == M->arr_ptr[(size_t)mm] || o[i] > hi[3 * mm + i]) hi[3 * mm + i] = o[i];
            }
        }
    M->escape_state.clear();
    const int nx = M->nx, ny = M->ny, nz = M->nz;
    for (int64_t v = 0; v < M->n_vox; ++v) {
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
        for (int mm = 0; mm < kLeb; ++mm) {
            // the offsets of a direction span a box; any offset leaving the grid
            // leaves through a face of that box, so test the offsets themselves
            bool out = false;
            if (x + lo[3 * mm] < 0 || x + hi[3 * mm] >= nx || y + lo[3 * mm + 1] < 0 || y + hi[3 * mm + 1] >= ny ||
                z + lo[3 * mm + 2] < 0 || z + hi[3 * mm + 2] >= nz) {
                for (int64_t e = M->arr_ptr[(size_t)mm]; e < M->arr_ptr[(size_t)mm + 1] && !out; ++e) {
                    const uint32_t k = M->arr_key[(size_t)e];
                    const int ux = x + off_dx(k), uy = y + off_dy(k), uz = z + off_dz(k);
                    out = ux < 0 || ux >= nx || uy < 0 || uy >= ny || uz < 0 || uz >= nz;
                }
            }
            if (out) M->escape_state.push_back(kLeb * v + mm);
        }
    }
    M->n_escape = (int64_t)M->escape_state.size();
    M->n_rows = M->n_states + M->n_escape;
    M->irr_row.clear();
    M->irr_vox.clear();
    M->irr_dir.clear();
    M->irr_f.clear();
    return DRTS_OK;
}

}  // namespace

void lebedev86(double *unit, double *weight)
{
    std::vector<LebPoint> P;
    leb_orbit(P, 1.0, 0.0, 0.0, kLebA1);
    leb_orbit(P, 0.0, 1.0, 0.0, kLebA1);
    leb_orbit(P, 0.0, 0.0, 1.0, kLebA1);
    const double r = std::sqrt(1.0 / 3.0);
    leb_orbit(P, r, r, r, kLebA3);
    for (int i = 0; i < 2; ++i) {
        const double l = kLebBL[i], mz = std::sqrt(1.0 - 2.0 * l * l);
        leb_orbit(P, l, l, mz, kLebBW[i]);
        leb_orbit(P, l, mz, l, kLebBW[i]);
        leb_orbit(P, mz, l, l, kLebBW[i]);
    }
    const double p = kLebCP, q = std::sqrt(1.0 - p * p);
    leb_orbit(P, p, q, 0.0, kLebCW);
    leb_orbit(P, q, p, 0.0, kLebCW);
    leb_orbit(P, p, 0.0, q, kLebCW);
    leb_orbit(P, q, 0.0, p, kLebCW);
    leb_orbit(P, 0.0, p, q, kLebCW);
    leb_orbit(P, 0.0, q, p, kLebCW);
    std::sort(P.begin(), P.end(), [](const LebPoint &a, const LebPoint &b) {
        if (a.z != b.z) return a.z < b.z;
        if (a.y != b.y) return a.y < b.y;
        return a.x < b.x;
    });
    double sum = 0.0;
    for (const LebPoint &t : P) sum += t.w;
    for (int i = 0; i < kLeb; ++i) {
        if (unit) {
            unit[3 * i] = P[(size_t)i].x;
            unit[3 * i + 1] = P[(size_t)i].y;
            unit[3 * i + 2] = P[(size_t)i].z;
        }
        if (weight) weight[i] = P[(size_t)i].w / sum;
    }
}

int build_model(const drts_medium_t *m, Model *M)
{
    if (!m) return set_error(DRTS_E_INVALID, "medium is NULL");
    const drts_grid_t &g = m->grid;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return set_error(DRTS_E_INVALID, "grid must be at least 1x1x1");
    if (!(g.h_mm > 0.0) || !std::isfinite(g.h_mm)) return set_error(DRTS_E_INVALID, "h_mm must be positive");
    if (m->n_mat < 1 || m->n_mat > 255 || !m->mat)
        return set_error(DRTS_E_INVALID, "need 1..255 materials");
    if (m->bc != DRTS_BC_VACUUM && m->bc != DRTS_BC_REFLECT) return set_error(DRTS_E_INVALID, "bad bc %d", m->bc);
    if (m->value_type != DRTS_F64 && m->value_type != DRTS_F32)
        return set_error(DRTS_E_INVALID, "bad value_type %d", m->value_type);
    if (m->rounding != DRTS_ROUND_NEAREST && m->rounding != DRTS_ROUND_DITHER)
        return set_error(DRTS_E_INVALID, "bad rounding %d", m->rounding);
    if (m->geom.kind < DRTS_GEOM_VOXELS || m->geom.kind > DRTS_GEOM_SPHERE)
        return set_error(DRTS_E_INVALID, "bad geometry kind %d", m->geom.kind);
    if (!(m->n_ref > 0.0)) return set_error(DRTS_E_INVALID, "n_ref must be positive");
    if (m->scatter_order < 0 || m->scatter_order > 16)
        return set_error(DRTS_E_INVALID, "scatter_order must be in 0..16");
    if (m->interface_model != DRTS_INTERFACE_ORIGIN && m->interface_model != DRTS_INTERFACE_SUBSTEP)
        return set_error(DRTS_E_INVALID, "unknown interface model %d", m->interface_model);
    for (int q = 0; q < m->n_mat; ++q) {
        const drts_material_t &mt = m->mat[q];
        if (!(mt.mu_s >= 0.0) || !(mt.mu_a >= 0.0) || !(mt.g > -1.0 && mt.g < 1.0) || !(mt.n > 0.0) ||
            !std::isfinite(mt.mu_s) || !std::isfinite(mt.mu_a))
            return set_error(DRTS_E_INVALID, "material %d out of range", q);
    }
    const int64_t V = (int64_t)g.nx * g.ny * g.nz;
    if (V * kDirs > (int64_t)INT32_MAX - 1)
        return set_error(DRTS_E_RANGE, "%lld states exceed the int32 column range", (long long)(V * kDirs));

    M->nx = g.nx;
    M->ny = g.ny;
    M->nz = g.nz;
    M->n_vox = V;
    M->n_states = V * kDirs;
    M->h_mm = g.h_mm;
    M->dt_s = g.h_mm * 1e-3 * m->n_ref / kC0;
    M->bc = m->bc;
    M->value_type = m->value_type;
    M->rounding = m->rounding;
    M->scatter_order = m->scatter_order < 1 ? 1 : m->scatter_order;
    M->mats.assign(m->mat, m->mat + m->n_mat);

    // material map
    M->mat_of_voxel.resize(V);
    if (m->mat_of_voxel) {
        for (int64_t v = 0; v < V; ++v) {
            if (m->mat_of_voxel[v] >= m->n_mat)
                return set_error(DRTS_E_INVALID, "voxel %lld uses material %d of %d", (long long)v,
                                 (int)m->mat_of_voxel[v], m->n_mat);
            M->mat_of_voxel[v] = m->mat_of_voxel[v];
        }
    } else if (m->geom.kind == DRTS_GEOM_LAYERS_Z) {
        if (m->geom.n_layers < 1 || !m->geom.layer_z0 || m->geom.layer_z0[0] != 0 ||
            m->geom.n_layers > m->n_mat)
            return set_error(DRTS_E_INVALID, "layers need layer_z0[0] == 0 and n_layers <= n_mat");
        for (int i = 1; i < m->geom.n_layers; ++i)
            if (m->geom.layer_z0[i] <= m->geom.layer_z0[i - 1])
                return set_error(DRTS_E_INVALID, "layer_z0 must ascend");
        for (int z = 0; z < g.nz; ++z) {
            int layer = 0;
            while (layer + 1 < m->geom.n_layers && z >= m->geom.layer_z0[layer + 1]) ++layer;
            std::fill(M->mat_of_voxel.begin() + (int64_t)z * g.nx * g.ny,
                      M->mat_of_voxel.begin() + (int64_t)(z + 1) * g.nx * g.ny, (uint8_t)layer);
        }
    } else if (m->geom.kind == DRTS_GEOM_SPHERE) {
        if (m->n_mat < 2) return set_error(DRTS_E_INVALID, "a sphere needs materials 0 and 1");
        const double r2 = m->geom.sphere_r * m->geom.sphere_r;
        for (int64_t v = 0; v < V; ++v) {
            const double x = (double)(v % g.nx) + 0.5 - m->geom.sphere_c[0];
            const double y = (double)((v / g.nx) % g.ny) + 0.5 - m->geom.sphere_c[1];
            const double z = (double)(v / ((int64_t)g.nx * g.ny)) + 0.5 - m->geom.sphere_c[2];
            M->mat_of_voxel[v] = (x * x + y * y + z * z <= r2) ? 1 : 0;
        }
    } else {
        std::fill(M->mat_of_voxel.begin(), M->mat_of_voxel.end(), (uint8_t)0);
    }

    // per-material tables
    M->absorb.resize(m->n_mat);
    M->index.resize(m->n_mat);
    for (int q = 0; q < m->n_mat; ++q) M->index[q] = m->mat[q].n;
    if (m->directions == DRTS_DIRS_LEBEDEV86) return build_lebedev_model(m, M);
    if (m->directions != DRTS_DIRS_LATTICE26) return set_error(DRTS_E_INVALID, "unknown directions %d", m->directions);
    if (m->c_dt != 0.0 && m->c_dt != 1.0)
        return set_error(DRTS_E_INVALID, "the lattice directions move one voxel per step (c_dt 0 or 1)");
    M->n_dir = kDirs;
    M->blocks.resize((size_t)m->n_mat * kDirs * kDirs);
    for (int q = 0; q < m->n_mat; ++q) {
        direction_block(m->mat[q], g.h_mm, M->scatter_order, &M->blocks[(size_t)q * kDirs * kDirs]);
        M->absorb[q] = -std::expm1(-m->mat[q].mu_a * g.h_mm);
        M->index[q] = m->mat[q].n;
    }

    // escape list and irregular moves
    M->escape_state.clear();
    std::vector<IrrMove> irr;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t v = x + (int64_t)nx * (y + (int64_t)ny * z);
                const bool face = x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1;
                const double n1 = M->index[M->mat_of_voxel[v]];
                for (int d = 0; d < kDirs; ++d) {
                    const int tx = x + dir_dx(d), ty = y + dir_dy(d), tz = z + dir_dz(d);
                    const bool in = tx >= 0 && tx < nx && ty >= 0 && ty < ny && tz >= 0 && tz < nz;
                    if (!in) {
                        if (!face) continue;
                        if (m->bc == DRTS_BC_VACUUM) {
                            M->escape_state.push_back(kDirs * v + d);
                        } else {
                            const int rx = (tx < 0 || tx >= nx) ? -dir_dx(d) : dir_dx(d);
                            const int ry = (ty < 0 || ty >= ny) ? -dir_dy(d) : dir_dy(d);
                            const int rz = (tz < 0 || tz >= nz) ? -dir_dz(d) : dir_dz(d);
                            irr.push_back({kDirs * v + dir_of(rx, ry, rz), v, d, 1.0});
                        }
                        continue;
                    }
                    const int64_t u = tx + (int64_t)nx * (ty + (int64_t)ny * tz);
                    const double n2 = M->index[M->mat_of_voxel[u]];
                    if (n1 == n2) continue;
                    double N[3];
                    crossing_normal(m->geom, x, y, z, d, N);
                    const Split sp = fresnel_split(d, n1, n2, N);
                    double T = sp.T;
                    int64_t vr = v;   // where the reflected part lands
                    if (m->interface_model == DRTS_INTERFACE_SUBSTEP) {
                        // the transmitted part is absorbed along its path in
                        // each medium; at a planar interface the reflected part
                        // lands one voxel over along the surface
                        const double f = crossing_fraction(m->geom, x, y, z, d);
                        const double mua1 = m->mat[M->mat_of_voxel[v]].mu_a, mua2 = m->mat[M->mat_of_voxel[u]].mu_a;
                        T = T * std::exp(-(mua2 - mua1) * ((1.0 - f) * g.h_mm));
                        if (m->geom.kind == DRTS_GEOM_LAYERS_Z && dir_dz(d) != 0) {
                            const int rx = x + dir_dx(d), ry = y + dir_dy(d);
                            if (rx >= 0 && rx < nx && ry >= 0 && ry < ny)
                                vr = rx + (int64_t)nx * (ry + (int64_t)ny * z);
                        }
                    }
                    for (int i = 0; i < sp.n_refl; ++i)
                        irr.push_back({kDirs * vr + sp.m_refl[i], v, d, sp.R / (double)sp.n_refl});
                    for (int i = 0; i < sp.n_trans; ++i)
                        irr.push_back({kDirs * u + sp.m_trans[i], v, d, T / (double)sp.n_trans});
                }
            }
    M->n_escape = (int64_t)M->escape_state.size();
    M->n_rows = M->n_states + M->n_escape;
    std::sort(irr.begin(), irr.end());
    const size_t ni = irr.size();
    M->irr_row.resize(ni);
    M->irr_vox.resize(ni);
    M->irr_dir.resize(ni);
    M->irr_f.resize(ni);
    for (size_t i = 0; i < ni; ++i) {
        M->irr_row[i] = irr[i].row;
        M->irr_vox[i] = irr[i].vox;
        M->irr_dir[i] = irr[i].dir;
        M->irr_f[i] = irr[i].f;
    }
    return DRTS_OK;
}

}  // namespace drts
