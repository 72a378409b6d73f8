/*
 * FP64 CPU oracle for the Dynamic Radiative Transfer System (DRTS).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The product
 * library never includes, links or calls it, and it shares no code with it.
 *
 * What it computes (plain definitions, written out slowly):
 *   - the system matrix A of Eq. (21)/(23): every state (voxel X_i, direction
 *     S_n) sends, in one step dt, the fraction a_{jm,in} of its photons to the
 *     state (X_j, S_m).  Single-scatter split of Eq. (9)-(10), scattering
 *     kernel g(S_n,S_m) of Eq. (19), forward scatter added on the diagonal of
 *     the direction block as in Eq. (21).  Space is a cubic voxel lattice and
 *     directions are the 26 lattice neighbours (Sec. 3 allows any partition);
 *     both the ballistic and the scattered population arrive at the
 *     neighbour voxel one lattice vector away, i.e. the arrival segment AB of
 *     Sec. 2 is collapsed to its end A.
 *   - escape rows L: photons leaving through a vacuum face are collected in
 *     extra rows (one per (voxel, direction) pair that leaves the grid), so
 *     the rectangular [A; L] has columns summing to exp(-mu_a c dt)
 *     (column-stochastic A_S of Eq. (24)).
 *   - interfaces between media of different refractive index (Sec. 4.2):
 *     the unpolarised Fresnel reflectance R splits the crossing population
 *     into a reflected part that stays in the voxel with the lattice
 *     direction closest to the specular direction, and a transmitted part
 *     that enters the next voxel with the lattice direction closest to the
 *     Snell direction.
 *   - the evolution J(t+dt) = A J(t) + B P(t) of Eq. (26) and the detector
 *     sums M(t) of Eq. (27) with a one-step window, in FP64, with a tracked
 *     power-of-two exponent so that long runs never underflow (scaling by a
 *     power of two is exact, so the values are the unscaled ones).
 *
 * Summation orders are fixed and sequential: a matrix entry that receives
 * several contributions from one column sums them in ascending order of the
 * collision direction m; an SpMV row sums its entries in ascending column
 * order.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NDIR 26

/* ---- lattice directions ------------------------------------------------ */

/* Direction d -> lattice vector.  k = 9(dz+1) + 3(dy+1) + (dx+1) runs over
 * the 27 offsets of the 3x3x3 block; k = 13 (the zero vector) is skipped. */
static void or_dir_vec(int d, int e[3])
{
    int k = d < 13 ? d : d + 1;
    e[0] = k % 3 - 1;
    e[1] = (k / 3) % 3 - 1;
    e[2] = k / 9 - 1;
}

static int or_dir_index(int dx, int dy, int dz)
{
    int k = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
    return k < 13 ? k : k - 1;
}

/* unit vector of direction d: each component of e_d divided by |e_d| */
static void or_dir_unit(int d, double s[3])
{
    int e[3];
    or_dir_vec(d, e);
    double len = sqrt((double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
    s[0] = (double)e[0] / len;
    s[1] = (double)e[1] / len;
    s[2] = (double)e[2] / len;
}

static double or_dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ---- coefficients of one material --------------------------------------- */

/* Henyey-Greenstein phase value for cosine cs (the constant 1/(4 pi) cancels
 * in the normalisation below). */
static double or_hg(double g, double cs)
{
    double q = 1.0 + g * g - 2.0 * g * cs;
    return (1.0 - g * g) / (q * sqrt(q));
}

/*
 * Direction block C[m][n] of one material: the fraction of the population of
 * direction n in a voxel that leaves it in direction m during one step.
 *   P0 = exp(-mu_s h)        unscattered, Eq. (9) without absorption
 *   alpha = exp(-mu_a h)     survival against absorption, Eq. (8)
 *   G[m][n] = p(cos_mn) / sum_k p(cos_kn)     discrete g(S_n, S_m)
 *   C[m][n] = alpha S[m][n]                   m != n      (w1 of Eq. (19))
 *   C[n][n] = alpha (P0 + S[n][n])                        (w0 + w1, Eq. (21))
 * where S is the scattered part.  With at most one scattering per step
 * (order K = 1, Eq. (6)-(7)): S = Ps G, Ps = 1 - P0.  With order K > 1, the
 * population scattered i times during the step (Poisson probability P_i of
 * Eq. (4)) leaves in the direction of i successive single scatterings, so
 * its share of the block is P_i G^i; the counts 0..K-1 take their Poisson
 * probabilities and count K takes what remains:
 *   S = P_1 G^1 + ... + P_{K-1} G^{K-1} + (1 - P_0 - ... - P_{K-1}) G^K
 * added in that order, with P_i = P_{i-1} (mu_s h) / i and
 * G^i[m][n] = sum_k G[m][k] G^{i-1}[k][n] (ascending k).
 * Here h = c dt is the voxel edge.
 */
void or_collision_block_k(double mu_s, double mu_a, double g, double h, int K,
                          double *C /* [26*26], row m, column n */)
{
    double P0 = exp(-mu_s * h);
    double alpha = exp(-mu_a * h);
    double p[NDIR][NDIR], G[NDIR][NDIR], Gi[NDIR][NDIR], Gn[NDIR][NDIR], S[NDIR][NDIR];
    for (int m = 0; m < NDIR; ++m) {
        int em[3];
        or_dir_vec(m, em);
        for (int n = 0; n < NDIR; ++n) {
            int en[3];
            or_dir_vec(n, en);
            int dot = em[0] * en[0] + em[1] * en[1] + em[2] * en[2];
            int nm = em[0] * em[0] + em[1] * em[1] + em[2] * em[2];
            int nn = en[0] * en[0] + en[1] * en[1] + en[2] * en[2];
            double cs = (double)dot / sqrt((double)(nm * nn));
            p[m][n] = or_hg(g, cs);
        }
    }
    for (int n = 0; n < NDIR; ++n) {
        double Z = 0.0;
        for (int k = 0; k < NDIR; ++k)
            Z += p[k][n];
        for (int m = 0; m < NDIR; ++m)
            G[m][n] = p[m][n] / Z;
    }
    if (K < 1) K = 1;
    double lam = mu_s * h;
    double Pi = P0, seen = P0;
    memcpy(Gi, G, sizeof G);
    for (int i = 1; i <= K; ++i) {
        double w;
        if (i < K) {
            Pi = (Pi * lam) / (double)i;   /* Poisson probability of i scatterings */
            w = Pi;
            seen = seen + Pi;
        } else {
            w = 1.0 - seen;                /* K or more scatterings */
        }
        for (int m = 0; m < NDIR; ++m)
            for (int n = 0; n < NDIR; ++n)
                S[m][n] = (i == 1) ? w * Gi[m][n] : S[m][n] + w * Gi[m][n];
        if (i < K) {
            for (int m = 0; m < NDIR; ++m)
                for (int n = 0; n < NDIR; ++n) {
                    double acc = 0.0;
                    for (int k = 0; k < NDIR; ++k)
                        acc += G[m][k] * Gi[k][n];
                    Gn[m][n] = acc;
                }
            memcpy(Gi, Gn, sizeof Gi);
        }
    }
    for (int n = 0; n < NDIR; ++n)
        for (int m = 0; m < NDIR; ++m)
            C[m * NDIR + n] = (m != n) ? alpha * S[m][n] : alpha * (P0 + S[n][n]);
}

/* the single-scatter block (order 1) */
void or_collision_block(double mu_s, double mu_a, double g, double h, double *C)
{
    or_collision_block_k(mu_s, mu_a, g, h, 1, C);
}

/* ---- interfaces ---------------------------------------------------------- */

/* Lattice directions nearest to `target` among those d whose side test
 * (s_d . N) has the requested sign: every such d whose s_d . target lies
 * within 1e-12 of the largest value.  Writes them in ascending order to
 * out[] and returns how many there are (0 when no direction is on that side).
 * A population snapped to k tied directions is split evenly between them. */
static int or_snap(const double target[3], const double N[3], int side, int out[NDIR])
{
    double best = -INFINITY;
    int any = 0;
    for (int d = 0; d < NDIR; ++d) {
        double s[3];
        or_dir_unit(d, s);
        double sn = or_dot3(s, N);
        if ((side < 0 && sn < 0.0) || (side > 0 && sn > 0.0)) {
            double v = or_dot3(s, target);
            if (!any || v > best) best = v;
            any = 1;
        }
    }
    int k = 0;
    for (int d = 0; any && d < NDIR; ++d) {
        double s[3];
        or_dir_unit(d, s);
        double sn = or_dot3(s, N);
        if ((side < 0 && sn < 0.0) || (side > 0 && sn > 0.0))
            if (or_dot3(s, target) >= best - 1e-12) out[k++] = d;
    }
    return k;
}

/*
 * Fresnel split of a population with lattice direction m crossing from index
 * n1 into index n2 through a surface with unit normal N (oriented so that
 * s_m . N > 0).  Outputs the reflectance R (1 on total internal reflection),
 * T = 1 - R, and the snapped reflected / transmitted directions (n_r and n_t
 * of them, tied directions sharing their part evenly; n_t = 0 when T = 0).
 */
void or_fresnel(int m, double n1, double n2, const double N[3],
                double *R_out, double *T_out, int *mr_out, int *nr_out, int *mt_out, int *nt_out)
{
    double s[3];
    or_dir_unit(m, s);
    double cos_i = or_dot3(s, N);
    double eta = n1 / n2;
    double sin2t = eta * eta * (1.0 - cos_i * cos_i);
    double R, T, cos_t;
    if (sin2t >= 1.0) {
        R = 1.0;
        T = 0.0;
        cos_t = 0.0;
    } else {
        cos_t = sqrt(1.0 - sin2t);
        double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
        double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
        R = 0.5 * (rs * rs + rp * rp);
        T = 1.0 - R;
    }
    double r[3], t[3];
    for (int i = 0; i < 3; ++i) {
        r[i] = s[i] - (2.0 * cos_i) * N[i];
        t[i] = eta * s[i] + (cos_t - eta * cos_i) * N[i];
    }
    *R_out = R;
    *T_out = T;
    *nr_out = or_snap(r, N, -1, mr_out);
    *nt_out = (T > 0.0) ? or_snap(t, N, +1, mt_out) : 0;
}

/* ---- medium ---------------------------------------------------------------- */

enum { OR_GEOM_VOXELS = 0, OR_GEOM_LAYERS_Z = 1, OR_GEOM_SPHERE = 2 };
enum { OR_BC_VACUUM = 0, OR_BC_REFLECT = 1 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t n_mat;
    double h_mm;
    const double *mat;           /* [n_mat][4] = mu_s (1/mm), mu_a (1/mm), g, n */
    const uint8_t *mat_of_voxel; /* [nx*ny*nz], voxel v = x + nx (y + ny z) */
    int32_t geom;                /* normal rule at interfaces */
    int32_t bc;                  /* outer faces */
    double sphere_c[3];          /* voxel units; voxel centres at index + 0.5 */
    double sphere_r;
    int32_t scatter_order;       /* scatterings per step the direction block resolves */
    int32_t directions;          /* 0: the 26 lattice directions; 1: Lebedev's 86 */
    double c_dt;                 /* Lebedev: the distance c dt light travels per step, in voxels */
    int32_t interface_model;     /* 0: the whole step in the source medium; 1: sub-step crossing */
} or_medium_t;

enum { OR_DIRS_LATTICE = 0, OR_DIRS_LEBEDEV86 = 1 };

/* unit normal at the crossing of voxel (x,y,z) along lattice vector e,
 * oriented so that it points from the first voxel to the second */
static void or_normal(const or_medium_t *M, int x, int y, int z, const int e[3],
                      const double s[3], double N[3])
{
    if (M->geom == OR_GEOM_LAYERS_Z && e[2] != 0) {
        N[0] = 0.0;
        N[1] = 0.0;
        N[2] = e[2] > 0 ? 1.0 : -1.0;
        return;
    }
    if (M->geom == OR_GEOM_SPHERE) {
        double P[3] = {(double)x + 0.5 + 0.5 * (double)e[0],
                       (double)y + 0.5 + 0.5 * (double)e[1],
                       (double)z + 0.5 + 0.5 * (double)e[2]};
        double w[3] = {P[0] - M->sphere_c[0], P[1] - M->sphere_c[1], P[2] - M->sphere_c[2]};
        double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (len > 0.0) {
            N[0] = w[0] / len;
            N[1] = w[1] / len;
            N[2] = w[2] / len;
            if (or_dot3(s, N) < 0.0) {
                N[0] = -N[0];
                N[1] = -N[1];
                N[2] = -N[2];
            }
            return;
        }
    }
    /* voxel maps without a surface description: normal incidence along s */
    N[0] = s[0];
    N[1] = s[1];
    N[2] = s[2];
}

/* Fraction of the centre-to-centre segment from voxel (x,y,z) along e that lies
 * in the first voxel's medium: 1/2 at a planar layer boundary or a voxel map's
 * face; on a sphere, where the segment meets the sphere's surface (the root of
 * |X + s e - c| = r in [0, 1]: leaving the sphere when the first centre lies
 * inside it, entering otherwise). */
static double or_crossing_fraction(const or_medium_t *M, int x, int y, int z, const int e[3])
{
    if (M->geom != OR_GEOM_SPHERE) return 0.5;
    double X[3] = {(double)x + 0.5 - M->sphere_c[0], (double)y + 0.5 - M->sphere_c[1], (double)z + 0.5 - M->sphere_c[2]};
    double a = (double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    double b = 2.0 * ((double)e[0] * X[0] + (double)e[1] * X[1] + (double)e[2] * X[2]);
    double c = X[0] * X[0] + X[1] * X[1] + X[2] * X[2] - M->sphere_r * M->sphere_r;
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) disc = 0.0;
    double q = sqrt(disc);
    double s = (c <= 0.0) ? (-b + q) / (2.0 * a) : (-b - q) / (2.0 * a);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    return s;
}

/* ---- assembled matrix ------------------------------------------------------ */

typedef struct {
    int64_t n_vox, n_states, n_escape, n_rows, nnz;
    int n_dir;               /* directions per voxel: 26 (lattice) or 86 (Lebedev) */
    int64_t *row_ptr;        /* [n_rows+1] */
    int32_t *col;            /* [nnz] */
    double *val;             /* [nnz] */
    int32_t *escape_of_state; /* [n_states], -1 when (v,m) does not leave */
    double *absorb_of_voxel; /* [n_vox] = 1 - exp(-mu_a h) */
} or_csr_t;

typedef struct {
    int count;
    int64_t row[2 * NDIR];
    double f[2 * NDIR];
} or_targets_t;

/* where the population that leaves voxel v=(x,y,z) with direction m goes */
static void or_move(const or_medium_t *M, const or_csr_t *A, int64_t v, int x, int y, int z,
                    int m, or_targets_t *T)
{
    int e[3];
    or_dir_vec(m, e);
    int ux = x + e[0], uy = y + e[1], uz = z + e[2];
    int inside = ux >= 0 && ux < M->nx && uy >= 0 && uy < M->ny && uz >= 0 && uz < M->nz;
    if (!inside) {
        if (M->bc == OR_BC_VACUUM) {
            T->count = 1;
            T->row[0] = A->n_states + A->escape_of_state[NDIR * v + m];
            T->f[0] = 1.0;
        } else {
            /* specular wall: every component that leaves is reversed, the
             * population stays in v */
            int r[3] = {e[0], e[1], e[2]};
            if (ux < 0 || ux >= M->nx) r[0] = -r[0];
            if (uy < 0 || uy >= M->ny) r[1] = -r[1];
            if (uz < 0 || uz >= M->nz) r[2] = -r[2];
            T->count = 1;
            T->row[0] = NDIR * v + or_dir_index(r[0], r[1], r[2]);
            T->f[0] = 1.0;
        }
        return;
    }
    int64_t u = (int64_t)ux + (int64_t)M->nx * ((int64_t)uy + (int64_t)M->ny * uz);
    double n1 = M->mat[4 * M->mat_of_voxel[v] + 3];
    double n2 = M->mat[4 * M->mat_of_voxel[u] + 3];
    if (n1 == n2) {
        T->count = 1;
        T->row[0] = NDIR * u + m;
        T->f[0] = 1.0;
        return;
    }
    double s[3], N[3];
    or_dir_unit(m, s);
    or_normal(M, x, y, z, e, s, N);
    double R, Tr;
    int mr[NDIR], mt[NDIR], nr, nt;
    or_fresnel(m, n1, n2, N, &R, &Tr, mr, &nr, mt, &nt);
    /* the crossing within the step (Sec. 4.2): with the sub-step model the
     * transmitted part is absorbed along its path in each medium, and at a
     * planar interface the reflected part lands one voxel over along the
     * surface (it meets the surface half way and returns for the other half) */
    int64_t vr = v;
    if (M->interface_model == 1) {
        double f = or_crossing_fraction(M, x, y, z, e);
        double mua1 = M->mat[4 * M->mat_of_voxel[v] + 1], mua2 = M->mat[4 * M->mat_of_voxel[u] + 1];
        Tr = Tr * exp(-(mua2 - mua1) * ((1.0 - f) * M->h_mm));
        if (M->geom == OR_GEOM_LAYERS_Z && e[2] != 0) {
            int tx = x + e[0], ty = y + e[1];
            if (tx >= 0 && tx < M->nx && ty >= 0 && ty < M->ny)
                vr = (int64_t)tx + (int64_t)M->nx * ((int64_t)ty + (int64_t)M->ny * z);
        }
    }
    T->count = 0;
    for (int i = 0; i < nr; ++i) {
        T->row[T->count] = NDIR * vr + mr[i];
        T->f[T->count] = R / (double)nr;
        T->count++;
    }
    for (int i = 0; i < nt; ++i) {
        T->row[T->count] = NDIR * u + mt[i];
        T->f[T->count] = Tr / (double)nt;
        T->count++;
    }
}

void or_free(or_csr_t *A)
{
    if (!A) return;
    free(A->row_ptr);
    free(A->col);
    free(A->val);
    free(A->escape_of_state);
    free(A->absorb_of_voxel);
    free(A);
}

/*
 * Push-style assembly.  For every column (v, n) in ascending order and every
 * collision direction m in ascending order, the value C_q(v)[m][n] (times the
 * Fresnel factor where the move crosses an interface) is appended to each
 * target row.  Appends to a row therefore arrive in ascending column order,
 * and several contributions of one column to one row are adjacent; they are
 * summed in m order.  Exact zeros are not stored.
 */
or_csr_t *or_build_lebedev(const or_medium_t *M);

or_csr_t *or_build(const or_medium_t *M)
{
    if (M->directions == OR_DIRS_LEBEDEV86) return or_build_lebedev(M);
    or_csr_t *A = (or_csr_t *)calloc(1, sizeof(or_csr_t));
    if (!A) return NULL;
    A->n_dir = NDIR;
    int64_t V = (int64_t)M->nx * M->ny * M->nz;
    A->n_vox = V;
    A->n_states = NDIR * V;
    A->escape_of_state = (int32_t *)malloc(sizeof(int32_t) * A->n_states);
    A->absorb_of_voxel = (double *)malloc(sizeof(double) * V);
    double *Cq = (double *)malloc(sizeof(double) * NDIR * NDIR * M->n_mat);
    if (!A->escape_of_state || !A->absorb_of_voxel || !Cq) goto fail;

    for (int q = 0; q < M->n_mat; ++q)
        or_collision_block_k(M->mat[4 * q], M->mat[4 * q + 1], M->mat[4 * q + 2], M->h_mm, M->scatter_order,
                             Cq + (int64_t)q * NDIR * NDIR);

    /* escape rows: (v, m) pairs leaving the grid, ascending state order */
    int64_t ne = 0;
    for (int64_t v = 0; v < V; ++v) {
        int x = (int)(v % M->nx), y = (int)((v / M->nx) % M->ny), z = (int)(v / ((int64_t)M->nx * M->ny));
        A->absorb_of_voxel[v] = -expm1(-M->mat[4 * M->mat_of_voxel[v] + 1] * M->h_mm);
        for (int m = 0; m < NDIR; ++m) {
            int e[3];
            or_dir_vec(m, e);
            int ux = x + e[0], uy = y + e[1], uz = z + e[2];
            int inside = ux >= 0 && ux < M->nx && uy >= 0 && uy < M->ny && uz >= 0 && uz < M->nz;
            A->escape_of_state[NDIR * v + m] = (!inside && M->bc == OR_BC_VACUUM) ? (int32_t)(ne++) : -1;
        }
    }
    A->n_escape = ne;
    A->n_rows = A->n_states + ne;

    /* pass 1: upper bound of entries per row (before merging) */
    int64_t *cnt = (int64_t *)calloc((size_t)A->n_rows + 1, sizeof(int64_t));
    if (!cnt) goto fail;
    for (int64_t v = 0; v < V; ++v) {
        int x = (int)(v % M->nx), y = (int)((v / M->nx) % M->ny), z = (int)(v / ((int64_t)M->nx * M->ny));
        const double *C = Cq + (int64_t)M->mat_of_voxel[v] * NDIR * NDIR;
        for (int m = 0; m < NDIR; ++m) {
            or_targets_t T;
            or_move(M, A, v, x, y, z, m, &T);
            int nz_in_row = 0;
            for (int n = 0; n < NDIR; ++n)
                nz_in_row += C[m * NDIR + n] != 0.0;
            for (int i = 0; i < T.count; ++i)
                cnt[T.row[i]] += nz_in_row;
        }
    }
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)A->n_rows + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)A->n_rows);
    if (!start || !fill) {
        free(cnt);
        free(start);
        free(fill);
        goto fail;
    }
    start[0] = 0;
    for (int64_t r = 0; r < A->n_rows; ++r)
        start[r + 1] = start[r] + cnt[r];
    free(cnt);
    int64_t cap = start[A->n_rows];
    A->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    A->val = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
    if (!A->col || !A->val) {
        free(start);
        free(fill);
        goto fail;
    }
    for (int64_t r = 0; r < A->n_rows; ++r)
        fill[r] = start[r];

    /* pass 2: push every column, merging adjacent equal columns */
    for (int64_t v = 0; v < V; ++v) {
        int x = (int)(v % M->nx), y = (int)((v / M->nx) % M->ny), z = (int)(v / ((int64_t)M->nx * M->ny));
        const double *C = Cq + (int64_t)M->mat_of_voxel[v] * NDIR * NDIR;
        or_targets_t T[NDIR];
        for (int m = 0; m < NDIR; ++m)
            or_move(M, A, v, x, y, z, m, &T[m]);
        for (int n = 0; n < NDIR; ++n) {
            int32_t c = (int32_t)(NDIR * v + n);
            for (int m = 0; m < NDIR; ++m) {
                double w = C[m * NDIR + n];
                if (w == 0.0) continue;
                for (int i = 0; i < T[m].count; ++i) {
                    int64_t r = T[m].row[i];
                    double a = T[m].f[i] * w;
                    if (fill[r] > start[r] && A->col[fill[r] - 1] == c) {
                        A->val[fill[r] - 1] += a;
                    } else {
                        A->col[fill[r]] = c;
                        A->val[fill[r]] = a;
                        fill[r]++;
                    }
                }
            }
        }
    }

    /* compact rows (merging may have left gaps) */
    A->row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)A->n_rows + 1));
    if (!A->row_ptr) {
        free(start);
        free(fill);
        goto fail;
    }
    int64_t w = 0;
    A->row_ptr[0] = 0;
    for (int64_t r = 0; r < A->n_rows; ++r) {
        for (int64_t j = start[r]; j < fill[r]; ++j) {
            if (A->val[j] == 0.0) continue;
            A->col[w] = A->col[j];
            A->val[w] = A->val[j];
            ++w;
        }
        A->row_ptr[r + 1] = w;
    }
    A->nnz = w;
    free(start);
    free(fill);
    free(Cq);
    return A;
fail:
    free(Cq);
    or_free(A);
    return NULL;
}

int64_t or_n_vox(const or_csr_t *A) { return A->n_vox; }
int64_t or_n_states(const or_csr_t *A) { return A->n_states; }
int64_t or_n_escape(const or_csr_t *A) { return A->n_escape; }
int64_t or_n_rows(const or_csr_t *A) { return A->n_rows; }
int64_t or_nnz(const or_csr_t *A) { return A->nnz; }
int or_n_dir(const or_csr_t *A) { return A->n_dir; }
const int64_t *or_row_ptr(const or_csr_t *A) { return A->row_ptr; }
const int32_t *or_col(const or_csr_t *A) { return A->col; }
const double *or_val(const or_csr_t *A) { return A->val; }
const double *or_absorb_of_voxel(const or_csr_t *A) { return A->absorb_of_voxel; }

/* row index of state s = n_dir v + m (escape = 0) or of its escape row (escape = 1);
 * -1 when the state does not leave the grid */
int64_t or_row_of(const or_csr_t *A, int64_t s, int escape)
{
    if (!escape) return s;
    int32_t e = A->escape_of_state[s];
    return e < 0 ? -1 : A->n_states + e;
}

/* ---- FP32 values ----------------------------------------------------------- */

static uint64_t or_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/*
 * FP64 -> FP32 value rounding.  mode 0: round to nearest even.  mode 1:
 * unbiased deterministic rounding: with r the nearest float and r' the other
 * float neighbour of a, r' is taken with probability p = |r - a| / |r' - r|,
 * the uniform variate being splitmix64((row << 32) ^ col) >> 11 scaled by
 * 2^-53.  The expected stored value is a, so the rounding of A is unbiased.
 */
void or_round_f32(const or_csr_t *A, int mode, float *out)
{
    for (int64_t r = 0; r < A->n_rows; ++r) {
        for (int64_t j = A->row_ptr[r]; j < A->row_ptr[r + 1]; ++j) {
            double a = A->val[j];
            float f = (float)a;
            if (mode == 1 && (double)f != a) {
                float f2 = nextafterf(f, (double)f < a ? INFINITY : -INFINITY);
                double p = fabs((double)f - a) / fabs((double)f2 - (double)f);
                uint64_t key = ((uint64_t)r << 32) ^ (uint64_t)(uint32_t)A->col[j];
                double u = (double)(or_splitmix64(key) >> 11) * 0x1p-53;
                if (u < p) f = f2;
            }
            out[j] = f;
        }
    }
}

/* ---- time stepping ----------------------------------------------------------- */

/* Threads of the SpMV loop (OpenMP) for the calls that follow; n < 1 leaves
 * the runtime's default.  Only the timing of the oracle uses it: the row sums
 * are the same sequential sums with any number of threads. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* y = A x over all rows (state rows then escape rows), each row summed in
 * ascending column order; vals32 replaces the FP64 values when not NULL */
void or_spmv(const or_csr_t *A, const float *vals32, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n_rows; ++r) {
        double acc = 0.0;
        for (int64_t j = A->row_ptr[r]; j < A->row_ptr[r + 1]; ++j) {
            double a = vals32 ? (double)vals32[j] : A->val[j];
            acc += a * x[A->col[j]];
        }
        y[r] = acc;
    }
}

static int or_exponent(double m)
{
    int e = 0;
    if (m > 0.0) frexp(m, &e);
    return e;
}

/*
 * Runs n_steps of J(t+1) = A J(t) + s(t) (Eq. (26)).  The state is kept as
 * 2^E x with max |x| in [0.5, 1) after every step (exact rescaling).
 *
 * Sources: entry i adds src_w[i] * amp[t * n_src + src_id[i]] to row
 * src_row[i] after the product of step t.
 * Detectors: M_d(t) = sum over entries with det_id d of det_F * J_row(t+1).
 * Outputs per step t (value, exponent pairs; physical = value * 2^exponent):
 *   tot[3t+0] = total of the state after the step, N(t+1)
 *   tot[3t+1] = escaped during the step (sum of the escape rows)
 *   tot[3t+2] = absorbed during the step, sum_v (1 - alpha_v) sum_n J(t)
 *   det[n_det t + d] = M_d(t)
 * x0 (may be NULL = zero state) is the initial state times 2^-e0; on return
 * x_out holds the final state times 2^-(*e_out).
 */
int or_run(const or_csr_t *A, const float *vals32, int64_t n_steps,
           const double *x0, int32_t e0,
           int64_t n_src_e, const int64_t *src_row, const int32_t *src_id, const double *src_w,
           int32_t n_src, const double *amp,
           int64_t n_det_e, const int64_t *det_row, const int32_t *det_id, const double *det_F,
           int32_t n_det,
           double *tot, int32_t *tot_exp, double *det, int32_t *det_exp,
           double *x_out, int32_t *e_out)
{
    int64_t R = A->n_rows, D = A->n_states;
    double *x = (double *)calloc((size_t)R, sizeof(double));
    double *y = (double *)calloc((size_t)R, sizeof(double));
    double *s = (double *)calloc((size_t)R, sizeof(double));
    if (!x || !y || !s) {
        free(x);
        free(y);
        free(s);
        return -1;
    }
    int E = 0;
    if (x0) {
        memcpy(x, x0, sizeof(double) * (size_t)D);
        E = e0;
    }
    for (int64_t t = 0; t < n_steps; ++t) {
        /* absorbed during this step, from the state entering it */
        double absorbed = 0.0;
        for (int64_t v = 0; v < A->n_vox; ++v) {
            double sv = 0.0;
            for (int n = 0; n < A->n_dir; ++n)
                sv += x[(int64_t)A->n_dir * v + n];
            absorbed += A->absorb_of_voxel[v] * sv;
        }
        tot[3 * t + 2] = absorbed;
        tot_exp[3 * t + 2] = E;

        or_spmv(A, vals32, x, y);

        /* source vector of this step (physical scale) */
        double smax = 0.0;
        for (int64_t i = 0; i < n_src_e; ++i)
            s[src_row[i]] += src_w[i] * amp[t * n_src + src_id[i]];
        for (int64_t i = 0; i < n_src_e; ++i)
            if (fabs(s[src_row[i]]) > smax) smax = fabs(s[src_row[i]]);
        double ymax = 0.0;
        for (int64_t r = 0; r < D; ++r)
            if (fabs(y[r]) > ymax) ymax = fabs(y[r]);
        int En = E;
        if (ymax > 0.0) En = E + or_exponent(ymax);
        if (smax > 0.0 && (ymax == 0.0 || or_exponent(smax) > En)) En = or_exponent(smax);
        for (int64_t r = 0; r < R; ++r)
            y[r] = ldexp(y[r], E - En);
        for (int64_t i = 0; i < n_src_e; ++i) {
            int64_t r = src_row[i];
            if (s[r] != 0.0) {
                y[r] += ldexp(s[r], -En);
                s[r] = 0.0;
            }
        }
        E = En;

        double N = 0.0, esc = 0.0;
        for (int64_t r = 0; r < D; ++r)
            N += y[r];
        for (int64_t r = D; r < R; ++r)
            esc += y[r];
        tot[3 * t + 0] = N;
        tot_exp[3 * t + 0] = E;
        tot[3 * t + 1] = esc;
        tot_exp[3 * t + 1] = E;
        for (int d = 0; d < n_det; ++d) {
            det[n_det * t + d] = 0.0;
            det_exp[n_det * t + d] = E;
        }
        for (int64_t i = 0; i < n_det_e; ++i)
            det[n_det * t + det_id[i]] += det_F[i] * y[det_row[i]];

        for (int64_t r = 0; r < D; ++r)
            x[r] = y[r];
    }
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)D);
    if (e_out) *e_out = E;
    free(x);
    free(y);
    free(s);
    return 0;
}

/* ---- sources -------------------------------------------------------------- */

/* time step of the lattice: the voxel edge h (mm) crossed at c0 / n_ref */
double or_dt_seconds(double h_mm, double n_ref)
{
    return h_mm * 1e-3 * n_ref / 299792458.0;
}

/*
 * Photons a normalised Gaussian pulse of full width at half maximum fwhm
 * (centred at 3 sigma) emits during step t, [t dt, (t+1) dt), with the lower
 * limit of step 0 taken to -infinity so the steps sum to one (the source
 * integrated over the step, Sec. 4.1).
 */
double or_gaussian_step(double fwhm_s, double dt_s, int64_t t)
{
    double sigma = fwhm_s / (2.0 * sqrt(2.0 * log(2.0)));
    double tc = 3.0 * sigma;
    double k = sigma * sqrt(2.0);
    double lo = (t == 0) ? 2.0 : erfc(((double)t * dt_s - tc) / k);
    double hi = erfc(((double)(t + 1) * dt_s - tc) / k);
    return 0.5 * (lo - hi);
}

/* the splitmix64 finaliser, exposed so that it can be checked against its
 * published output sequence */
uint64_t or_splitmix64_value(uint64_t x) { return or_splitmix64(x); }

/* ==== Lebedev-86 directions with multi-voxel weights (Sec. 3, Eq. (18)-(21)) ==== */

#define NLEB 86

/*
 * Lebedev's 86-point quadrature rule on the unit sphere (exact for spherical
 * polynomials of degree 15), built from its published generators:
 *   a1: the 6 points (+-1, 0, 0) and permutations
 *   a3: the 8 points (+-r, +-r, +-r), r = sqrt(1/3)
 *   b_k: the 24 points (+-l, +-l, +-m) and permutations, m = sqrt(1 - 2 l^2),
 *        for two values of l
 *   c_1: the 24 points (+-p, +-q, 0) and permutations, q = sqrt(1 - p^2)
 * Weights are normalised to sum to one.  The points are ordered by ascending
 * z, then y, then x (the direction index of a state).
 */
static const double OR_LEB_A1 = 0.1154401154401154e-1;
static const double OR_LEB_A3 = 0.1194390908585628e-1;
static const double OR_LEB_B_L[2] = {0.3696028464541502, 0.6943540066026664};
static const double OR_LEB_B_W[2] = {0.1111055571060340e-1, 0.1187650129453714e-1};
static const double OR_LEB_C_P = 0.3742430390903412;
static const double OR_LEB_C_W = 0.1181230374690448e-1;

static int or_leb_add(double S[NLEB][3], double w[NLEB], int k, double x, double y, double z, double wt)
{
    S[k][0] = x;
    S[k][1] = y;
    S[k][2] = z;
    w[k] = wt;
    return k + 1;
}

/* all sign combinations of (a, b, c), skipping signs of zero components */
static int or_leb_signs(double S[NLEB][3], double w[NLEB], int k, double a, double b, double c, double wt)
{
    for (int sa = -1; sa <= 1; sa += 2)
        for (int sb = -1; sb <= 1; sb += 2)
            for (int sc = -1; sc <= 1; sc += 2) {
                if ((a == 0.0 && sa < 0) || (b == 0.0 && sb < 0) || (c == 0.0 && sc < 0)) continue;
                k = or_leb_add(S, w, k, sa * a, sb * b, sc * c, wt);
            }
    return k;
}

static int or_leb_before(const double *a, const double *b)
{
    if (a[2] != b[2]) return a[2] < b[2];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[0] < b[0];
}

void or_lebedev86(double *S_out /* [86][3] */, double *w_out /* [86] */)
{
    double S[NLEB][3], w[NLEB];
    int k = 0;
    k = or_leb_signs(S, w, k, 1.0, 0.0, 0.0, OR_LEB_A1);
    k = or_leb_signs(S, w, k, 0.0, 1.0, 0.0, OR_LEB_A1);
    k = or_leb_signs(S, w, k, 0.0, 0.0, 1.0, OR_LEB_A1);
    double r = sqrt(1.0 / 3.0);
    k = or_leb_signs(S, w, k, r, r, r, OR_LEB_A3);
    for (int i = 0; i < 2; ++i) {
        double l = OR_LEB_B_L[i], m = sqrt(1.0 - 2.0 * l * l);
        k = or_leb_signs(S, w, k, l, l, m, OR_LEB_B_W[i]);
        k = or_leb_signs(S, w, k, l, m, l, OR_LEB_B_W[i]);
        k = or_leb_signs(S, w, k, m, l, l, OR_LEB_B_W[i]);
    }
    double p = OR_LEB_C_P, q = sqrt(1.0 - p * p);
    k = or_leb_signs(S, w, k, p, q, 0.0, OR_LEB_C_W);
    k = or_leb_signs(S, w, k, q, p, 0.0, OR_LEB_C_W);
    k = or_leb_signs(S, w, k, p, 0.0, q, OR_LEB_C_W);
    k = or_leb_signs(S, w, k, q, 0.0, p, OR_LEB_C_W);
    k = or_leb_signs(S, w, k, 0.0, p, q, OR_LEB_C_W);
    k = or_leb_signs(S, w, k, 0.0, q, p, OR_LEB_C_W);
    /* insertion sort by (z, y, x) */
    for (int i = 1; i < NLEB; ++i) {
        double t[3] = {S[i][0], S[i][1], S[i][2]}, tw = w[i];
        int j = i - 1;
        while (j >= 0 && or_leb_before(t, S[j])) {
            S[j + 1][0] = S[j][0];
            S[j + 1][1] = S[j][1];
            S[j + 1][2] = S[j][2];
            w[j + 1] = w[j];
            --j;
        }
        S[j + 1][0] = t[0];
        S[j + 1][1] = t[1];
        S[j + 1][2] = t[2];
        w[j + 1] = tw;
    }
    double sum = 0.0;
    for (int i = 0; i < NLEB; ++i)
        sum += w[i];
    for (int i = 0; i < NLEB; ++i) {
        S_out[3 * i + 0] = S[i][0];
        S_out[3 * i + 1] = S[i][1];
        S_out[3 * i + 2] = S[i][2];
        w_out[i] = w[i] / sum;
    }
}

/*
 * Direction block of one material over the 86 directions, for a step in
 * which light travels L = c dt (mm):
 *   P0 = exp(-mu_s L), Ps = 1 - P0, alpha = exp(-mu_a L)          (Eq. (9)-(10))
 *   G[m][n] = w_m p(S_m . S_n) / sum_k w_k p(S_k . S_n)           (kernel g of Eq. (19),
 *             the quadrature weights w of the rule measuring the solid angle of each direction)
 *   C[m][n] = alpha (Ps G[m][n]), C[n][n] = alpha (P0 + Ps G[n][n])   (Eq. (21))
 */
void or_lebedev_block(double mu_s, double mu_a, double g, double L, const double *S, const double *wq,
                      double *C /* [86*86] */)
{
    double P0 = exp(-mu_s * L);
    double Ps = 1.0 - P0;
    double alpha = exp(-mu_a * L);
    for (int n = 0; n < NLEB; ++n) {
        double p[NLEB];
        double Z = 0.0;
        for (int m = 0; m < NLEB; ++m) {
            double cs = S[3 * m] * S[3 * n] + S[3 * m + 1] * S[3 * n + 1] + S[3 * m + 2] * S[3 * n + 2];
            p[m] = wq[m] * or_hg(g, cs);
        }
        for (int k = 0; k < NLEB; ++k)
            Z += p[k];
        for (int m = 0; m < NLEB; ++m) {
            double G = p[m] / Z;
            C[m * NLEB + n] = (m != n) ? alpha * (Ps * G) : alpha * (P0 + Ps * G);
        }
    }
}

/* distance from point P to the segment from a to b (a point when a == b) */
static double or_seg_dist(const double P[3], const double a[3], const double b[3])
{
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ap[3] = {P[0] - a[0], P[1] - a[1], P[2] - a[2]};
    double L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
    double t = 0.0;
    if (L2 > 0.0) {
        t = (ap[0] * ab[0] + ap[1] * ab[1] + ap[2] * ab[2]) / L2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double q[3] = {a[0] + t * ab[0], a[1] + t * ab[1], a[2] + t * ab[2]};
    double d[3] = {P[0] - q[0], P[1] - q[1], P[2] - q[2]};
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/*
 * Multi-voxel weights of Eq. (18)-(19).  Voxel centres are the lattice points
 * (spacing h) and the partition spheres have radius dr = h/2, so 2 dr is one
 * voxel.  A population of voxel X_i in direction S_n that leaves in
 * direction S_m arrives, after the step, spread over the voxels X_j whose
 * centres lie within 2 dr of the segment AB, A = X_i + c dt S_m,
 * B = X_i + c dt S_n (for m = n the segment is the point B: the unscattered
 * population of Eq. (18) together with the zero-angle scatter of Eq. (21)),
 * with weights (2 dr - d(X_j, AB)) / sum_k (2 dr - d(X_k, AB)).  In voxel
 * units: offsets delta = X_j - X_i, distance below 1, weight (1 - d) / sum.
 * The weights depend only on (m, n) and the offset; offsets are scanned in
 * ascending (dz, dy, dx) over the box [-R, R]^3, R = ceil(c + 1), and the sum
 * is taken in that order.
 */
typedef struct {
    int R;
    int64_t ptr[NLEB * NLEB + 1]; /* pair (m, n) -> entries ptr[m*86+n] .. ptr[m*86+n+1]-1 */
    int8_t *off;                  /* [entries][3] */
    double *w;                    /* [entries] */
} or_stencil_t;

static or_stencil_t *or_stencil(const double *S, double c)
{
    or_stencil_t *T = (or_stencil_t *)calloc(1, sizeof(or_stencil_t));
    if (!T) return NULL;
    T->R = (int)ceil(c + 1.0);
    int R = T->R, B = 2 * R + 1;
    int64_t cap = (int64_t)NLEB * NLEB * B * B * B;
    int8_t *off = (int8_t *)malloc((size_t)cap * 3);
    double *w = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!off || !w) {
        free(off);
        free(w);
        free(T);
        return NULL;
    }
    int64_t k = 0;
    double raw[1024];
    for (int m = 0; m < NLEB; ++m)
        for (int n = 0; n < NLEB; ++n) {
            double a[3] = {c * S[3 * m], c * S[3 * m + 1], c * S[3 * m + 2]};
            double b[3] = {c * S[3 * n], c * S[3 * n + 1], c * S[3 * n + 2]};
            T->ptr[m * NLEB + n] = k;
            int cnt = 0;
            double sum = 0.0;
            for (int dz = -R; dz <= R; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        double P[3] = {(double)dx, (double)dy, (double)dz};
                        double d = or_seg_dist(P, a, b);
                        if (d < 1.0) {
                            off[3 * (k + cnt) + 0] = (int8_t)dx;
                            off[3 * (k + cnt) + 1] = (int8_t)dy;
                            off[3 * (k + cnt) + 2] = (int8_t)dz;
                            raw[cnt] = 1.0 - d;
                            sum += raw[cnt];
                            ++cnt;
                        }
                    }
            for (int i = 0; i < cnt; ++i)
                w[k + i] = raw[i] / sum;
            k += cnt;
        }
    T->ptr[NLEB * NLEB] = k;
    T->off = off;
    T->w = w;
    return T;
}

static void or_stencil_free(or_stencil_t *T)
{
    if (!T) return;
    free(T->off);
    free(T->w);
    free(T);
}

/* the host tables of a Lebedev medium, shared by the push assembly and the
 * single-row function */
typedef struct {
    int nx, ny, nz;
    int64_t V, D;
    double S[NLEB * 3], wq[NLEB];
    double *Cq;             /* [n_mat][86][86] */
    const uint8_t *mat;
    or_stencil_t *st;
    int8_t *m_out;          /* [86][(2R+1)^3]: 1 when some n puts direction m at that offset */
    int32_t *escape_of_state; /* [D], escape row index - D, or -1 */
    int64_t n_escape;
    double *absorb_of_voxel;
} or_leb_t;

static int or_leb_inside(const or_leb_t *L, int x, int y, int z)
{
    return x >= 0 && x < L->nx && y >= 0 && y < L->ny && z >= 0 && z < L->nz;
}

static void or_leb_free(or_leb_t *L)
{
    if (!L) return;
    free(L->Cq);
    or_stencil_free(L->st);
    free(L->m_out);
    free(L->escape_of_state);
    free(L->absorb_of_voxel);
    free(L);
}

static or_leb_t *or_leb_model(const or_medium_t *M)
{
    or_leb_t *L = (or_leb_t *)calloc(1, sizeof(or_leb_t));
    if (!L) return NULL;
    L->nx = M->nx;
    L->ny = M->ny;
    L->nz = M->nz;
    L->V = (int64_t)M->nx * M->ny * M->nz;
    L->D = NLEB * L->V;
    L->mat = M->mat_of_voxel;
    or_lebedev86(L->S, L->wq);
    double c = M->c_dt > 0.0 ? M->c_dt : 1.0;
    double Lmm = c * M->h_mm;
    L->Cq = (double *)malloc(sizeof(double) * NLEB * NLEB * M->n_mat);
    L->st = or_stencil(L->S, c);
    int R = L->st ? L->st->R : 0, B = 2 * R + 1;
    L->m_out = (int8_t *)calloc((size_t)NLEB * B * B * B, 1);
    L->escape_of_state = (int32_t *)malloc(sizeof(int32_t) * (size_t)L->D);
    L->absorb_of_voxel = (double *)malloc(sizeof(double) * (size_t)L->V);
    if (!L->Cq || !L->st || !L->m_out || !L->escape_of_state || !L->absorb_of_voxel) {
        or_leb_free(L);
        return NULL;
    }
    for (int q = 0; q < M->n_mat; ++q)
        or_lebedev_block(M->mat[4 * q], M->mat[4 * q + 1], M->mat[4 * q + 2], Lmm, L->S, L->wq,
                         L->Cq + (int64_t)q * NLEB * NLEB);
    /* offsets any column can send direction m to */
    for (int m = 0; m < NLEB; ++m)
        for (int n = 0; n < NLEB; ++n)
            for (int64_t e = L->st->ptr[m * NLEB + n]; e < L->st->ptr[m * NLEB + n + 1]; ++e) {
                const int8_t *o = L->st->off + 3 * e;
                L->m_out[(int64_t)m * B * B * B + ((o[2] + R) * B + (o[1] + R)) * B + (o[0] + R)] = 1;
            }
    /* escape rows: (v, m) such that some offset of direction m leaves the grid */
    int64_t ne = 0;
    for (int64_t v = 0; v < L->V; ++v) {
        int x = (int)(v % L->nx), y = (int)((v / L->nx) % L->ny), z = (int)(v / ((int64_t)L->nx * L->ny));
        L->absorb_of_voxel[v] = -expm1(-M->mat[4 * M->mat_of_voxel[v] + 1] * Lmm);
        for (int m = 0; m < NLEB; ++m) {
            int out = 0;
            for (int i = 0; i < B * B * B && !out; ++i) {
                if (!L->m_out[(int64_t)m * B * B * B + i]) continue;
                int dx = i % B - R, dy = (i / B) % B - R, dz = i / (B * B) - R;
                out = !or_leb_inside(L, x + dx, y + dy, z + dz);
            }
            L->escape_of_state[NLEB * v + m] = out ? (int32_t)(ne++) : -1;
        }
    }
    L->n_escape = ne;
    return L;
}

/*
 * Push assembly of [A; L] for a Lebedev medium.  For every column (v, n) in
 * ascending order, every arrival direction m in ascending order and every
 * offset of the pair's stencil in its scan order, the value
 * w_{nm}(offset) C_q(v)[m][n] goes to row (v + offset, m) when that voxel is
 * inside the grid; the weights of the offsets outside the grid are summed (in
 * scan order) and their total times C_q(v)[m][n] goes to the escape row of
 * (v, m).  A column reaches each row at most once, so every entry is one
 * product.  Exact zeros are not stored.
 */
or_csr_t *or_build_lebedev(const or_medium_t *M)
{
    or_leb_t *L = or_leb_model(M);
    if (!L) return NULL;
    or_csr_t *A = (or_csr_t *)calloc(1, sizeof(or_csr_t));
    int64_t *cnt = NULL, *fill = NULL;
    if (!A) goto fail;
    A->n_dir = NLEB;
    A->n_vox = L->V;
    A->n_states = L->D;
    A->n_escape = L->n_escape;
    A->n_rows = L->D + L->n_escape;
    A->escape_of_state = L->escape_of_state;
    A->absorb_of_voxel = L->absorb_of_voxel;
    L->escape_of_state = NULL;
    L->absorb_of_voxel = NULL;
    cnt = (int64_t *)calloc((size_t)A->n_rows + 1, sizeof(int64_t));
    if (!cnt) goto fail;
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t v = 0; v < L->V; ++v) {
            int x = (int)(v % L->nx), y = (int)((v / L->nx) % L->ny), z = (int)(v / ((int64_t)L->nx * L->ny));
            const double *C = L->Cq + (int64_t)L->mat[v] * NLEB * NLEB;
            for (int n = 0; n < NLEB; ++n) {
                int32_t col = (int32_t)(NLEB * v + n);
                for (int m = 0; m < NLEB; ++m) {
                    double cmn = C[m * NLEB + n];
                    if (cmn == 0.0) continue;
                    double esc = 0.0;
                    int any_out = 0;
                    for (int64_t e = L->st->ptr[m * NLEB + n]; e < L->st->ptr[m * NLEB + n + 1]; ++e) {
                        const int8_t *o = L->st->off + 3 * e;
                        int ux = x + o[0], uy = y + o[1], uz = z + o[2];
                        if (or_leb_inside(L, ux, uy, uz)) {
                            int64_t r = NLEB * ((int64_t)ux + (int64_t)L->nx * ((int64_t)uy + (int64_t)L->ny * uz)) + m;
                            double a = L->st->w[e] * cmn;
                            if (a == 0.0) continue;
                            if (pass == 0) {
                                cnt[r]++;
                            } else {
                                A->col[fill[r]] = col;
                                A->val[fill[r]] = a;
                                fill[r]++;
                            }
                        } else {
                            esc += L->st->w[e];
                            any_out = 1;
                        }
                    }
                    if (any_out) {
                        int64_t r = A->n_states + A->escape_of_state[NLEB * v + m];
                        double a = esc * cmn;
                        if (a == 0.0) continue;
                        if (pass == 0) {
                            cnt[r]++;
                        } else {
                            A->col[fill[r]] = col;
                            A->val[fill[r]] = a;
                            fill[r]++;
                        }
                    }
                }
            }
        }
        if (pass == 0) {
            A->row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)A->n_rows + 1));
            fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)A->n_rows + 1));
            if (!A->row_ptr || !fill) goto fail;
            A->row_ptr[0] = 0;
            for (int64_t r = 0; r < A->n_rows; ++r)
                A->row_ptr[r + 1] = A->row_ptr[r] + cnt[r];
            A->nnz = A->row_ptr[A->n_rows];
            for (int64_t r = 0; r < A->n_rows; ++r)
                fill[r] = A->row_ptr[r];
            A->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A->nnz > 0 ? A->nnz : 1));
            A->val = (double *)malloc(sizeof(double) * (size_t)(A->nnz > 0 ? A->nnz : 1));
            if (!A->col || !A->val) goto fail;
        }
    }
    free(cnt);
    free(fill);
    or_leb_free(L);
    return A;
fail:
    free(cnt);
    free(fill);
    or_leb_free(L);
    or_free(A);
    return NULL;
}

/* ---- single rows of a Lebedev medium, without assembling the matrix --------- */

void *or_leb_open(const or_medium_t *M) { return or_leb_model(M); }
void or_leb_close(void *h) { or_leb_free((or_leb_t *)h); }
int64_t or_leb_n_rows(const void *h) { return ((const or_leb_t *)h)->D + ((const or_leb_t *)h)->n_escape; }
int64_t or_leb_n_escape(const void *h) { return ((const or_leb_t *)h)->n_escape; }

/*
 * Entries of one row of [A; L] pulled from its sources (the same products as
 * the push assembly, so the same values): a state row (j, m) takes, from
 * every voxel i = j - offset and direction n whose stencil (m, n) holds the
 * offset, w C_q(i)[m][n]; an escape row (v, m) takes, per direction n, the
 * scan-order sum of the weights of the offsets leaving the grid times
 * C_q(v)[m][n].  Writes at most cap entries in ascending column order and
 * returns the row's entry count.
 */
int64_t or_leb_row(const void *h, int64_t row, int32_t *col, double *val, int64_t cap)
{
    const or_leb_t *L = (const or_leb_t *)h;
    int64_t k = 0;
    if (row < L->D) {
        int m = (int)(row % NLEB);
        int64_t j = row / NLEB;
        int jx = (int)(j % L->nx), jy = (int)((j / L->nx) % L->ny), jz = (int)(j / ((int64_t)L->nx * L->ny));
        for (int n = 0; n < NLEB; ++n)
            for (int64_t e = L->st->ptr[m * NLEB + n]; e < L->st->ptr[m * NLEB + n + 1]; ++e) {
                const int8_t *o = L->st->off + 3 * e;
                int ix = jx - o[0], iy = jy - o[1], iz = jz - o[2];
                if (!or_leb_inside(L, ix, iy, iz)) continue;
                int64_t i = (int64_t)ix + (int64_t)L->nx * ((int64_t)iy + (int64_t)L->ny * iz);
                double cmn = L->Cq[(int64_t)L->mat[i] * NLEB * NLEB + m * NLEB + n];
                double a = L->st->w[e] * cmn;
                if (cmn == 0.0 || a == 0.0) continue;
                if (k < cap) {
                    col[k] = (int32_t)(NLEB * i + n);
                    val[k] = a;
                }
                ++k;
            }
        /* ascending columns (insertion sort; rows hold a few hundred entries) */
        int64_t kk = k < cap ? k : cap;
        for (int64_t a = 1; a < kk; ++a) {
            int32_t c0 = col[a];
            double v0 = val[a];
            int64_t b = a - 1;
            while (b >= 0 && col[b] > c0) {
                col[b + 1] = col[b];
                val[b + 1] = val[b];
                --b;
            }
            col[b + 1] = c0;
            val[b + 1] = v0;
        }
        return k;
    }
    /* escape row: find its state */
    int64_t ei = row - L->D;
    int64_t s = -1;
    for (int64_t t = 0; t < L->D; ++t)
        if (L->escape_of_state[t] == ei) {
            s = t;
            break;
        }
    if (s < 0) return 0;
    int m = (int)(s % NLEB);
    int64_t v = s / NLEB;
    int x = (int)(v % L->nx), y = (int)((v / L->nx) % L->ny), z = (int)(v / ((int64_t)L->nx * L->ny));
    const double *C = L->Cq + (int64_t)L->mat[v] * NLEB * NLEB;
    for (int n = 0; n < NLEB; ++n) {
        double cmn = C[m * NLEB + n];
        if (cmn == 0.0) continue;
        double esc = 0.0;
        int any_out = 0;
        for (int64_t e = L->st->ptr[m * NLEB + n]; e < L->st->ptr[m * NLEB + n + 1]; ++e) {
            const int8_t *o = L->st->off + 3 * e;
            if (!or_leb_inside(L, x + o[0], y + o[1], z + o[2])) {
                esc += L->st->w[e];
                any_out = 1;
            }
        }
        double a = esc * cmn;
        if (!any_out || a == 0.0) continue;
        if (k < cap) {
            col[k] = (int32_t)(NLEB * v + n);
            val[k] = a;
        }
        ++k;
    }
    return k;
}

/* the stencil of one pair (m, n) for the pins: count, offsets [cnt][3], weights */
int64_t or_leb_stencil(const void *h, int m, int n, int32_t *off, double *w, int64_t cap)
{
    const or_leb_t *L = (const or_leb_t *)h;
    int64_t b = L->st->ptr[m * NLEB + n], e = L->st->ptr[m * NLEB + n + 1];
    for (int64_t i = b; i < e && i - b < cap; ++i) {
        off[3 * (i - b) + 0] = L->st->off[3 * i + 0];
        off[3 * (i - b) + 1] = L->st->off[3 * i + 1];
        off[3 * (i - b) + 2] = L->st->off[3 * i + 2];
        w[i - b] = L->st->w[i];
    }
    return e - b;
}

/* the direction block of material q of an open Lebedev medium */
void or_leb_block(const void *h, int q, double *C)
{
    const or_leb_t *L = (const or_leb_t *)h;
    memcpy(C, L->Cq + (int64_t)q * NLEB * NLEB, sizeof(double) * NLEB * NLEB);
}
