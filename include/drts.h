/*
 * drts.h -- C ABI of the MI355X (gfx950) implementation of the Dynamic
 * Radiative Transfer System (DRTS) time step.
 *
 * The method (Georgakopoulos, Politopoulos, Georgiou, arXiv 1611.08536):
 * photons in a scattering and absorbing medium are counted per state
 * (voxel X_i, direction S_n).  One time step dt maps the state vector J to
 *     J(t + dt) = A J(t) + B P(t)                                   (Eq. 26)
 * where A (Eq. 21/23) is a time-independent sparse matrix built once from the
 * medium, and B P(t) injects the photons that sources emit during the step
 * (Sec. 4.1).  Detectors read weighted sums of J (Eq. 27, one-step window).
 *
 * Discretisation implemented here (Sec. 3 allows any space and direction
 * partition):
 *   - cubic voxels of edge h, voxel index v = x + nx (y + ny z);
 *   - the 26 lattice directions e = (dx,dy,dz) in {-1,0,1}^3 \ {0}, indexed
 *     d = k - (k > 13) with k = 9(dz+1) + 3(dy+1) + (dx+1);
 *   - state index s = 26 v + d (the 26 directions of a voxel are contiguous);
 *   - dt = h n_ref / c0, so light crosses one voxel per step;
 *   - in one step the population of (v, n) leaves v with direction m with
 *     probability C_q(v)[m][n] (single-scatter split Eq. (9)-(10),
 *     Henyey-Greenstein kernel Eq. (19), forward scatter on the diagonal
 *     Eq. (21)) and arrives at (v + e_m, m);
 *   - crossing into a voxel of different refractive index splits the
 *     population by the unpolarised Fresnel reflectance (Sec. 4.2): the
 *     reflected part stays in v with the lattice direction nearest the
 *     specular direction, the transmitted part enters v + e_m with the
 *     lattice direction nearest the Snell direction (directions tied within
 *     1e-12 in cosine share a part evenly);
 *   - at vacuum faces the population leaving the grid is collected in escape
 *     rows (row index >= n_states), so the matrix is [A; L] with
 *     n_rows = n_states + n_escape rows; at reflecting faces every leaving
 *     component of e_m is reversed and the population stays in v.
 *
 * Numbers: coefficients are computed in FP64 on the host.  The matrix values
 * are stored in FP64 or FP32 (round to nearest, or the unbiased "dither"
 * rounding DRTS_ROUND_DITHER).  FP32 states are kept as 2^E * x with a
 * per-right-hand-side power-of-two exponent E chosen every step (exact
 * scaling), so femtosecond-pulse runs spanning 1e20 and more never underflow.
 * Totals and detector sums are accumulated in FP64 in a fixed order (results
 * are bitwise reproducible run to run).
 *
 * Conventions of every call:
 *   - return 0 on success, a negative DRTS_E_* code on failure; the message
 *     of the last failure of the calling thread is drts_last_error();
 *   - no C++ exception crosses this interface;
 *   - handles are opaque, owned by the library, freed by their *_destroy;
 *   - host arrays passed in are read during the call only (copied);
 *   - device memory is allocated through the caller's drts_device_t hooks
 *     (or hipMalloc when the hooks are NULL) and all work is enqueued on the
 *     hook's stream (or the null stream); calls that return host data
 *     synchronise that stream.
 */
#ifndef DRTS_H
#define DRTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define DRTS_OK 0
#define DRTS_E_INVALID (-1) /* malformed argument or medium */
#define DRTS_E_NOMEM (-2)   /* an allocation (device or host) failed */
#define DRTS_E_HIP (-3)     /* a HIP runtime call failed */
#define DRTS_E_RANGE (-4)   /* an index or step count exceeds what was sized */
#define DRTS_E_STATE (-5)   /* call not valid in the handle's current state */

/* ---- enumerations -------------------------------------------------------- */
#define DRTS_GEOM_VOXELS 0   /* interfaces use normal incidence along e_m */
#define DRTS_GEOM_LAYERS_Z 1 /* planar layers stacked along z, normal +-z */
#define DRTS_GEOM_SPHERE 2   /* sphere: normal radial at the step midpoint */

#define DRTS_BC_VACUUM 0  /* leaving photons go to escape rows */
#define DRTS_BC_REFLECT 1 /* specular walls, nothing leaves */

#define DRTS_F64 0
#define DRTS_F32 1

#define DRTS_ROUND_NEAREST 0 /* FP64 -> FP32 values: IEEE round to nearest */
#define DRTS_ROUND_DITHER 1  /* unbiased: the other float neighbour r' of a is
                                taken iff u < |r - a| / |r' - r|, where
                                u = (splitmix64((row << 32) ^ col) >> 11) 2^-53 */

/* ---- medium ---------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz; /* voxels per axis, each >= 1 */
    double h_mm;        /* voxel edge = c dt, in mm */
} drts_grid_t;

typedef struct {
    double mu_s; /* scattering coefficient, 1/mm (Eq. 2) */
    double mu_a; /* absorption coefficient, 1/mm (Eq. 8) */
    double g;    /* Henyey-Greenstein anisotropy, -1 < g < 1 */
    double n;    /* refractive index (Sec. 4.2) */
} drts_material_t;

typedef struct {
    int32_t kind;            /* DRTS_GEOM_* : rule for interface normals */
    double sphere_c[3];      /* DRTS_GEOM_SPHERE: centre, voxel units, voxel
                                (x,y,z) has its centre at (x+.5, y+.5, z+.5) */
    double sphere_r;         /* DRTS_GEOM_SPHERE: radius, voxel units */
    int32_t n_layers;        /* DRTS_GEOM_LAYERS_Z: number of layers */
    const int32_t *layer_z0; /* DRTS_GEOM_LAYERS_Z: first z of each layer,
                                ascending, layer_z0[0] == 0; layer i uses
                                material i */
} drts_geometry_t;

typedef struct {
    drts_grid_t grid;
    int32_t n_mat;               /* 1..255 */
    const drts_material_t *mat;  /* host [n_mat] */
    const uint8_t *mat_of_voxel; /* host [nx*ny*nz] material id per voxel, or
                                    NULL: derived from geom (LAYERS_Z: layer of
                                    z; SPHERE: material 1 where the voxel centre
                                    lies within the sphere, else 0) */
    drts_geometry_t geom;
    int32_t bc;         /* DRTS_BC_* */
    int32_t value_type; /* DRTS_F64 | DRTS_F32 */
    int32_t rounding;   /* DRTS_ROUND_* (DRTS_F32 only) */
    double n_ref;       /* refractive index that sets dt = h n_ref / c0 */
    int32_t scatter_order; /* scatterings within one step that the direction
                              block resolves (Eq. 4): 0 or 1 = at most one
                              (Eq. 6-7: every scattered photon changes
                              direction once); K in 2..16 = the Poisson
                              weights of 0..K-1 scatterings with powers of the
                              scattering kernel (a sequence of single
                              scatterings), the remaining probability taking
                              K scatterings */
    int32_t directions;    /* DRTS_DIRS_*: the angular partition (Sec. 3) */
    double c_dt;           /* DRTS_DIRS_LEBEDEV86: the distance light travels
                              per step, in voxels (0 = 1); dt = c_dt h n_ref / c0.
                              Must be 0 or 1 with the lattice directions */
    int32_t interface_model; /* DRTS_INTERFACE_*: how a move crossing into a
                              voxel of another refractive index is treated */
} drts_medium_t;

/* Interface crossings (Sec. 4.2), lattice directions:
 *   DRTS_INTERFACE_ORIGIN   the whole step uses the source voxel's medium; the
 *                           reflected part stays in its voxel;
 *   DRTS_INTERFACE_SUBSTEP  the crossing happens a fraction f of the way
 *                           between the voxel centres (1/2 at planar layers and
 *                           voxel faces; where the segment meets the surface
 *                           for a sphere): the transmitted part is absorbed
 *                           along its path in each medium,
 *                           T exp(-mu_a1 f h - mu_a2 (1 - f) h) instead of
 *                           T exp(-mu_a1 h); at planar layers the reflected
 *                           part lands one voxel over along the surface,
 *                           v + (dx, dy, 0) (in v when that voxel lies outside
 *                           the grid).  Scattering stays at the step's origin. */
#define DRTS_INTERFACE_ORIGIN 0
#define DRTS_INTERFACE_SUBSTEP 1

/* Angular partitions (Sec. 3 allows any):
 *   DRTS_DIRS_LATTICE26  the 26 lattice directions above: every population
 *                        moves to the neighbour voxel e_m in one step;
 *   DRTS_DIRS_LEBEDEV86  Lebedev's 86-point rule (degree 15), the paper's own
 *                        choice, with the multi-voxel weights of Eq. (18)-(19):
 *                        partition spheres of radius dr = h/2 on the voxel
 *                        centres; a population of X_i in direction S_n leaving
 *                        in direction S_m (Eq. 21) arrives spread over the
 *                        voxels whose centres lie within 2 dr of the segment
 *                        from X_i + c dt S_m to X_i + c dt S_n (a point when
 *                        m = n), weighted by the normalised ramp 2 dr - d; the
 *                        scattering kernel weighs each direction by the rule's
 *                        solid angle.  States index 86 v + n with the
 *                        directions in ascending (z, y, x) order
 *                        (drts_direction_set).  Vacuum faces, one refractive
 *                        index, scatter_order 0 or 1, 0 < c_dt <= 8 voxels;
 *                        the CSR step kernels only (not the matrix-free ones,
 *                        not the serving loop).  Rows hold several hundred
 *                        entries. */
#define DRTS_DIRS_LATTICE26 0
#define DRTS_DIRS_LEBEDEV86 1

/* Unit vectors [n][3] and solid-angle weights [n] (summing to one; 1/26 each
 * for the lattice) of an angular partition; either output may be NULL.
 * Returns the number of directions, or DRTS_E_INVALID. */
int drts_direction_set(int32_t directions, double *unit, double *weight);

/* ---- device hooks ---------------------------------------------------------- */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream); /* NULL on failure */
    void (*free)(void *ctx, void *ptr, void *stream);
    void *stream; /* hipStream_t every kernel and copy is enqueued on */
} drts_device_t;

/* ---- sources: s(t) = B P(t) (Eq. 26) ------------------------------------------ */
/* Ownership: the library keeps the table's address, never a copy.  A solver
 * calls support() when it is first handed a table and stages the result; on
 * later calls it recognises the table by its address, ctx and n_src and calls
 * only amplitude().  A caller that changes what support() returns therefore
 * passes a table at another address or with another ctx.  The table and its
 * ctx stay valid while a solver may still run with it, and until a submitted
 * serving request has finished. */
typedef struct {
    void *ctx;
    int32_t n_src; /* number of source functions */
    /* Spatial/directional support of source src: writes up to cap (state,
     * weight) pairs and returns how many it has (the library calls again with a
     * larger buffer when the return value exceeds cap).  States index
     * 26 v + d (< n_states). */
    int64_t (*support)(void *ctx, int32_t src, int64_t *state, double *w, int64_t cap);
    /* Photons source src emits during step `step` (between step dt and
     * (step+1) dt); t0_s = step * dt_s.  Called on the host. */
    double (*amplitude)(void *ctx, int32_t src, int64_t step, double t0_s, double dt_s);
    /* Right-hand side (column of the multi-source state) that src feeds;
     * may be NULL when the solver has one right-hand side. */
    int32_t (*rhs_of)(void *ctx, int32_t src);
} drts_source_table_t;

/* Pulse shapes for amplitude() (Sec. 4.1, Eq. 26 with a time profile that
 * varies within a step): the photons of a pulse of unit total emitted during
 * step `step`, i.e. its time profile integrated over [step dt, (step+1) dt).
 *   DRTS_PULSE_IMPULSE   every photon in step 0;
 *   DRTS_PULSE_GAUSSIAN  a Gaussian of full width at half maximum fwhm_s
 *                        seconds with its peak at three standard deviations;
 *                        step 0 also takes the (tiny) part before t = 0, so
 *                        the steps sum to one.  Evaluated with erfc, so the
 *                        tails carry no cancellation. */
#define DRTS_PULSE_IMPULSE 0
#define DRTS_PULSE_GAUSSIAN 1
typedef struct {
    int32_t kind;  /* DRTS_PULSE_* */
    double fwhm_s; /* Gaussian: full width at half maximum, seconds (> 0) */
} drts_pulse_t;

/* Photons pulse p emits during step `step` of length dt_s seconds.  Host
 * function, no device work.  Returns NaN for a NULL or unknown pulse, a
 * Gaussian with fwhm_s <= 0, dt_s <= 0 or step < 0 (and sets the last
 * error). */
double drts_pulse_step(const drts_pulse_t *p, int64_t step, double dt_s);

/* ---- detectors: M_d(t) = sum F J (Eq. 27 with a one-step window) --------------- */
typedef struct {
    int32_t n_det;
    const int64_t *det_ptr; /* host [n_det+1]: entries of detector d are
                               det_ptr[d] .. det_ptr[d+1]-1 */
    const int64_t *state;   /* host: state index 26 v + d */
    const uint8_t *escape;  /* host: 1 = the escape row of that state (the
                               photons leaving the grid from it during the
                               step), 0 = the state itself after the step */
    const double *F;        /* host: weight */
} drts_detectors_t;

typedef struct drts_matrix drts_matrix_t;
typedef struct drts_solver drts_solver_t;
typedef struct drts_batch drts_batch_t;
typedef struct drts_server drts_server_t;

/* ---- matrix ------------------------------------------------------------------- */

/* Assembles [A; L] (Eq. 21/23 plus escape rows) on the device, once per
 * medium (Fig. 3: "build A").  Coefficient tables are computed on the host in
 * FP64; the CSR is filled on the device (int32 columns, int32 or int64 row
 * pointers, FP64 or FP32 values).  Errors: DRTS_E_INVALID (bad sizes,
 * materials or geometry), DRTS_E_RANGE (more than 2^31 - 1 states),
 * DRTS_E_NOMEM, DRTS_E_HIP. */
int drts_build_matrix(const drts_medium_t *medium, const drts_device_t *dev, drts_matrix_t **out);

/* Sizes of an assembled matrix; any output pointer may be NULL.  bytes = device
 * bytes of the CSR (row pointers, columns, values) and, once a solo solver
 * has asked for the grouped step, of the row groups (descriptors, members'
 * rows and materials, values in group order, the fast and listed rows, the
 * two-voxel rows' copy, the value-indexed slots, dictionaries and bricks);
 * dt_s in seconds. */
int drts_matrix_info(const drts_matrix_t *A, int64_t *n_states, int64_t *n_escape, int64_t *nnz,
                     int64_t *bytes, double *dt_s);

/* The row groups of an assembled matrix (rows whose column lists are equal),
 * built when a solo solver first runs a grouped step, and how the single-rhs
 * grouped step takes the rows:
 *   n_groups        groups (of at most 26 rows);
 *   n_fast          fast groups: full lattice rows, 26 columns that are one
 *                   voxel's states (one run), formed by row groups;
 *   n_vox2_rows     two-voxel rows (52 columns in two runs of 26, e.g. rows
 *                   that take a transmitted and a reflected part at an
 *                   interface), taken one by one from a compact copy of
 *                   their values, x read as the two runs;
 *   n_list_rows     all other rows (empty rows, other column patterns),
 *                   taken one by one from the CSR;
 *   n_list_entries  their entries;
 *   value_tables    > 0: the fast groups' values are value-indexed, one byte
 *                   per entry into value_tables dictionaries of at most 256
 *                   FP32 values (one per material: the material of the voxel
 *                   whose states are the group's columns), so the step
 *                   streams a quarter of the bytes and takes the same values;
 *                   0: a material's fast groups hold more than 256 distinct
 *                   values (or there are more than 16 materials) and the
 *                   values stream as FP32. */
typedef struct {
    int64_t n_groups, n_fast, n_vox2_rows, n_list_rows, n_list_entries, value_tables;
} drts_groups_info_t;

/* Fills *info.  DRTS_E_INVALID for a NULL argument; DRTS_E_STATE while the
 * groups are not built; all counts 0 when the rows do not group. */
int drts_matrix_groups(const drts_matrix_t *A, drts_groups_info_t *info);

/* Row index of state s (escape = 0 -> s itself; escape = 1 -> its escape row,
 * or -1 when the state does not leave the grid or faces reflect). */
int64_t drts_matrix_row_of(const drts_matrix_t *A, int64_t state, int32_t escape);

/* Host copy of rows [row0, row0 + n_rows): row_ptr[n_rows+1] (absolute entry
 * offsets), col[row_ptr[n_rows]-row_ptr[0]], val (double or float as stored).
 * Pass col = val = NULL to fetch row_ptr only.  Synchronises the stream. */
int drts_matrix_export_rows(const drts_matrix_t *A, int64_t row0, int64_t n_rows, int64_t *row_ptr,
                            int32_t *col, void *val);

void drts_matrix_destroy(drts_matrix_t *A);

/* ---- solver ------------------------------------------------------------------- */

#define DRTS_KERNEL_CSR 0        /* CSR SpMV / SpMM over the stored [A; L] */
#define DRTS_KERNEL_STRUCTURED 1 /* matrix-free: every entry re-derived from the
                                    per-voxel direction block and rounded as
                                    stored, so the result equals the CSR step's
                                    bit for bit (one rhs: any rounding; several
                                    rhs: nearest-rounded FP32 values only) */
#define DRTS_KERNEL_STRUCTURED_F64SUM 2 /* matrix-free, FP32 state: each row is
                                    the FP64 sum (in column order, one fma per
                                    term) of the FP64 coefficients times the
                                    FP32 x, rounded once to FP32; more accurate
                                    than either stored rounding, equal to the
                                    CSR step within rounding.  With several rhs
                                    each column equals the one-rhs result of
                                    this kernel bit for bit */

typedef struct {
    int32_t kernel;       /* DRTS_KERNEL_* */
    int32_t rows_per_tile; /* rows a workgroup reduces per tile (64..256) */
    int32_t tiles_per_chunk; /* tiles whose sums form one FP64 partial */
    int32_t grid;         /* persistent workgroups (0 = from the device) */
    int32_t xcd_remap;    /* 0 = workgroups walk the chunks round robin;
                             1 = each XCD takes a contiguous range of chunks
                             in row order; 2 = as 1, with the chunks ordered
                             so that each XCD's range is one slab of y lines
                             swept in z (its x gathers stay in its L2) */
    int32_t graph_steps;  /* steps captured per hipGraph replay (0 = eager) */
    int32_t rescale;      /* 1 = power-of-two rescale every step (default) */
    int32_t variant;      /* n_rhs > 1: DRTS_SPMM_GROUPED, DRTS_SPMM_ROWS or
                             DRTS_SPMM_GROUPED_F64SUM;
                             one rhs: DRTS_SPMV_ROW, DRTS_SPMV_LDS or
                             DRTS_SPMV_GROUPED (below) */
    int32_t queue;        /* one rhs only: 1 = workgroups take chunks from a
                             device counter (dynamic balance), 0 = fixed walk */
} drts_options_t;

/* One rhs: the tiled step, a thread per row and its tile's entries staged in
 * LDS -- through registers (DRTS_SPMV_ROW, the default for FP64 values) or
 * loaded straight into LDS (DRTS_SPMV_LDS, FP32 values) -- or the step by
 * row groups (DRTS_SPMV_GROUPED, FP32 values, the default for them): rows
 * whose column lists are equal form groups (as for DRTS_SPMM_GROUPED); a
 * half-wave forms a fast group (26 columns in one run), reading x at the run
 * once and the values from a group-order copy the matrix keeps once a solo
 * solver asks for it; two-voxel rows (two runs) take a thread each over a
 * compact copy of their values, every other row a thread over its CSR entries
 * (drts_matrix_groups counts them).  Batch members of the shared launch
 * take DRTS_SPMV_LDS, and so does a matrix whose rows do not group.  All give
 * the same state bit for bit. */
#define DRTS_SPMV_ROW 0
#define DRTS_SPMV_LDS 1
#define DRTS_SPMV_GROUPED 2
/* n_rhs > 1: rows whose column lists are equal (on a lattice, the rows that
 * pull from one source voxel) share one gather of their right-hand-side rows
 * (the default; the library takes the row-by-row step for a matrix whose
 * rows do not group, at least two rows a group on average), or every row
 * gathers its own.  Both give the same result bit for bit, and each column
 * equals the single-rhs step's.  DRTS_SPMM_GROUPED_F64SUM is the step by row
 * groups with each row summed in FP64 (one fma per term in column order; the
 * product of two FP32 numbers is exact there) and rounded once to FP32: the
 * FP32 accumulation error no longer builds up over long runs (the rounding of
 * the stored values and of the state stays).  It needs rows that group:
 * drts_solver_set_options builds the matrix's groups when they are not built
 * yet, and returns DRTS_E_INVALID (options unchanged) when its rows do not
 * group or hold several hundred entries. */
#define DRTS_SPMM_GROUPED 0
#define DRTS_SPMM_ROWS 1
#define DRTS_SPMM_GROUPED_F64SUM 2

/* Creates the time-stepping state for n_rhs right-hand sides sharing A: the
 * state (zero), detectors, series buffers for max_steps steps.  n_rhs > 1
 * selects the SpMM kernels (FP32 matrices only).  det may be NULL. */
int drts_solver_create(const drts_matrix_t *A, int32_t n_rhs, const drts_detectors_t *det,
                       int64_t max_steps, const drts_device_t *dev, drts_solver_t **out);

int drts_solver_get_options(const drts_solver_t *S, drts_options_t *opt);
int drts_solver_set_options(drts_solver_t *S, const drts_options_t *opt);

/* One step J <- A J + B P(t) (Eq. 26), t += 1.  Calls src->amplitude for the
 * current step only.  Returns once the step's amplitudes are copied to the
 * device (which waits for work already queued on the stream), without
 * waiting for the step itself. */
int drts_step(drts_solver_t *S, const drts_source_table_t *src);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same step as
 * drts_step -- same kernels, same results bit for bit -- whose scratch memory
 * (the device copy of the step descriptor, the work counter of the dynamic
 * walk and the per-chunk FP64 partials of the totals and detectors) lives in
 * a fixed 16 MiB device array of the library instead of the solver's
 * buffers.  It allocates nothing, device or host.  Each GPU that runs it
 * holds its own copy of the array until the process ends; the call looks up
 * that copy's address on the current device (which must be the solver's) the
 * first time it runs there.  Every call on one GPU shares the array and the
 * call rewrites what it reads (descriptor, counter, partials) before reading
 * it, so nothing carries over from a previous call; calls that overlap on one
 * GPU (two host threads, or two streams with work in flight) race and must
 * not be issued.  Errors: DRTS_E_STATE when src is not the source table
 * already staged in the solver (staging another table allocates: hand it to
 * drts_step or drts_run once first; a solver created without sources accepts
 * src = NULL); DRTS_E_RANGE when the step's partials exceed the array
 * (16 MiB - 4 KiB: (4 + n_det) x n_rhs x (chunks + 256) doubles; use more
 * tiles per chunk, or drts_step) or beyond max_steps; DRTS_E_HIP. */
int drts_step_noalloc(drts_solver_t *S, const drts_source_table_t *src);

/* n_steps steps.  Calls src->amplitude for all of them up front, then
 * replays hipGraphs of graph_steps steps (no host synchronisation inside).
 * n_steps = 0 only stages the source table (its support is read and
 * uploaded), which a later drts_step_noalloc requires.
 * DRTS_E_RANGE when t + n_steps exceeds max_steps.  Returns once the
 * amplitudes are copied (as drts_step), without waiting for the steps. */
int drts_run(drts_solver_t *S, const drts_source_table_t *src, int64_t n_steps);

/* Current step count (synchronises). */
int drts_solver_time(const drts_solver_t *S, int64_t *t);

/* FP64 series of steps [first, first + count): for step t and right-hand side
 * k the physical values are value * 2^exp2[t][k]:
 *   series[t][d][k]  detector d (Eq. 27)             may be NULL
 *   totals[t][0][k]  photons in the grid after the step      may be NULL
 *   totals[t][1][k]  photons that left during the step
 *   totals[t][2][k]  photons absorbed during the step
 *   exp2[t][k]                                       may be NULL
 * Synchronises the stream. */
int drts_detector_readout(const drts_solver_t *S, int64_t first, int64_t count, double *series,
                          int32_t *exp2, double *totals);

/* Windowed measurement (Eq. 27 with a window of several steps, Sec. 4.2): a
 * sensor responds to the photons reaching it through its impulse response,
 * so its reading at step t is the per-step detector sum m_d (the series of
 * drts_detector_readout) filtered by that response:
 *     M_d(t) = sum_{j=0}^{n_taps-1} taps[d][j] m_d(t - tap0 - j)
 * taps: host [n_det][n_taps], detector d's response at delays
 * tap0 .. tap0 + n_taps - 1 steps (tap0 < 0 lets a reading include later
 * steps, the symmetric window of Eq. 27).  Steps outside 0 .. t - 1 of the
 * solver's current step count t contribute nothing.  Output for steps
 * [first, first + count): out[t][d][k] * 2^out_exp[t][d][k] (host arrays),
 * computed on the device in FP64 (each reading's terms brought to the largest
 * exponent among them, added in ascending tap order).  Synchronises the
 * stream; device memory for the taps and the output comes from the solver's
 * hooks during the call.  Errors: DRTS_E_INVALID (no detectors, n_taps
 * outside 1..65536, NULL arrays), DRTS_E_RANGE (steps beyond max_steps). */
int drts_detector_window(const drts_solver_t *S, const double *taps, int32_t n_taps, int32_t tap0, int64_t first,
                         int64_t count, double *out, int32_t *out_exp);

/* State transfer for checkpoint/resume (bit-exact): host_x is
 * [n_rows][n_rhs] in the value type (state rows, then the escape rows of the
 * last step), exp2[n_rhs], t.  state_write zeroes nothing else and keeps the
 * series recorded so far. */
int drts_state_read(const drts_solver_t *S, void *host_x, int32_t *exp2, int64_t *t);
int drts_state_write(drts_solver_t *S, const void *host_x, const int32_t *exp2, int64_t t);

/* Kernel timing with HIP events around every launch of the step kernel
 * (enable = 1 also disables graph replay); stats return the launch count and
 * the summed milliseconds since the last enable. */
int drts_solver_profile(drts_solver_t *S, int32_t enable);
int drts_solver_profile_stats(drts_solver_t *S, int64_t *launches, double *total_ms);

void drts_solver_destroy(drts_solver_t *S);

/* ---- uneven batch: independent solvers in one persistent launch --------------- */

/* Groups n single-rhs FP32 solvers (different matrices and sizes) so that one
 * launch per step advances all of them.  A CSR member of at least 512 * 1024
 * rows whose options ask for the step by row groups (the default) keeps that
 * step: its launches go to one of the batch's auxiliary streams (forked from
 * the batch's stream and joined back around each run, so that the members'
 * launch gaps overlap; such a batch launches without graph capture); the
 * others take the tiled step and share one launch.
 * Each solver keeps its own state, exponent and series; results equal those
 * of the solver run alone with the same step, bit for bit.  The solvers must
 * outlive the batch. */
int drts_batch_create(drts_solver_t *const *solvers, int32_t n, const drts_device_t *dev,
                      drts_batch_t **out);

/* Advances solver i by n_steps[i] steps (0 = idle) with source table src[i];
 * solvers that finish drop out of later launches.  Every member must use the
 * same step (DRTS_E_INVALID otherwise): the CSR step (kernel option
 * DRTS_KERNEL_CSR, the same rows_per_tile for the members of the shared
 * launch), or the matrix-free step
 * with direction-major tiles (DRTS_KERNEL_STRUCTURED on nearest-rounded
 * values, or DRTS_KERNEL_STRUCTURED_F64SUM; at most 8 materials), whose two
 * kernels then each cover every member in one launch per step. */
int drts_batch_run(drts_batch_t *B, const drts_source_table_t *const *src, const int64_t *n_steps);

/* Chooses one shape for the batch's shared launch (rows per tile, tiles per
 * chunk, kernel variant, workgroups of the step launch) by timing a few
 * steps of its members at once for each candidate, then restores every
 * member's state and control words and keeps the fastest shape in those
 * members' options (chosen, may be NULL, receives it; its grid is the
 * batch's); members with their own grouped step keep their options.  Before the first step of every member (DRTS_E_STATE otherwise)
 * and for CSR members only (DRTS_E_INVALID otherwise); results stay equal to
 * solo runs with the same options, bit for bit. */
int drts_batch_autotune(drts_batch_t *B, drts_options_t *chosen);

void drts_batch_destroy(drts_batch_t *B);

/* ---- serving: continuous batching of independent solves ----------------------- */

/* A request loop over the uneven batch, for many media solved at once.
 * Submitted requests wait in arrival order.  Each tick
 *   1. admits waiting requests whose HBM footprint fits the budget beside the
 *      requests already admitted, first-fit in the policy's order (arrival,
 *      or least work first; a request that has been passed over max_skips
 *      times stops the ones after it from being admitted ahead of it), and
 *      assembles their matrices on the device (the host model built at
 *      submission is reused);
 *   2. advances every admitted request by up to `quantum` steps in batched
 *      launches: one launch per step covers all of them, so their work
 *      overlaps on the device;
 *   3. retires the requests that have finished: their series go to host
 *      memory and their device memory is freed, which lets the next tick
 *      admit more.
 * The footprint of a request is its matrix [A; L] (an upper bound from the
 * medium before assembly, the exact size after), two state buffers, its
 * series and its source table.  CSR requests take the tiled step, all of
 * them in the batch's shared launch.  Results equal those of the same solve
 * run alone (drts_run) with the same step, bit for bit.  budget_bytes > 0; 1 <= quantum <= 100000;
 * 1 <= max_active <= 4096; max_skips >= 0; policy DRTS_SERVE_*.
 * drts_serve_submit may be called from any thread, also while another call
 * on the same server runs (it builds the request's host model before it
 * takes the server's lock), so a client can keep submitting while a tick
 * runs on the device; the other calls on one server must not overlap each
 * other, and drts_serve_destroy must not overlap any call. */
#define DRTS_SERVE_ARRIVAL 0  /* waiting requests are considered in arrival order */
#define DRTS_SERVE_SHORTEST 1 /* ... in order of work (entries x steps), least first */

int drts_serve_create(const drts_device_t *dev, int64_t budget_bytes, int32_t quantum, int32_t max_active,
                      int32_t max_skips, int32_t policy, drts_server_t **out);

/* Selects the step of the requests admitted from now on: DRTS_KERNEL_CSR
 * (the default: all CSR requests advance together, one batched launch per
 * step) or a matrix-free kernel (DRTS_KERNEL_STRUCTURED or
 * DRTS_KERNEL_STRUCTURED_F64SUM, with 8 tiles per chunk and 16 workgroups
 * per CU): the matrix-free requests that a batch takes (FP64 row sums, or
 * exact values when nearest-rounded; at most 8 materials) advance together
 * as a second batch, any other runs its quantum with its own graph-replayed
 * drts_run, all in turn on the server's stream.  A served result equals the
 * same solve run alone with the same options, bit for bit.  The matrix is still
 * assembled (and counted in the footprint).  DRTS_E_INVALID for another
 * kernel.  Thread-safe like drts_serve_submit. */
int drts_serve_set_step(drts_server_t *Q, int32_t kernel);

/* Queues one solve of n_steps steps: an FP32 medium (its host arrays are
 * copied), its sources (the table must stay valid until the request has
 * finished) and detectors (copied; NULL for none).  Ids increase in the
 * order the calls start, and that is the arrival order of the queue, also
 * when calls on several threads overlap.  DRTS_E_NOMEM when the request's
 * footprint exceeds the whole budget; DRTS_E_INVALID for an FP64 medium or
 * a malformed argument. */
int drts_serve_submit(drts_server_t *Q, const drts_medium_t *medium, const drts_source_table_t *src,
                      const drts_detectors_t *det, int64_t n_steps, int64_t *request_id);

/* The footprint bound drts_serve_submit admits a request by, without
 * queueing it (host work only: no device memory is touched). */
int drts_serve_footprint(const drts_medium_t *medium, const drts_source_table_t *src, const drts_detectors_t *det,
                         int64_t n_steps, int64_t *bytes);

/* One tick (admit, run one quantum, retire); returns once the quantum's
 * launches have completed.  Outputs (each may be NULL): requests admitted
 * and waiting after the tick, requests finished during it, and the device
 * bytes the admitted requests hold. */
int drts_serve_tick(drts_server_t *Q, int32_t *n_active, int32_t *n_waiting, int32_t *n_finished,
                    int64_t *bytes_in_use);

/* Ids of finished requests not reported before, in the order they finished;
 * at most cap of them, *n_out receives the count. */
int drts_serve_poll(drts_server_t *Q, int64_t *ids, int32_t cap, int32_t *n_out);

/* Series of a finished request over all its steps, laid out as in
 * drts_detector_readout (series [n_steps][n_det], exp2 [n_steps], totals
 * [n_steps][3]); any output may be NULL.  DRTS_E_STATE before it finishes,
 * DRTS_E_INVALID for an unknown or released id. */
int drts_serve_result(const drts_server_t *Q, int64_t request_id, double *series, int32_t *exp2,
                      double *totals);

/* Forgets a finished request (its host copy of the results). */
int drts_serve_release(drts_server_t *Q, int64_t request_id);

void drts_serve_destroy(drts_server_t *Q);

/* ---- autotuning ------------------------------------------------------------------- */

/* Times the candidate launch shapes on the solver's own matrix (a few steps
 * each, state restored afterwards) and keeps the fastest as its options.
 * cache_path (may be NULL) is a text file of "key options" lines read before
 * and appended after tuning; the key is the size class of the problem. */
int drts_autotune(drts_solver_t *S, const char *cache_path, drts_options_t *chosen);

const char *drts_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DRTS_H */
