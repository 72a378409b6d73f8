// Internal declarations of the DRTS library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "drts.h"

namespace drts {

constexpr int kDirs = 26;

// ---- lattice ---------------------------------------------------------------
// Direction d <-> lattice vector: k = 9(dz+1) + 3(dy+1) + (dx+1), d = k - (k>13).
__host__ __device__ inline int dir_dx(int d) { int k = d + (d >= 13); return k % 3 - 1; }
__host__ __device__ inline int dir_dy(int d) { int k = d + (d >= 13); return (k / 3) % 3 - 1; }
__host__ __device__ inline int dir_dz(int d) { int k = d + (d >= 13); return k / 9 - 1; }
__host__ __device__ inline int dir_of(int dx, int dy, int dz)
{
    int k = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
    return k - (k > 13);
}

// ---- errors ----------------------------------------------------------------
int set_error(int code, const char *fmt, ...);
const char *hip_name(hipError_t e);

#define DRTS_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::drts::set_error(DRTS_E_HIP, "%s failed: %s (%s:%d)", #call,            \
                                     ::drts::hip_name(e_), __FILE__, __LINE__);             \
    } while (0)

// ---- device memory through the caller's hooks --------------------------------
struct Device {
    drts_device_t hooks{};
    hipStream_t stream = nullptr;
    void *alloc(size_t bytes);  // nullptr on failure (error message set)
    void free(void *p);
};

// Typed device buffer that releases itself through the hooks.
struct Buffer {
    Device *dev = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
    Buffer() = default;
    Buffer(const Buffer &) = delete;
    Buffer &operator=(const Buffer &) = delete;
    ~Buffer() { reset(); }
    int allocate(Device *d, size_t n);  // DRTS_OK or DRTS_E_NOMEM
    void reset();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// ---- host model of a medium (coefficient tables, escape and interface lists) ----
struct Model {
    int nx = 0, ny = 0, nz = 0;
    int64_t n_vox = 0, n_states = 0, n_escape = 0, n_rows = 0;
    double h_mm = 0, dt_s = 0;
    int bc = DRTS_BC_VACUUM;
    int value_type = DRTS_F32, rounding = DRTS_ROUND_DITHER;
    int scatter_order = 1;                  // scatterings per step resolved by the blocks
    int n_dir = kDirs;                      // directions per voxel: 26 (lattice) or 86 (Lebedev)
    double c_dt = 1.0;                      // light path per step, in voxels
    // Lebedev-86 (n_dir = 86): the rule, and the multi-voxel weights of every
    // direction pair (m, n): offsets within one voxel of the arrival segment
    // in scan order (ascending dz, dy, dx) with their weights ...
    std::vector<double> dir_unit, dir_w;    // [86][3], [86]
    std::vector<int64_t> pair_ptr;          // [86*86 + 1], pair m*86+n
    std::vector<uint32_t> pair_key;         // packed offset
    std::vector<double> pair_w;
    // ... and, per arrival direction m, every (offset, n) it receives from, in
    // descending (dz, dy, dx) then ascending n: a row pulls its entries in
    // ascending column order
    std::vector<int64_t> arr_ptr;           // [86 + 1]
    std::vector<uint32_t> arr_key;          // packed offset | n << 15
    std::vector<double> arr_w;
    std::vector<drts_material_t> mats;
    std::vector<uint8_t> mat_of_voxel;      // [n_vox]
    std::vector<double> blocks;             // [n_mat][26][26] C_q[m][n]
    std::vector<double> absorb;             // [n_mat] 1 - exp(-mu_a h)
    std::vector<double> index;              // [n_mat] refractive index
    std::vector<int64_t> escape_state;      // [n_escape] ascending states (v, m) leaving the grid
    // moves whose targets are not the plain neighbour: wall reflections and
    // interface splits, as (target row, source voxel, direction, factor),
    // sorted by (row, voxel, direction)
    std::vector<int64_t> irr_row, irr_vox;
    std::vector<int32_t> irr_dir;
    std::vector<double> irr_f;
};

int build_model(const drts_medium_t *m, Model *out);

// Lebedev's 86-point rule (ascending z, y, x; weights summing to one).
void lebedev86(double *unit, double *weight);
// packed lattice offset of the Lebedev tables: (dx + 16) | (dy + 16) << 5 | (dz + 16) << 10
__host__ __device__ inline int off_dx(uint32_t k) { return (int)(k & 31u) - 16; }
__host__ __device__ inline int off_dy(uint32_t k) { return (int)((k >> 5) & 31u) - 16; }
__host__ __device__ inline int off_dz(uint32_t k) { return (int)((k >> 10) & 31u) - 16; }
__host__ __device__ inline int off_n(uint32_t k) { return (int)(k >> 15); }

// ---- assembled matrix ----------------------------------------------------------
struct Matrix {
    Device dev;
    Model model;
    int64_t nnz = 0;
    bool rp64 = false;       // int64 row pointers (nnz >= 2^31)
    bool has_csr = true;     // false: only the tables the matrix-free steps read were built
    Buffer row_ptr, col, val;
    Buffer mat_of_voxel, absorb, index, blocks64, blocks32;
    Buffer irr_row, irr_vox, irr_dir, irr_f, irr_bits, escape_state;
    Buffer pair_ptr, pair_key, pair_w, arr_ptr, arr_key, arr_w;   // Lebedev weights
    // rows with equal column lists (built on first use by a solo solver that
    // asks for the grouped step): per group a GroupDesc; per member (group
    // order) its row and material; the values in group order (column-major
    // within a group).  n_groups < 0 = not built, 0 = the rows do not group
    Buffer grp_desc, grp_row, grp_mat, grp_val;
    int64_t n_groups = -1;
    // for the single-rhs step: the fast groups (kSpmmUnroll columns in one
    // run, by index), the two-voxel rows (two runs: info and values, see
    // StepInst) and the rows of all other groups
    Buffer grp_fast, slow_rows, vox2_info, vox2_val;
    int64_t n_fast = 0, n_slow = 0, n_slow_nnz = 0, n_vox2 = 0;
    // the fast groups' values as one-byte indices into per-material
    // dictionaries (vi_ntab > 0; 0 = a material has more than kViDict
    // distinct values, or more than kViTabs materials: FP32 group values)
    Buffer vi_idx, vi_dict;
    int32_t vi_ntab = 0;
    // the fast list's bricks of kBrick^3 source voxels (the fast list is in
    // brick order): first fast index of each brick (n_brick + 1) and its
    // origin voxel
    Buffer brick_ptr, brick_org;
    int64_t n_brick = 0;
    // per fast group (fast-list order): first member, member count, first
    // column of its run, group index (int32 x 4), and per group its fast
    // index (-1: not a fast group), with value indexing
    Buffer vi_fdesc, vi_fast_of;
    int64_t bytes() const;         // the CSR arrays (and the row groups, once built)
    int64_t table_bytes() const;   // everything else on the device (tables of the model)
};

// with_csr = false builds only the tables the matrix-free steps read (and
// counts the entries the CSR would hold).
int assemble_on_device(Matrix *A, bool with_csr = true);
// Builds A's row groups once (no groups: n_groups = 0, when the matrix has
// no CSR, FP64 values, 2^31 rows or more, or fewer than two rows a group on
// average).
int row_groups(const Matrix &A);
// Per group of A one bit (words of 32): set when a member's row is in the
// ascending list rows[0 .. n) (device memory).
int group_flags(const Matrix &A, const int64_t *rows, int64_t n, uint32_t *bits, hipStream_t stream);
// bit f of fbits: bit gfast[f] of gbits (the source bits in fast-list order)
int fast_flags(const Matrix &A, const uint32_t *gbits, uint32_t *fbits, hipStream_t stream);

// ---- windowed measurement (Eq. 27 over several steps) --------------------------
struct WindowArgs {
    const double *ser_det;   // [max_steps][n_det][n_rhs]
    const int32_t *ser_exp;  // [max_steps][n_rhs]
    const double *taps;      // [n_det][n_taps]
    int32_t n_det, n_rhs, n_taps, tap0;
    int64_t first, count, t_done;
    double *out;             // [count][n_det][n_rhs]
    int32_t *out_exp;        // [count][n_det][n_rhs]
};
hipError_t launch_detector_window(const WindowArgs &a, hipStream_t stream);

// drts_build_matrix for a medium whose host model is already built (the
// model is moved into the matrix).
int build_matrix_from_model(Model &&model, const drts_device_t *dev, drts_matrix_t **out, bool with_csr = true);
// device bytes a matrix holds (CSR arrays and tables)
int64_t matrix_device_bytes(const drts_matrix_t *A);
// builds A's row groups now (row_groups) on A's stream
int matrix_row_groups(const drts_matrix_t *A);
// A CSR batch member (or served request) of at least this many rows takes its
// own step by row groups instead of the batch's shared tiled launch.  On one
// MI355X a solo grouped step costs about 60 us of launches plus about 10 ns
// per thousand rows, while in the shared launch a member costs its CSR bytes
// at about 4.5 TB/s, some 47 ns per thousand rows.  With the own steps spread
// over the batch's auxiliary streams their launch gaps overlap, which moves
// the break-even down: on 256 cubes of edge 16..64 thresholds of 256K to 768K
// rows with 7 or 15 streams all gave 26.6-27.0 thousand instance-steps/s
// (1.5M rows with 3 streams: 23.5 thousand).
constexpr int64_t kBatchOwnRows = 512 * 1024;
// moves a solver's work to another stream (after finishing what its current
// stream holds)
int solver_set_stream(drts_solver_t *S, hipStream_t stream);

}  // namespace drts
