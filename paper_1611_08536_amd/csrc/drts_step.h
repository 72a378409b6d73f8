// Device-side descriptors of the DRTS time step (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace drts {

// Slots of the per-chunk FP64 partials, each [n_rhs] wide.
enum : int { kSlotN = 0, kSlotEsc = 1, kSlotAbs = 2, kSlotMax = 3, kSlotDet = 4 };
// Segments of the first reduction level of the finalize kernels; the partials
// buffer holds [slots][n_chunks] chunk values followed by [slots][kFinSeg].
constexpr int kFinSeg = 256;
constexpr int kFinDetMax = 256;   // detectors per solver
constexpr int kXcdBounds = 9;     // XCDs + 1

// Everything the step and finalize kernels need of one solver.  Lives in
// device memory; the kernels read it with uniform (scalar) loads.
struct StepInst {
    // matrix [A; L]
    const void *row_ptr;
    const int32_t *col;
    const void *val;
    int64_t n_rows, n_states;
    int64_t nnz;            // entries of [A; L] (the arrays hold 4 more, zero)
    int32_t rp64;
    int32_t rows_per_tile;
    int64_t n_tiles;
    int32_t tiles_per_chunk;
    int32_t n_rhs;
    // state: x_t lives in buf[t & 1], the step writes buf[(t + 1) & 1];
    // layout [n_rows][n_rhs]
    void *buf0, *buf1;
    const uint8_t *mat;     // material of every voxel
    const double *absorb;   // per material: 1 - exp(-mu_a h)
    // sources, entries sorted by row then rhs; src_tile[k] = first entry of tile k
    const int32_t *src_tile;
    const int64_t *src_row;
    const int32_t *src_id;
    const int32_t *src_rhs;
    const double *src_w;
    const double *amp;      // [max_steps][n_src]
    const double *smax;     // [max_steps][n_rhs] bound of |s_t| per rhs
    int32_t n_src;
    // detectors, entries sorted by tile then row; det_tile[k] = first entry of tile k
    int32_t n_det;
    const int32_t *det_tile;
    const int64_t *det_row;
    const int32_t *det_id;
    const double *det_F;
    // control, one per rhs
    int64_t *t;             // [n_rhs] steps done
    int32_t *E;             // [n_rhs] exponent of x_t
    double *M;              // [n_rhs] max of the scaled state x_t
    double *abs_cur;        // [n_rhs] absorbed during step t (from x_t), scaled by 2^-E
    const int64_t *t_end;   // steps are skipped once t >= *t_end
    int32_t rescale;
    int32_t n_mat;          // entries of absorb
    uint64_t vox_mul;       // vox_mul_of(directions per voxel): row -> voxel
    int64_t max_steps;
    // the step by row groups: groups of rows with equal column lists (NULL =
    // none), described by grp[g]; the members' rows and materials and the
    // values in group order; grp_src bit g: a member of group g has sources
    const struct GroupDesc *grp;
    const int32_t *grp_row;
    const uint8_t *grp_mat;
    const float *grp_val;
    const uint32_t *grp_src;
    int64_t n_groups;
    // the single-rhs step by row groups: the fast groups (full lattice rows,
    // columns in one run) by index, then the rows of the other groups one by
    // one, whose partials start at index slow_part
    const int32_t *grp_fast;
    const int32_t *slow_rows;
    int64_t n_fast, n_slow, slow_part;
    // the two-voxel rows (columns two runs of a voxel's states each, kVox2Len
    // entries), taken apart from the row list: per row {row, first column of
    // the first run, first column of the second run, material} and its values
    // (kVox2Len per row, list order); their partials start at index vox2_part
    const int32_t *vox2_info;
    const float *vox2_val;
    int64_t n_vox2, vox2_part;
    // the fast groups' values as one-byte indices (NULL = read as FP32 in
    // group order) and the dictionaries they index ([vi_ntab][kViDict])
    const uint8_t *vi_idx;
    const float *vi_dict;
    int32_t vi_ntab;
    // bricks of the fast list: brick b holds fast groups brick_ptr[b] ..
    // brick_ptr[b + 1] - 1 and its window's first voxel is brick_org[b] -
    // (1, 1, 1) (voxel index of the brick's origin in brick_org); grid extents
    const int32_t *brick_ptr;
    const int32_t *brick_org;
    int64_t n_brick;
    int32_t grid_nx, grid_ny;
    // per fast group, in fast-list order: {first member, member count, first
    // column of its run, group}; per group its fast index (-1: not fast); the
    // source bits by fast index
    const int32_t *vi_fdesc;
    const int32_t *vi_fast_of;
    const uint32_t *grp_src_f;
    // det_direct: the detector sums come from their own kernel (a value per
    // detector and rhs after the finalize segments of the partials, see
    // det_direct_sums), which takes the detector entries grouped by detector,
    // rows ascending within each: detector d owns ddet_row/ddet_F
    // [ddet_ptr[d], ddet_ptr[d+1])
    int32_t det_direct;
    const int64_t *ddet_ptr, *ddet_row;
    const double *ddet_F;
    // partials [slot * n_rhs + rhs][n_chunks], then [slot * n_rhs + rhs][kFinSeg]
    double *partials;
    int64_t n_chunks;
    // series
    double *ser_tot;        // [max_steps][3][n_rhs]: N(t+1), escaped(t), absorbed(t)
    double *ser_det;        // [max_steps][n_det][n_rhs]
    int32_t *ser_exp;       // [max_steps][n_rhs]: exponent E_{t+1} of the above
    int32_t *ser_abs_exp;   // [max_steps][n_rhs]: exponent E_t of absorbed(t)
};

// Parts of a detector's entry list whose direct sums are formed apart (and
// added in part order by the finalize).
constexpr int kDetParts = 64;
// Bytes of a solver's partials buffer: [slots][n_rhs][n_chunks] chunk values,
// [slots][n_rhs][kFinSeg] finalize segments, then [n_det][kDetParts][n_rhs]
// direct detector sums.
inline size_t partials_bytes(int n_det, int n_rhs, int64_t n_chunks)
{
    const size_t slots = (size_t)(kSlotDet + n_det) * n_rhs;
    return (slots * (size_t)(n_chunks + kFinSeg) + (size_t)n_det * kDetParts * n_rhs) * sizeof(double);
}
__host__ __device__ inline double *det_direct_sums(double *partials, int n_det, int n_rhs, int64_t n_chunks)
{
    return partials + (size_t)(kSlotDet + n_det) * n_rhs * (size_t)(n_chunks + kFinSeg);
}

// Voxel of state row r (< 2^32): r / n_dir as the high half of r * mul with
// mul = ceil(2^64 / n_dir), exact for every r < 2^32 (the error of mul, below
// n_dir, moves r * mul by less than 2^64 / n_dir).
__device__ __forceinline__ int64_t vox_of(int64_t r, uint64_t mul) { return (int64_t)__umul64hi((uint64_t)r, mul); }
inline uint64_t vox_mul_of(int n_dir) { return ~0ull / (uint64_t)n_dir + 1ull; }

// One unit of work of a launch: chunk `chunk` of instance `inst`.
struct WorkItem {
    int32_t inst;
    int32_t chunk;
};

// Launch variant (bits 1..4 of xcd_remap) of the wave-per-row SpMV for rows of
// several hundred entries; chosen by the library for such matrices, not an
// option of the caller.
constexpr int kVariantLongRows = 3;
// mean entries per row from which a matrix takes the wave-per-row SpMV
constexpr int kLongRowMean = 96;

// Members of one row group at most (larger sets of equal rows are split).
constexpr int kGroupMax = 26;
constexpr int kVox2Run = 26;             // entries of each run of a two-voxel row
constexpr int kVox2Len = 2 * kVox2Run;   // entries of a two-voxel row
constexpr int kVox2Item = 256;           // two-voxel rows of one work item
constexpr int kStatePad = 32;            // padding entries after a single-rhs state buffer
// value-indexed fast groups: each member's kSpmmUnrollHost values as one-byte
// indices into its group's dictionary (kViDict FP32 values, at most kViTabs
// dictionaries), in a kViSlot-byte slot whose byte kViTabByte names the
// dictionary; a fast group's slots are kViBlock bytes in fast-list order
constexpr int kViSlot = 32;
constexpr int kViTabByte = 26;
constexpr int kViBlock = 26 * kViSlot;
constexpr int kViDict = 256;
constexpr int kViTabs = 16;
constexpr int kViHash = 4096;            // slots of a dictionary's build-time hash set
constexpr int kViPosByte = 27;           // slot byte: the group's position in its brick
constexpr int kViRowWord = 7;            // slot word (bytes 28..31): the member's row
// value-indexed fast groups are ordered in bricks of kBrick^3 source voxels;
// a workgroup forms a brick's groups and stages the rows they write into the
// brick's window of (kBrick + 2)^3 destination voxels in LDS, then writes the
// window out in address order
constexpr int kBrick = 4;
constexpr int kWin = kBrick + 2;
constexpr int kWinSlots = kWin * kWin * kWin * 26;
// Entries of a full lattice row (the grouped steps' fast path).
constexpr int kSpmmUnrollHost = 26;
// Rows a workgroup of the single-rhs row-list kernel takes per work item.
constexpr int kRowListItem = 256;

// One row group (rows with equal column lists): its members are grp_row and
// grp_mat [m0, m0 + nm), rows ascending; its values start at grp_val + voff,
// column-major (entry k of member j at k * nm + j, n entries a member); its
// columns are the leader's, col [coff, coff + n), or the run cstart,
// cstart + 1, ... when they are one (cstart = -1 otherwise).
struct alignas(16) GroupDesc {
    int64_t voff;
    int64_t coff;
    int32_t m0;
    int32_t nm;
    int32_t n;
    int32_t cstart;
};

// Launches the SpMV (n_rhs == 1) or SpMM step over a work list.  xcd_remap
// bit 0 selects the XCD-aware order, bit 1 the pipelined SpMV.  Returns a
// hipError_t.
// queue (may be NULL): a zeroed device counter from which the SpMV workgroups
// take work items; the finalize kernel resets it.
// spmm: 0 = one rhs, 1 = many rhs row by row, 2 = many rhs by row groups
// (work item c takes groups c * n_groups / n_chunks onwards), 3 = as 2 with
// each row summed in FP64 and rounded once to FP32.
// xcd_bounds (may be NULL): with the XCD-aware walk, XCD i takes work items
// xcd_bounds[i] .. xcd_bounds[i+1]-1 (kXcdBounds entries), else equal counts.
// n_slow, n_vox2: with the grouped single-rhs step, the rows it takes one by
// one from the CSR and its two-voxel rows; vi: the number of dictionaries of
// its value-indexed fast groups (0: FP32 values), plus 0x100 when a fast
// group holds a source row; with spmm 2 or 3 the number of dictionaries that
// the fast groups' values index (0: FP32 group values; spmm 3 reads them).
hipError_t launch_step(const StepInst *insts_dev, const WorkItem *work_dev, int64_t n_work, int n_inst,
                       int n_rhs_max, int value_f64, int rp64, int spmm, int grid, int xcd_remap,
                       const int64_t *xcd_bounds, int rows_per_tile, int n_det_max, int32_t *queue,
                       hipStream_t stream, int64_t n_slow = 0, int64_t n_vox2 = 0, int vi = 0);
hipError_t launch_finalize(const StepInst *insts_dev, int n_inst, int n_rhs_max, int n_det_max, int32_t *queue,
                           hipStream_t stream);

// Matrix-free step (single rhs): every row's entries are re-derived from the
// per-material direction blocks, the irregular-move list and the escape list
// (the rule the device assembly applies), rounded as the stored values are,
// and multiplied by x in column order -- the same result as the CSR step.
struct StructArgs {
    int nx, ny, nz;
    int rounding;              // DRTS_ROUND_* of the FP32 values
    int64_t n_states, n_rows;
    const uint8_t *mat;
    const double *index;       // refractive index per material
    const float *blocks32;     // [q][m][n], nearest-rounded
    const double *blocks64;    // [q][m][n]
    int32_t n_mat;
    const int64_t *irr_row, *irr_vox;
    const int32_t *irr_dir;
    const double *irr_f;
    const uint32_t *irr_bits;
    int64_t n_irr;
    const int64_t *escape_state;
    // tiling: voxel tiles, segments of seg_len voxels of one x-line,
    // segs_per_line of them per line, n_vox_tiles in all
    int32_t seg_len, segs_per_line;
    int64_t n_vox_tiles;
    // rows left to the second kernel: irregular rows and escape rows, in
    // ascending order; its work item j writes the partials of chunk
    // chunk_base + j
    const int64_t *xrows;
    const int64_t *xirr;       // [n_xrows + 1]: row k's irregular moves are xirr[k] .. xirr[k+1]-1
    const int32_t *xsrc;       // [n_xrows]: first source entry at or after row k (row-sorted list)
    const int32_t *xdet;       // [n_xrows]: first detector entry at or after row k
    const int64_t *xdrng;      // one rhs: [work item][detector][2], the item's range of the detector's entries
    const int64_t *zrows;      // many rhs: rows with no move and no source (value zero), written by the pull kernel
    int64_t n_zrows;
    int64_t n_xrows;
    int64_t chunk_base;
    // entries of the row-sorted source and detector lists
    int64_t n_src_entries, n_det_entries;
    // many right-hand sides: rows the push kernel leaves to the pull kernel,
    // one bit per row of [A; L]; and per voxel, the offset of its first
    // escape row from n_states (its escape rows follow in ascending m)
    const uint32_t *pull_bits;
    const int32_t *esc_base;
    // their grids: one set of partials per workgroup, push then pull
    int32_t mm_push_grid, mm_pull_grid;
    // detector entries grouped by detector, rows ascending within each:
    // detector d owns ddet_row/ddet_F [ddet_ptr[d], ddet_ptr[d+1])
    const int64_t *ddet_ptr, *ddet_row;
    const double *ddet_F;
};
constexpr int kStructSegLen = 16;         // voxels per tile of the gather kernel (modes 0 and 3)
constexpr int kStructDmSeg = 64;          // voxels per tile of the direction-major kernel (modes 1 and 2)
constexpr int kStructXRows = 256;     // rows per work item of the single-rhs second kernel
constexpr int kStructMatLdsHost = 8;      // materials the single-rhs direction-major kernel takes
constexpr int kStructVoxPerChunk = 64;   // voxels per work item of the push kernel
constexpr int kStructMmXRows = 64;       // rows per work item of the many-rhs pull kernel
// mode: 0 = exact values with global gathers, 1 = exact nearest values with
// the LDS halo, 2 = FP64 coefficients and FP64 row sums with the LDS halo,
// 3 = the same arithmetic with global gathers (more materials than the LDS
// holds)
hipError_t launch_structured(const StructArgs &sa, const StepInst *insts_dev, const WorkItem *work_dev,
                             int64_t n_work, int value_f64, int mode, int grid, int xcd_remap,
                             const int64_t *xcd_bounds, hipStream_t stream);

// Matrix-free step of an uneven batch in one launch per kernel (FP32, modes 1
// and 2: the direction-major tiles): sas_dev[i] holds instance i's arguments
// (each checked on the host as launch_structured checks its own), the work
// list (instance, chunk) covers the tiles of all active instances and the
// x list (instance, item) their irregular and escape rows.
hipError_t launch_structured_batch(const StructArgs *sas_dev, const StepInst *insts_dev, const WorkItem *work_dev,
                                   int64_t n_work, const WorkItem *xwork_dev, int64_t n_xwork, int mode, int grid,
                                   hipStream_t stream);

// Matrix-free step for n_rhs > 1 (FP32 state; mode 1 = exact nearest values,
// 2 = FP64 coefficients and FP64 row sums): the push kernel over the voxel
// chunks of the work list, then the pull kernel over sa.xrows.
hipError_t launch_structured_mm(const StructArgs &sa, const StepInst *insts_dev, const WorkItem *work_dev,
                                int64_t n_work, int mode, int grid, int n_det, hipStream_t stream);

}  // namespace drts
