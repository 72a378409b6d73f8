// C ABI of the DRTS library: handles, device memory hooks, sources and
// detectors, the step loop (eager or hipGraph replay), readout, state
// transfer, kernel timing, uneven batches and the autotuner.
#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "drts_internal.h"
#include "drts_step.h"

namespace drts {

static thread_local std::string g_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

const char *hip_name(hipError_t e) { return hipGetErrorString(e); }

void *Device::alloc(size_t bytes)
{
    void *p = nullptr;
    if (hooks.alloc) {
        p = hooks.alloc(hooks.ctx, bytes, hooks.stream);
        if (!p) set_error(DRTS_E_NOMEM, "device allocation of %zu bytes failed (caller hook)", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            set_error(DRTS_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
            p = nullptr;
        }
    }
    return p;
}

void Device::free(void *p)
{
    if (!p) return;
    if (hooks.free) hooks.free(hooks.ctx, p, hooks.stream);
    else (void)hipFree(p);
}

int Buffer::allocate(Device *d, size_t n)
{
    reset();
    dev = d;
    ptr = d->alloc(n ? n : 16);
    if (!ptr) return DRTS_E_NOMEM;
    bytes = n;
    return DRTS_OK;
}

void Buffer::reset()
{
    if (ptr && dev) dev->free(ptr);
    ptr = nullptr;
    bytes = 0;
}

int64_t Matrix::bytes() const
{
    const Buffer *b[] = {&row_ptr,   &col,      &val,      &grp_desc, &grp_row,   &grp_mat,  &grp_val,
                         &grp_fast,  &slow_rows, &vox2_info, &vox2_val, &vi_idx,  &vi_dict, &brick_ptr,
                         &brick_org, &vi_fdesc, &vi_fast_of};
    int64_t n = 0;
    for (const Buffer *x : b) n += (int64_t)x->bytes;
    return n;
}
int64_t Matrix::table_bytes() const
{
    const Buffer *b[] = {&mat_of_voxel, &absorb, &index, &blocks64, &blocks32, &irr_row, &irr_vox, &irr_dir,
                         &irr_f, &irr_bits, &escape_state, &pair_ptr, &pair_key, &pair_w, &arr_ptr, &arr_key, &arr_w};
    int64_t n = 0;
    for (const Buffer *x : b) n += (int64_t)x->bytes;
    return n;
}

static Device make_device(const drts_device_t *d)
{
    Device dev;
    if (d) {
        dev.hooks = *d;
        dev.stream = (hipStream_t)d->stream;
    }
    return dev;
}

static int device_cu_count()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

}  // namespace drts

using namespace drts;

struct drts_matrix {
    Matrix m;
};

// ---- solver --------------------------------------------------------------------

struct SourceEntry {
    int64_t row;
    int32_t rhs, id;
    double w;
};
struct DetEntry {
    int64_t row;
    int32_t id;
    double F;
};

struct drts_solver {
    Device dev;
    const drts_matrix *A = nullptr;
    int n_rhs = 1;
    int64_t max_steps = 0;
    drts_options_t opt{};
    int grid = 0;
    int64_t n_tiles = 0, n_chunks = 0, n_xchunks = 0;
    int64_t t_host = 0;

    Buffer buf0, buf1, ctl_t, ctl_E, ctl_M, ctl_abs, t_end, partials, xcd_bounds, xrows, xirr, xsrc, xdet, zrows, xdrng,
        ddet_ptr, ddet_row,
        ddet_F, pull_bits, esc_base, grp_src, grp_src_f;
    Buffer ser_tot, ser_det, ser_exp, ser_abs_exp, amp, smax;
    Buffer src_tile, src_row, src_id, src_rhs, src_w;
    Buffer det_tile, det_row, det_id, det_F;
    Buffer inst_dev, work_dev, queue;

    // host copies
    std::vector<DetEntry> dets;
    int n_det = 0;
    std::vector<SourceEntry> srcs;
    const drts_source_table_t *src_key = nullptr;
    void *src_ctx_key = nullptr;
    int n_src = 0;
    std::vector<double> amp_h, smax_h;
    StepInst inst_h{};
    StructArgs sa{};
    std::vector<WorkItem> work_h;

    // graph replay
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;

    // profiling
    bool profile = false;
    bool grouped = false;        // the CSR step runs by row groups
    bool group_pending = false;  // grouped step asked for, the matrix's groups not built yet
    bool fast_src = false;       // a fast group holds a source row
    bool no_group = false;       // a batch member: the tiled step
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
};

// streams that carry the batch members with their own grouped step
constexpr int kBatchAuxStreams = 7;

struct drts_batch {
    Device dev;
    std::vector<drts_solver *> solvers;
    Buffer inst_dev, work_dev, queue;
    Buffer sas_dev, xwork_dev;   // matrix-free members: their arguments, their irregular-row items
    int grid = 0;                // workgroups of the step launch; 0: 16 per CU
    int mode = 0;                // 0: CSR step; 1 or 2: the matrix-free mode of every member
    int lead = 0;                // a member of the shared launch: its options give the launch's
    // streams of the members with their own grouped step (forked from the
    // batch's stream and joined back around each run of steps)
    hipStream_t aux[kBatchAuxStreams] = {};
    hipEvent_t fork = nullptr, join[kBatchAuxStreams] = {};
    // graphs of the last run, destroyed once the stream has passed them
    std::vector<hipGraphExec_t> spent;
    hipEvent_t done = nullptr;   // recorded after the last run's launches
};

namespace {

int upload_bytes(Device &dev, Buffer &b, const void *h, size_t bytes)
{
    int rc = b.allocate(&dev, std::max<size_t>(bytes, 16));
    if (rc) return rc;
    if (bytes) DRTS_HIP(hipMemcpyAsync(b.ptr, h, bytes, hipMemcpyHostToDevice, dev.stream));
    return DRTS_OK;
}
template <typename T> int upload_vec(Device &dev, Buffer &b, const std::vector<T> &v)
{
    return upload_bytes(dev, b, v.data(), v.size() * sizeof(T));
}

void drop_graph(drts_solver *S)
{
    if (S->graph) {
        (void)hipGraphExecDestroy(S->graph);
        S->graph = nullptr;
    }
    S->graph_steps = 0;
}

// per-tile offsets of entries sorted by row
template <typename E> std::vector<int32_t> tile_offsets(const std::vector<E> &v, int64_t n_tiles, int rows_per_tile)
{
    std::vector<int32_t> off((size_t)n_tiles + 1, 0);
    size_t e = 0;
    for (int64_t k = 0; k <= n_tiles; ++k) {
        const int64_t r0 = k * (int64_t)rows_per_tile;
        while (e < v.size() && v[e].row < r0) ++e;
        off[(size_t)k] = (int32_t)e;
    }
    return off;
}

// per-tile offsets for explicit tile row boundaries
template <typename E> std::vector<int32_t> tile_offsets_bounds(const std::vector<E> &v, const std::vector<int64_t> &b)
{
    std::vector<int32_t> off(b.size(), 0);
    size_t e = 0;
    for (size_t k = 0; k < b.size(); ++k) {
        while (e < v.size() && v[e].row < b[k]) ++e;
        off[k] = (int32_t)e;
    }
    return off;
}

bool spmm_of(const drts_solver *S) { return S->n_rhs > 1; }
bool structured_of(const drts_solver *S) { return S->opt.kernel != DRTS_KERNEL_CSR; }

// Tile row boundaries of the structured kernel: segments of kStructSegLen
// voxels of every x-line (the last boundary is n_states).
// Kernel mode of a single-rhs matrix-free step: 0 exact values with global
// gathers (FP64, dithered FP32), 1 exact nearest FP32 values, 2 FP64 row sums,
// 3 FP64 row sums with global gathers (more materials than the
// direction-major kernel takes).
int structured_mode(const drts_solver *S)
{
    const Model &M = S->A->m.model;
    const bool f64 = M.value_type == DRTS_F64;
    const bool many = M.mats.size() > (size_t)kStructMatLdsHost;
    if (S->opt.kernel == DRTS_KERNEL_STRUCTURED)
        return (f64 || M.rounding == DRTS_ROUND_DITHER || many) ? 0 : 1;
    return f64 ? 0 : (many ? 3 : 2);
}

std::vector<int64_t> structured_bounds(const Model &M, StructArgs *sa, int L)
{
    const int segs = (M.nx + L - 1) / L;
    const int64_t lines = (int64_t)M.ny * M.nz;
    std::vector<int64_t> b;
    b.reserve((size_t)(lines * segs + 1));
    for (int64_t line = 0; line < lines; ++line)
        for (int sg = 0; sg < segs; ++sg) b.push_back((int64_t)kDirs * (sg * L + (int64_t)M.nx * line));
    b.push_back(M.n_states);
    sa->seg_len = L;
    sa->segs_per_line = segs;
    sa->n_vox_tiles = lines * segs;
    return b;
}

// Rows of the second structured kernel: the irregular rows, then the escape
// rows, ascending; with each row's range of the (row-sorted) irregular-move
// list, so the kernel needs no search (escape rows: empty ranges).
void structured_xrows(const Model &M, std::vector<int64_t> *rows, std::vector<int64_t> *irr)
{
    std::vector<int64_t> &r = *rows, &k = *irr;
    r.clear();
    k.clear();
    r.reserve(M.irr_row.size() + (size_t)M.n_escape);
    k.reserve(M.irr_row.size() + (size_t)M.n_escape + 1);
    for (size_t i = 0; i < M.irr_row.size(); ++i)
        if (r.empty() || r.back() != M.irr_row[i]) {
            r.push_back(M.irr_row[i]);
            k.push_back((int64_t)i);
        }
    const int64_t n_irr = (int64_t)M.irr_row.size();
    for (int64_t e = M.n_states; e < M.n_rows; ++e) {
        r.push_back(e);
        k.push_back(n_irr);
    }
    k.push_back(n_irr);
}

// Rows the many-rhs push kernel leaves to the pull kernel (marked in *bits):
// irregular rows, rows holding a source or a detector entry (escape rows
// included), and state rows that take no plain move (upstream voxel outside
// the grid or across an index change).  Those of them that take no move at
// all and no source (their value is zero; a detector entry adds nothing) go
// to *zero; the others to *rows, ascending, with each row's range of the
// irregular-move list.  And per voxel the offset of its first escape row.
void structured_mm_pull(const Model &M, const std::vector<SourceEntry> &srcs, const std::vector<DetEntry> &dets,
                        std::vector<uint32_t> *bits, std::vector<int64_t> *rows, std::vector<int64_t> *irr,
                        std::vector<int64_t> *zero, std::vector<int32_t> *esc_base)
{
    std::vector<uint32_t> &b = *bits;
    const size_t words = (size_t)((M.n_rows + 31) / 32);
    b.assign(words, 0u);
    std::vector<uint32_t> full(words, 0u);   // rows with an irregular move or a source
    auto mark = [&](int64_t r) { b[(size_t)(r >> 5)] |= 1u << (r & 31); };
    auto mark_full = [&](int64_t r) { full[(size_t)(r >> 5)] |= 1u << (r & 31); };
    for (int64_t r : M.irr_row) {
        mark(r);
        mark_full(r);
    }
    for (const SourceEntry &e : srcs) {
        mark(e.row);
        mark_full(e.row);
    }
    for (const DetEntry &e : dets) mark(e.row);
    std::vector<uint32_t> noplain(words, 0u);
    for (int z = 0; z < M.nz; ++z)
        for (int y = 0; y < M.ny; ++y)
            for (int x = 0; x < M.nx; ++x) {
                const int64_t w = x + (int64_t)M.nx * (y + (int64_t)M.ny * z);
                const double nw = M.index[M.mat_of_voxel[(size_t)w]];
                for (int m = 0; m < kDirs; ++m) {
                    const int ux = x - dir_dx(m), uy = y - dir_dy(m), uz = z - dir_dz(m);
                    bool plain = ux >= 0 && ux < M.nx && uy >= 0 && uy < M.ny && uz >= 0 && uz < M.nz;
                    if (plain) {
                        const int64_t u = ux + (int64_t)M.nx * (uy + (int64_t)M.ny * uz);
                        plain = M.index[M.mat_of_voxel[(size_t)u]] == nw;
                    }
                    if (!plain) {
                        const int64_t r = kDirs * w + m;
                        mark(r);
                        noplain[(size_t)(r >> 5)] |= 1u << (r & 31);
                    }
                }
            }
    // row k's irregular moves are entries irr[k] .. irr[k+1]-1: irr[k] is the
    // first entry at or after row k; every irregular row is listed, so no
    // entry lies between two listed rows and the ranges are exact (empty for
    // rows that are not irregular)
    rows->clear();
    irr->clear();
    zero->clear();
    size_t k = 0;
    for (int64_t r = 0; r < M.n_rows; ++r) {
        const uint32_t bit = 1u << (r & 31);
        if (!(b[(size_t)(r >> 5)] & bit)) continue;
        if ((noplain[(size_t)(r >> 5)] & bit) && !(full[(size_t)(r >> 5)] & bit)) {
            zero->push_back(r);
            continue;
        }
        while (k < M.irr_row.size() && M.irr_row[k] < r) ++k;
        rows->push_back(r);
        irr->push_back((int64_t)k);
    }
    irr->push_back((int64_t)M.irr_row.size());
    esc_base->assign((size_t)M.n_vox, 0);
    for (int64_t i = (int64_t)M.escape_state.size() - 1; i >= 0; --i)
        (*esc_base)[(size_t)(M.escape_state[(size_t)i] / kDirs)] = (int32_t)i;
}

// For each listed row (ascending), the index of the first entry of a
// row-sorted entry list at or after that row: the kernels walk a row's
// entries from there without a search.
template <typename E>
std::vector<int32_t> first_entries(const std::vector<int64_t> &rows, const std::vector<E> &entries)
{
    std::vector<int32_t> f(rows.size());
    size_t k = 0;
    for (size_t i = 0; i < rows.size(); ++i) {
        while (k < entries.size() && entries[k].row < rows[i]) ++k;
        f[i] = (int32_t)k;
    }
    return f;
}

// XCD-aware order of a solver's chunks.  With the remapped walk, XCD i takes
// the i-th eighth of the work list; this order makes that eighth one slab of
// y lines (ny / 8 of them) swept in z, so the x values a chunk gathers (the
// 26 neighbours of its voxels) come from a few planes of its own slab and stay
// in that XCD's L2 while the neighbouring chunks use them.  Escape chunks sit
// beside the voxels they leave from.  Only the order of the list changes:
// every chunk keeps its own partials, so results are the same bit for bit.
constexpr int kXcdCount = 8;
void order_by_slabs(drts_solver *S, const std::vector<int64_t> &bounds)
{
    const Model &M = S->A->m.model;
    const int64_t tpc = S->opt.tiles_per_chunk, rpt = S->opt.rows_per_tile;
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)S->n_chunks);
    for (int64_t c = 0; c < S->n_chunks; ++c) {
        const int64_t r0 = bounds.empty() ? c * tpc * rpt : bounds[(size_t)(c * tpc)];
        const bool esc = r0 >= M.n_states;
        const int64_t v = (esc ? M.escape_state[(size_t)(r0 - M.n_states)] : r0) / kDirs;
        const int64_t x = v % M.nx, y = (v / M.nx) % M.ny, z = v / ((int64_t)M.nx * M.ny);
        const int64_t slab = y * kXcdCount / M.ny;
        const uint64_t k = ((((uint64_t)slab * M.nz + z) * M.ny + y) * M.nx + x) * 2 + (esc ? 1 : 0);
        key[(size_t)c] = {k, (int32_t)c};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    for (size_t i = 0; i < key.size(); ++i) S->work_h[i] = {0, key[i].second};
}

// Boundaries of the XCDs' ranges of the work list with about equal work in
// each: entries of [A; L] for the CSR kernels (read from the device row
// pointers at the chunk starts), rows for the matrix-free kernel.
int balanced_xcd_bounds(drts_solver *S, const std::vector<int64_t> &bounds, std::vector<int64_t> *out)
{
    const Matrix &A = S->A->m;
    const int64_t nc = S->n_chunks, tpc = S->opt.tiles_per_chunk, rpt = S->opt.rows_per_tile;
    std::vector<int64_t> w((size_t)nc, 0);
    if (!bounds.empty()) {
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t a = bounds[(size_t)std::min(c * tpc, (int64_t)bounds.size() - 1)];
            const int64_t b = bounds[(size_t)std::min((c + 1) * tpc, (int64_t)bounds.size() - 1)];
            w[(size_t)c] = b - a;
        }
    } else {
        const int64_t step = tpc * rpt;   // rows per chunk
        const size_t es = A.rp64 ? 8 : 4;
        std::vector<int64_t> rp((size_t)nc + 1);
        std::vector<char> raw(((size_t)nc + 1) * es);
        DRTS_HIP(hipMemcpy2DAsync(raw.data(), es, A.row_ptr.ptr, (size_t)step * es, es, (size_t)nc, hipMemcpyDeviceToHost,
                                  S->dev.stream));
        DRTS_HIP(hipMemcpyAsync(raw.data() + (size_t)nc * es, (const char *)A.row_ptr.ptr + (size_t)A.model.n_rows * es,
                                es, hipMemcpyDeviceToHost, S->dev.stream));
        DRTS_HIP(hipStreamSynchronize(S->dev.stream));
        for (size_t i = 0; i <= (size_t)nc; ++i)
            rp[i] = A.rp64 ? ((const int64_t *)raw.data())[i] : (int64_t)((const int32_t *)raw.data())[i];
        for (int64_t c = 0; c < nc; ++c) w[(size_t)c] = rp[(size_t)c + 1] - rp[(size_t)c];
    }
    int64_t total = 0;
    for (const WorkItem &it : S->work_h) total += w[(size_t)it.chunk];
    out->assign(kXcdBounds, nc);
    (*out)[0] = 0;
    int64_t acc = 0;
    int x = 1;
    for (int64_t i = 0; i < nc && x < kXcdBounds - 1; ++i) {
        acc += w[(size_t)S->work_h[(size_t)i].chunk];
        while (x < kXcdBounds - 1 && acc * (kXcdBounds - 1) >= total * x) (*out)[(size_t)x++] = i + 1;
    }
    return DRTS_OK;
}

// Matrices whose rows hold several hundred entries (the multi-voxel weights of
// Lebedev media) step with the wave-per-row SpMV.
bool long_rows(const Matrix &A) { return A.model.n_rows > 0 && A.nnz >= (int64_t)kLongRowMean * A.model.n_rows; }

int prepare(drts_solver *S);

// Builds the matrix's row groups if the solver asked for the grouped step
// and they are not built yet, then lays the solver out for them.
int settle_groups(drts_solver *S)
{
    if (!S->group_pending) return DRTS_OK;
    int rc = row_groups(S->A->m);
    return rc ? rc : prepare(S);
}

// Detector entries grouped by detector (stable: rows stay ascending within
// each), uploaded; ptr and row receive the host copies.
int upload_dets_by_detector(drts_solver *S, std::vector<int64_t> *ptr_out, std::vector<int64_t> *row_out)
{
    std::vector<int64_t> &ptr = *ptr_out, &row = *row_out;
    ptr.assign((size_t)S->n_det + 1, 0);
    row.assign(S->dets.size(), 0);
    std::vector<double> F(S->dets.size());
    for (const DetEntry &d : S->dets) ++ptr[(size_t)d.id + 1];
    for (int d = 0; d < S->n_det; ++d) ptr[(size_t)d + 1] += ptr[(size_t)d];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (const DetEntry &d : S->dets) {
        const size_t at = (size_t)fill[(size_t)d.id]++;
        row[at] = d.row;
        F[at] = d.F;
    }
    int rc;
    if ((rc = upload_vec(S->dev, S->ddet_ptr, ptr))) return rc;
    if ((rc = upload_vec(S->dev, S->ddet_row, row))) return rc;
    return upload_vec(S->dev, S->ddet_F, F);
}

// (Re)builds every structure that depends on the options and the sources.
int prepare(drts_solver *S)
{
    const Matrix &A = S->A->m;
    Device &dev = S->dev;
    const drts_options_t &o = S->opt;
    int rc;
    std::vector<int64_t> bounds;
    if (structured_of(S)) {
        StructArgs &sa = S->sa;
        sa.nx = A.model.nx;
        sa.ny = A.model.ny;
        sa.nz = A.model.nz;
        sa.rounding = A.model.rounding;
        sa.n_states = A.model.n_states;
        sa.n_rows = A.model.n_rows;
        sa.mat = A.mat_of_voxel.as<uint8_t>();
        sa.index = A.index.as<double>();
        sa.blocks32 = A.blocks32.as<float>();
        sa.blocks64 = A.blocks64.as<double>();
        sa.n_mat = (int32_t)A.model.mats.size();
        sa.irr_row = A.irr_row.as<int64_t>();
        sa.irr_vox = A.irr_vox.as<int64_t>();
        sa.irr_dir = A.irr_dir.as<int32_t>();
        sa.irr_f = A.irr_f.as<double>();
        sa.irr_bits = A.irr_bits.as<uint32_t>();
        sa.n_irr = (int64_t)A.model.irr_row.size();
        sa.escape_state = A.escape_state.as<int64_t>();
        std::vector<int64_t> xr, xk;
        if (spmm_of(S)) {
            // many rhs: push work items of kStructVoxPerChunk voxels, the pull list
            const int64_t nvox = A.model.n_states / kDirs;
            S->n_tiles = (nvox + kStructVoxPerChunk - 1) / kStructVoxPerChunk;
            std::vector<uint32_t> pb;
            std::vector<int32_t> eb;
            std::vector<int64_t> zr;
            structured_mm_pull(A.model, S->srcs, S->dets, &pb, &xr, &xk, &zr, &eb);
            if ((rc = upload_vec(dev, S->pull_bits, pb))) return rc;
            if ((rc = upload_vec(dev, S->esc_base, eb))) return rc;
            if ((rc = upload_vec(dev, S->zrows, zr))) return rc;
            sa.pull_bits = S->pull_bits.as<uint32_t>();
            sa.esc_base = S->esc_base.as<int32_t>();
            sa.zrows = S->zrows.as<int64_t>();
            sa.n_zrows = (int64_t)zr.size();
            // the pull kernel's workgroups: its row items, or the zero rows
            // (kStructMmXRows per workgroup) if those are more
            S->n_xchunks = std::max(((int64_t)xr.size() + kStructMmXRows - 1) / kStructMmXRows,
                                    (sa.n_zrows + kStructMmXRows - 1) / kStructMmXRows);
        } else {
            const int mode = structured_mode(S);
            bounds = structured_bounds(A.model, &sa, (mode == 1 || mode == 2) ? kStructDmSeg : kStructSegLen);
            sa.zrows = nullptr;
            sa.n_zrows = 0;
            S->n_tiles = (int64_t)bounds.size() - 1;
            structured_xrows(A.model, &xr, &xk);
            S->n_xchunks = ((int64_t)xr.size() + kStructXRows - 1) / kStructXRows;
        }
        if ((rc = upload_vec(dev, S->xrows, xr))) return rc;
        if ((rc = upload_vec(dev, S->xirr, xk))) return rc;
        if ((rc = upload_vec(dev, S->xsrc, first_entries(xr, S->srcs)))) return rc;
        if ((rc = upload_vec(dev, S->xdet, first_entries(xr, S->dets)))) return rc;
        sa.xrows = S->xrows.as<int64_t>();
        sa.xirr = S->xirr.as<int64_t>();
        sa.xsrc = S->xsrc.as<int32_t>();
        sa.xdet = S->xdet.as<int32_t>();
        sa.n_xrows = (int64_t)xr.size();
        sa.n_src_entries = (int64_t)S->srcs.size();
        sa.n_det_entries = (int64_t)S->dets.size();
        {
            std::vector<int64_t> ptr, row;
            if ((rc = upload_dets_by_detector(S, &ptr, &row))) return rc;
            if (!spmm_of(S)) {
                // per work item of the second kernel (kStructXRows listed rows) and
                // detector: the range of the detector's entries whose rows lie in
                // the item's row span
                const int64_t n_items = ((int64_t)xr.size() + kStructXRows - 1) / kStructXRows;
                std::vector<int64_t> rng((size_t)std::max<int64_t>(n_items * S->n_det * 2, 1), 0);
                for (int d = 0; d < S->n_det; ++d) {
                    const auto b0 = row.begin() + ptr[(size_t)d], b1 = row.begin() + ptr[(size_t)d + 1];
                    for (int64_t j = 0; j < n_items; ++j) {
                        const int64_t ra = xr[(size_t)(j * kStructXRows)];
                        const int64_t rb = xr[(size_t)std::min<int64_t>((j + 1) * kStructXRows, (int64_t)xr.size()) - 1];
                        rng[(size_t)((j * S->n_det + d) * 2)] = std::lower_bound(b0, b1, ra) - row.begin();
                        rng[(size_t)((j * S->n_det + d) * 2 + 1)] = std::upper_bound(b0, b1, rb) - row.begin();
                    }
                }
                if ((rc = upload_vec(dev, S->xdrng, rng))) return rc;
                sa.xdrng = S->xdrng.as<int64_t>();
            }
            sa.ddet_ptr = S->ddet_ptr.as<int64_t>();
            sa.ddet_row = S->ddet_row.as<int64_t>();
            sa.ddet_F = S->ddet_F.as<double>();
        }
    } else {
        S->n_tiles = (A.model.n_rows + o.rows_per_tile - 1) / o.rows_per_tile;
        S->n_xchunks = 0;
    }
    // the CSR step by row groups when the rows group (at least two rows a
    // group on average; rows of several hundred entries take their own
    // step).  The matrix's groups are built at the first solo step or run
    // (settle_groups), not here: batch members never use them.
    S->grouped = false;
    S->group_pending = false;
    const bool f64sum = spmm_of(S) && o.kernel == DRTS_KERNEL_CSR && o.variant == DRTS_SPMM_GROUPED_F64SUM;
    if (!S->no_group && o.kernel == DRTS_KERNEL_CSR &&
        (spmm_of(S) ? o.variant != DRTS_SPMM_ROWS : o.variant == DRTS_SPMV_GROUPED) && !long_rows(A)) {
        if (A.n_groups < 0) S->group_pending = true;
        else S->grouped = A.n_groups > 0;
    }
    if (f64sum && !S->grouped && !S->group_pending)
        return set_error(DRTS_E_INVALID, "DRTS_SPMM_GROUPED_F64SUM needs rows that group (and are not several "
                                         "hundred entries long)");
    // a work item of the many-rhs matrix-free step is one tile (kStructVoxPerChunk
    // voxels); its kernels, and the step by row groups, keep one set of
    // partials per workgroup
    const bool smm = structured_of(S) && spmm_of(S);
    const int64_t tpc = smm ? 1 : o.tiles_per_chunk;
    S->n_chunks = (S->n_tiles + tpc - 1) / tpc;
    if (structured_of(S)) S->sa.chunk_base = S->n_chunks;
    int64_t n_part = S->n_chunks + S->n_xchunks;   // chunk partials the finalize reduces
    S->grid = o.grid > 0 ? o.grid : device_cu_count() * (spmm_of(S) ? 4 : 8);
    if (smm) {
        S->sa.mm_push_grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(S->grid, S->n_chunks));
        S->sa.mm_pull_grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(S->grid, S->n_xchunks));
        S->sa.chunk_base = S->sa.mm_push_grid;
        n_part = S->sa.mm_push_grid + (S->n_xchunks > 0 ? S->sa.mm_pull_grid : 0);
    }
    if (S->grouped) {
        // partials per work item and wave (single rhs: then per row-list item
        // and wave); detector entries by detector; the groups holding source rows
        n_part = 4 * S->n_chunks;
        if (!spmm_of(S))
            n_part += 4 * ((A.n_slow + kRowListItem - 1) / kRowListItem) + 4 * ((A.n_vox2 + kVox2Item - 1) / kVox2Item);
        std::vector<int64_t> ptr, row;
        if ((rc = upload_dets_by_detector(S, &ptr, &row))) return rc;
        std::vector<int64_t> srows;
        for (const SourceEntry &e : S->srcs)
            if (srows.empty() || srows.back() != e.row) srows.push_back(e.row);
        Buffer sr;
        if ((rc = upload_vec(dev, sr, srows))) return rc;
        if ((rc = S->grp_src.allocate(&dev, (size_t)((A.n_groups + 31) / 32 + 1) * sizeof(uint32_t)))) return rc;
        if ((rc = group_flags(A, sr.as<int64_t>(), (int64_t)srows.size(), S->grp_src.as<uint32_t>(), dev.stream)))
            return rc;
        S->fast_src = false;
        if (A.vi_ntab > 0) {
            const size_t words = (size_t)((A.n_fast + 31) / 32 + 1);
            if ((rc = S->grp_src_f.allocate(&dev, words * sizeof(uint32_t)))) return rc;
            DRTS_HIP(hipMemsetAsync(S->grp_src_f.ptr, 0, words * sizeof(uint32_t), dev.stream));
            if ((rc = fast_flags(A, S->grp_src.as<uint32_t>(), S->grp_src_f.as<uint32_t>(), dev.stream))) return rc;
            // whether any fast group holds a source row (the step leaves the
            // source code out when none does)
            std::vector<uint32_t> fw(words);
            DRTS_HIP(hipMemcpyAsync(fw.data(), S->grp_src_f.ptr, words * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                    dev.stream));
            DRTS_HIP(hipStreamSynchronize(dev.stream));
            for (uint32_t x : fw) S->fast_src = S->fast_src || x != 0u;
        }
        DRTS_HIP(hipStreamSynchronize(dev.stream));
    }
    if (S->n_chunks > INT32_MAX) return set_error(DRTS_E_RANGE, "too many chunks");

    // sources and detectors per tile (the many-rhs matrix-free kernels look
    // them up in the row-sorted lists instead)
    if (structured_of(S) && spmm_of(S)) {
        if ((rc = upload_vec(dev, S->src_tile, tile_offsets(S->srcs, S->n_tiles, kStructVoxPerChunk * kDirs))))
            return rc;
        if ((rc = upload_vec(dev, S->det_tile, tile_offsets(S->dets, S->n_tiles, kStructVoxPerChunk * kDirs))))
            return rc;
    } else if (structured_of(S)) {
        if ((rc = upload_vec(dev, S->src_tile, tile_offsets_bounds(S->srcs, bounds)))) return rc;
        if ((rc = upload_vec(dev, S->det_tile, tile_offsets_bounds(S->dets, bounds)))) return rc;
    } else {
        if ((rc = upload_vec(dev, S->src_tile, tile_offsets(S->srcs, S->n_tiles, o.rows_per_tile)))) return rc;
        if ((rc = upload_vec(dev, S->det_tile, tile_offsets(S->dets, S->n_tiles, o.rows_per_tile)))) return rc;
    }
    if ((rc = S->partials.allocate(&dev, partials_bytes(S->n_det, S->n_rhs, n_part)))) return rc;

    StepInst &I = S->inst_h;
    memset(&I, 0, sizeof I);
    I.row_ptr = A.row_ptr.ptr;
    I.col = A.col.as<int32_t>();
    I.val = A.val.ptr;
    I.n_rows = A.model.n_rows;
    I.n_states = A.model.n_states;
    I.nnz = A.nnz;
    I.rp64 = A.rp64 ? 1 : 0;
    I.rows_per_tile = o.rows_per_tile;
    I.n_tiles = S->n_tiles;
    I.tiles_per_chunk = (int32_t)tpc;
    I.n_rhs = S->n_rhs;
    I.buf0 = S->buf0.ptr;
    I.buf1 = S->buf1.ptr;
    I.mat = A.mat_of_voxel.as<uint8_t>();
    I.absorb = A.absorb.as<double>();
    I.src_tile = S->src_tile.as<int32_t>();
    I.src_row = S->src_row.as<int64_t>();
    I.src_id = S->src_id.as<int32_t>();
    I.src_rhs = S->src_rhs.as<int32_t>();
    I.src_w = S->src_w.as<double>();
    I.amp = S->amp.as<double>();
    I.smax = S->smax.as<double>();
    I.n_src = S->n_src;
    I.n_det = S->n_det;
    I.det_tile = S->det_tile.as<int32_t>();
    I.det_row = S->det_row.as<int64_t>();
    I.det_id = S->det_id.as<int32_t>();
    I.det_F = S->det_F.as<double>();
    I.t = S->ctl_t.as<int64_t>();
    I.E = S->ctl_E.as<int32_t>();
    I.M = S->ctl_M.as<double>();
    I.abs_cur = S->ctl_abs.as<double>();
    I.t_end = S->t_end.as<int64_t>();
    I.rescale = o.rescale;
    I.n_mat = (int32_t)A.model.mats.size();
    I.vox_mul = vox_mul_of(A.model.n_dir);
    I.max_steps = S->max_steps;
    if (S->grouped) {
        I.grp = A.grp_desc.as<GroupDesc>();
        I.grp_row = A.grp_row.as<int32_t>();
        I.grp_mat = A.grp_mat.as<uint8_t>();
        I.grp_val = A.grp_val.as<float>();
        I.grp_src = S->grp_src.as<uint32_t>();
        I.n_groups = A.n_groups;
        I.grp_fast = A.grp_fast.as<int32_t>();
        I.slow_rows = A.slow_rows.as<int32_t>();
        I.n_fast = A.n_fast;
        I.n_slow = A.n_slow;
        I.slow_part = 4 * S->n_chunks;
        I.vox2_info = A.vox2_info.as<int32_t>();
        I.vox2_val = A.vox2_val.as<float>();
        I.n_vox2 = A.n_vox2;
        I.vox2_part = I.slow_part + 4 * ((A.n_slow + kRowListItem - 1) / kRowListItem);
        I.vi_idx = A.vi_ntab > 0 ? A.vi_idx.as<uint8_t>() : nullptr;
        I.vi_dict = A.vi_ntab > 0 ? A.vi_dict.as<float>() : nullptr;
        I.vi_ntab = A.vi_ntab;
        I.brick_ptr = A.brick_ptr.as<int32_t>();
        I.brick_org = A.brick_org.as<int32_t>();
        I.n_brick = A.n_brick;
        I.grid_nx = A.model.nx;
        I.grid_ny = A.model.ny;
        I.vi_fdesc = A.vi_ntab > 0 ? A.vi_fdesc.as<int32_t>() : nullptr;
        I.vi_fast_of = A.vi_ntab > 0 ? A.vi_fast_of.as<int32_t>() : nullptr;
        I.grp_src_f = A.vi_ntab > 0 ? S->grp_src_f.as<uint32_t>() : nullptr;
        I.det_direct = 1;
        I.ddet_ptr = S->ddet_ptr.as<int64_t>();
        I.ddet_row = S->ddet_row.as<int64_t>();
        I.ddet_F = S->ddet_F.as<double>();
    }
    I.partials = S->partials.as<double>();
    I.n_chunks = n_part;   // the finalize reduces both kernels' chunks
    I.ser_tot = S->ser_tot.as<double>();
    I.ser_det = S->ser_det.as<double>();
    I.ser_exp = S->ser_exp.as<int32_t>();
    I.ser_abs_exp = S->ser_abs_exp.as<int32_t>();
    if ((rc = upload_bytes(dev, S->inst_dev, &I, sizeof I))) return rc;

    S->work_h.resize((size_t)S->n_chunks);
    for (int64_t c = 0; c < S->n_chunks; ++c) S->work_h[(size_t)c] = {0, (int32_t)c};
    // (the many-rhs matrix-free kernels walk their voxel chunks in order)
    if (o.xcd_remap == 2 && !(structured_of(S) && spmm_of(S))) order_by_slabs(S, bounds);
    if ((rc = upload_vec(dev, S->work_dev, S->work_h))) return rc;
    S->xcd_bounds.reset();
    if (o.xcd_remap && !(structured_of(S) && spmm_of(S))) {
        std::vector<int64_t> xb;
        if ((rc = balanced_xcd_bounds(S, bounds, &xb))) return rc;
        if ((rc = upload_vec(dev, S->xcd_bounds, xb))) return rc;
    }
    drop_graph(S);
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    return DRTS_OK;
}

int set_sources(drts_solver *S, const drts_source_table_t *src)
{
    if (!src || src->n_src <= 0) {
        if (S->n_src == 0 && S->src_key == nullptr) return DRTS_OK;
        S->srcs.clear();
        S->n_src = 0;
        S->src_key = nullptr;
        S->src_ctx_key = nullptr;
    } else {
        if (src == S->src_key && src->ctx == S->src_ctx_key && src->n_src == S->n_src) return DRTS_OK;
        if (!src->support || !src->amplitude) return set_error(DRTS_E_INVALID, "source table lacks callbacks");
        if (S->n_rhs > 1 && !src->rhs_of) return set_error(DRTS_E_INVALID, "rhs_of is required with n_rhs > 1");
        std::vector<SourceEntry> e;
        std::vector<int64_t> st(64);
        std::vector<double> w(64);
        const int64_t D = S->A->m.model.n_states;
        for (int32_t k = 0; k < src->n_src; ++k) {
            int64_t n = src->support(src->ctx, k, st.data(), w.data(), (int64_t)st.size());
            if (n > (int64_t)st.size()) {
                st.resize((size_t)n);
                w.resize((size_t)n);
                n = src->support(src->ctx, k, st.data(), w.data(), (int64_t)st.size());
            }
            if (n < 0 || n > (int64_t)st.size()) return set_error(DRTS_E_INVALID, "source %d: bad support size", k);
            const int32_t rhs = src->rhs_of ? src->rhs_of(src->ctx, k) : 0;
            if (rhs < 0 || rhs >= S->n_rhs) return set_error(DRTS_E_INVALID, "source %d feeds rhs %d", k, rhs);
            for (int64_t i = 0; i < n; ++i) {
                if (st[(size_t)i] < 0 || st[(size_t)i] >= D)
                    return set_error(DRTS_E_INVALID, "source %d: state %lld out of range", k, (long long)st[(size_t)i]);
                e.push_back({st[(size_t)i], rhs, k, w[(size_t)i]});
            }
        }
        std::stable_sort(e.begin(), e.end(), [](const SourceEntry &a, const SourceEntry &b) {
            return a.row != b.row ? a.row < b.row : a.rhs < b.rhs;
        });
        S->srcs.swap(e);
        S->n_src = src->n_src;
        S->src_key = src;
        S->src_ctx_key = src->ctx;
    }
    Device &dev = S->dev;
    std::vector<int64_t> row(S->srcs.size());
    std::vector<int32_t> id(S->srcs.size()), rhs(S->srcs.size());
    std::vector<double> w(S->srcs.size());
    for (size_t i = 0; i < S->srcs.size(); ++i) {
        row[i] = S->srcs[i].row;
        id[i] = S->srcs[i].id;
        rhs[i] = S->srcs[i].rhs;
        w[i] = S->srcs[i].w;
    }
    int rc;
    if ((rc = upload_vec(dev, S->src_row, row))) return rc;
    if ((rc = upload_vec(dev, S->src_id, id))) return rc;
    if ((rc = upload_vec(dev, S->src_rhs, rhs))) return rc;
    if ((rc = upload_vec(dev, S->src_w, w))) return rc;
    if ((rc = S->amp.allocate(&dev, (size_t)S->max_steps * std::max(S->n_src, 1) * sizeof(double)))) return rc;
    DRTS_HIP(hipMemsetAsync(S->amp.ptr, 0, S->amp.bytes, dev.stream));
    // one step's host amplitudes never reallocate after this (drts_step_noalloc)
    S->amp_h.reserve((size_t)std::max(S->n_src, 1));
    S->smax_h.reserve((size_t)S->n_rhs);
    return prepare(S);
}

// Host amplitudes and per-rhs source bounds for steps [t0, t0 + n), uploaded.
int upload_amplitudes(drts_solver *S, const drts_source_table_t *src, int64_t t0, int64_t n)
{
    const int ns = S->n_src, nr = S->n_rhs;
    S->smax_h.assign((size_t)n * nr, 0.0);
    if (ns > 0) {
        const double dt = S->A->m.model.dt_s;
        S->amp_h.resize((size_t)n * ns);
        for (int64_t s = 0; s < n; ++s)
            for (int k = 0; k < ns; ++k)
                S->amp_h[(size_t)(s * ns + k)] = src->amplitude(src->ctx, k, t0 + s, (double)(t0 + s) * dt, dt);
        // bound of |s_t| per rhs: the largest |row sum| over source rows
        for (int64_t s = 0; s < n; ++s) {
            size_t i = 0;
            while (i < S->srcs.size()) {
                size_t j = i;
                double acc = 0.0;
                while (j < S->srcs.size() && S->srcs[j].row == S->srcs[i].row && S->srcs[j].rhs == S->srcs[i].rhs) {
                    acc += S->srcs[j].w * S->amp_h[(size_t)(s * ns + S->srcs[j].id)];
                    ++j;
                }
                double &m = S->smax_h[(size_t)(s * nr + S->srcs[i].rhs)];
                m = std::max(m, std::fabs(acc));
                i = j;
            }
        }
        DRTS_HIP(hipMemcpyAsync(S->amp.as<double>() + t0 * ns, S->amp_h.data(), (size_t)n * ns * sizeof(double),
                                hipMemcpyHostToDevice, S->dev.stream));
    }
    DRTS_HIP(hipMemcpyAsync(S->smax.as<double>() + t0 * nr, S->smax_h.data(), (size_t)n * nr * sizeof(double),
                            hipMemcpyHostToDevice, S->dev.stream));
    // the copies read host vectors that the next call may overwrite
    DRTS_HIP(hipStreamSynchronize(S->dev.stream));
    return DRTS_OK;
}

hipEvent_t next_event(drts_solver *S)
{
    if (S->ev_used == S->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        S->ev_pool.push_back(e);
    }
    return S->ev_pool[S->ev_used++];
}


// The single-rhs kernel a solver's CSR step takes: rows of several hundred
// entries the wave-per-row step, rows that group (FP32) the grouped step, a
// grouped request on rows that do not group the LDS layout.
int spmv_variant(const drts_solver *S)
{
    if (long_rows(S->A->m)) return kVariantLongRows;
    if (S->grouped) return DRTS_SPMV_GROUPED;
    return S->opt.variant == DRTS_SPMV_GROUPED ? DRTS_SPMV_LDS : S->opt.variant;
}

// One step's launches.  inst (NULL = the solver's own) is the device copy of
// the step descriptor the kernels read (matrix, state, partials, series);
// queue_override (used when inst is given) is the work counter of the
// dynamic walk.
int launch_one(drts_solver *S, hipStream_t stream, const StepInst *inst = nullptr, int32_t *queue_override = nullptr)
{
    const Matrix &A = S->A->m;
    const bool spmm = spmm_of(S);
    const StepInst *insts = inst ? inst : S->inst_dev.as<StepInst>();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (S->profile && stream == S->dev.stream) {
        e0 = next_event(S);
        e1 = next_event(S);
        if (!e0 || !e1) return set_error(DRTS_E_HIP, "hipEventCreate failed");
        DRTS_HIP(hipEventRecord(e0, stream));
    }
    if (!structured_of(S) && !A.has_csr)
        return set_error(DRTS_E_STATE, "the CSR step needs the matrix's CSR arrays (built without them)");
    int32_t *queue = (!spmm && S->opt.queue && S->opt.kernel == DRTS_KERNEL_CSR && !S->grouped)
                         ? (inst ? queue_override : S->queue.as<int32_t>())
                         : nullptr;
    hipError_t e;
    if (structured_of(S) && spmm) {
        e = launch_structured_mm(S->sa, insts, S->work_dev.as<WorkItem>(), S->n_chunks,
                                 S->opt.kernel == DRTS_KERNEL_STRUCTURED_F64SUM ? 2 : 1, S->grid, S->n_det, stream);
    } else if (structured_of(S)) {
        e = launch_structured(S->sa, insts, S->work_dev.as<WorkItem>(), S->n_chunks,
                              A.model.value_type == DRTS_F64, structured_mode(S), S->grid,
                              S->opt.xcd_remap ? 1 : 0, S->xcd_bounds.as<int64_t>(), stream);
    } else {
    const int variant = spmv_variant(S);
    e = launch_step(insts, S->work_dev.as<WorkItem>(), S->n_chunks, 1, S->n_rhs,
                               A.model.value_type == DRTS_F64, A.rp64 ? 1 : 0,
                               spmm ? (S->grouped ? (S->opt.variant == DRTS_SPMM_GROUPED_F64SUM ? 3 : 2) : 1) : 0,
                               S->grid,
                               (S->opt.xcd_remap ? 1 : 0) | ((variant & 15) << 1), S->xcd_bounds.as<int64_t>(),
                               S->opt.rows_per_tile, S->n_det, queue, stream, S->grouped ? A.n_slow : 0,
                               S->grouped && !spmm ? A.n_vox2 : 0,
                               S->grouped && A.vi_ntab > 0 ? A.vi_ntab | (!spmm && S->fast_src ? 0x100 : 0) : 0);
    }
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "step launch failed: %s", hipGetErrorString(e));
    if (e1) DRTS_HIP(hipEventRecord(e1, stream));
    e = launch_finalize(insts, 1, S->n_rhs, S->n_det, queue, stream);
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "finalize launch failed: %s", hipGetErrorString(e));
    return DRTS_OK;
}

int collect_profile(drts_solver *S)
{
    if (S->ev_used == 0) return DRTS_OK;
    DRTS_HIP(hipStreamSynchronize(S->dev.stream));
    for (size_t i = 0; i + 1 < S->ev_used; i += 2) {
        float ms = 0.f;
        DRTS_HIP(hipEventElapsedTime(&ms, S->ev_pool[i], S->ev_pool[i + 1]));
        S->prof_ms += ms;
        S->prof_launches += 1;
    }
    S->ev_used = 0;
    return DRTS_OK;
}

int ensure_graph(drts_solver *S, int K)
{
    if (S->graph && S->graph_steps == K) return DRTS_OK;
    drop_graph(S);
    if (!S->cap_stream) DRTS_HIP(hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking));
    DRTS_HIP(hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = DRTS_OK;
    for (int k = 0; k < K && rc == DRTS_OK; ++k) rc = launch_one(S, S->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(S->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&S->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        S->graph = nullptr;
        return set_error(DRTS_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    S->graph_steps = K;
    return DRTS_OK;
}

drts_options_t default_options(const drts_solver *S)
{
    // defaults measured on MI355X: one rhs on the 128^3 three-layer workload
    // (FP32: by row groups, work items of 256-row tiles x 16; FP64: the
    // tiled step, 4 tiles per chunk; 64 workgroups per CU launched: the
    // surplus waits and gives dynamic balance; round-robin walk), 64 rhs on
    // the 96^3 slab (by row groups; work items of 64-row tiles x 32, 32
    // workgroups per CU)
    const bool f64 = S->A->m.model.value_type == DRTS_F64;
    drts_options_t o{};
    o.kernel = DRTS_KERNEL_CSR;
    o.rows_per_tile = spmm_of(S) ? 64 : 256;
    o.tiles_per_chunk = spmm_of(S) ? 32 : (f64 ? 4 : 16);
    o.grid = device_cu_count() * (spmm_of(S) ? 32 : 64);
    o.xcd_remap = 0;
    o.graph_steps = 0;
    o.rescale = 1;
    o.variant = spmm_of(S) ? DRTS_SPMM_GROUPED : (f64 ? DRTS_SPMV_ROW : DRTS_SPMV_GROUPED);
    o.queue = 0;
    return o;
}

int check_options(const drts_solver *S, const drts_options_t *o)
{
    if (o->kernel < DRTS_KERNEL_CSR || o->kernel > DRTS_KERNEL_STRUCTURED_F64SUM)
        return set_error(DRTS_E_INVALID, "unknown kernel %d", o->kernel);
    if (o->kernel != DRTS_KERNEL_CSR && S->A->m.model.n_dir != kDirs)
        return set_error(DRTS_E_INVALID, "the matrix-free steps take the 26 lattice directions");
    if (o->kernel != DRTS_KERNEL_CSR && S->n_rhs != 1) {
        const Model &M = S->A->m.model;
        if (o->kernel == DRTS_KERNEL_STRUCTURED && M.rounding != DRTS_ROUND_NEAREST)
            return set_error(DRTS_E_INVALID,
                             "the exact many-rhs matrix-free step needs nearest-rounded values "
                             "(use DRTS_KERNEL_STRUCTURED_F64SUM)");
    }
    if (S->n_rhs == 1) {
        if (o->rows_per_tile != 64 && o->rows_per_tile != 128 && o->rows_per_tile != 256)
            return set_error(DRTS_E_INVALID, "rows_per_tile must be 64, 128 or 256 for one right-hand side");
        if (o->tiles_per_chunk < 1 || o->tiles_per_chunk > 64)
            return set_error(DRTS_E_INVALID, "tiles_per_chunk in 1..64 for one right-hand side");
    } else {
        if (o->rows_per_tile < 16 || o->rows_per_tile > 256)
            return set_error(DRTS_E_INVALID, "rows_per_tile in 16..256");
        if (o->tiles_per_chunk < 1 || o->tiles_per_chunk > (1 << 20))
            return set_error(DRTS_E_INVALID, "tiles_per_chunk in 1..2^20");
    }
    if (o->queue != 0 && o->queue != 1) return set_error(DRTS_E_INVALID, "queue must be 0 or 1");
    if (o->xcd_remap < 0 || o->xcd_remap > 2) return set_error(DRTS_E_INVALID, "xcd_remap must be 0, 1 or 2");
    if (S->n_rhs > 1 && o->variant != DRTS_SPMM_GROUPED && o->variant != DRTS_SPMM_ROWS &&
        o->variant != DRTS_SPMM_GROUPED_F64SUM)
        return set_error(DRTS_E_INVALID,
                         "variant %d: many rhs take DRTS_SPMM_GROUPED, DRTS_SPMM_ROWS or DRTS_SPMM_GROUPED_F64SUM",
                         o->variant);
    if (o->variant < DRTS_SPMV_ROW || o->variant > DRTS_SPMV_GROUPED)
        return set_error(DRTS_E_INVALID, "unknown variant %d", o->variant);
    if (S->n_rhs == 1 && (o->variant == DRTS_SPMV_LDS || o->variant == DRTS_SPMV_GROUPED) &&
        S->A->m.model.value_type == DRTS_F64)
        return set_error(DRTS_E_INVALID, "the LDS and grouped variants take FP32 values");
    if (o->grid < 0 || o->graph_steps < 0 || o->graph_steps > 4096)
        return set_error(DRTS_E_INVALID, "bad grid or graph_steps");
    return DRTS_OK;
}

}  // namespace

// ---- C ABI ---------------------------------------------------------------------------

extern "C" {

const char *drts_last_error(void) { return g_error.c_str(); }

}  // extern "C"

namespace drts {

int64_t matrix_device_bytes(const drts_matrix_t *A) { return A->m.bytes() + A->m.table_bytes(); }

int matrix_row_groups(const drts_matrix_t *A) { return row_groups(A->m); }

int solver_set_stream(drts_solver_t *S, hipStream_t stream)
{
    DRTS_HIP(hipStreamSynchronize(S->dev.stream));
    drop_graph(S);
    S->dev.stream = stream;
    S->dev.hooks.stream = (void *)stream;
    return DRTS_OK;
}

int build_matrix_from_model(Model &&model, const drts_device_t *dev, drts_matrix_t **out, bool with_csr)
{
    if (!out) return set_error(DRTS_E_INVALID, "out is NULL");
    *out = nullptr;
    drts_matrix *A = new (std::nothrow) drts_matrix;
    if (!A) return set_error(DRTS_E_NOMEM, "host allocation failed");
    A->m.dev = make_device(dev);
    int rc;
    try {
        A->m.model = std::move(model);
        rc = assemble_on_device(&A->m, with_csr);
    } catch (const std::bad_alloc &) {
        rc = set_error(DRTS_E_NOMEM, "host allocation failed during assembly");
    } catch (...) {
        rc = set_error(DRTS_E_INVALID, "unexpected failure during assembly");
    }
    if (rc) {
        delete A;
        return rc;
    }
    *out = A;
    return DRTS_OK;
}

}  // namespace drts

extern "C" {

int drts_build_matrix(const drts_medium_t *medium, const drts_device_t *dev, drts_matrix_t **out)
{
    if (!out) return set_error(DRTS_E_INVALID, "out is NULL");
    *out = nullptr;
    drts_matrix *A = new (std::nothrow) drts_matrix;
    if (!A) return set_error(DRTS_E_NOMEM, "host allocation failed");
    A->m.dev = make_device(dev);
    int rc;
    try {
        rc = build_model(medium, &A->m.model);
        if (!rc) rc = assemble_on_device(&A->m);
    } catch (const std::bad_alloc &) {
        rc = set_error(DRTS_E_NOMEM, "host allocation failed during assembly");
    } catch (...) {
        rc = set_error(DRTS_E_INVALID, "unexpected failure during assembly");
    }
    if (rc) {
        delete A;
        return rc;
    }
    *out = A;
    return DRTS_OK;
}

double drts_pulse_step(const drts_pulse_t *p, int64_t step, double dt_s)
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (!p || step < 0 || !(dt_s > 0.0)) {
        set_error(DRTS_E_INVALID, "drts_pulse_step: NULL pulse, step < 0 or dt_s <= 0");
        return nan;
    }
    if (p->kind == DRTS_PULSE_IMPULSE) return step == 0 ? 1.0 : 0.0;
    if (p->kind != DRTS_PULSE_GAUSSIAN || !(p->fwhm_s > 0.0)) {
        set_error(DRTS_E_INVALID, "drts_pulse_step: unknown kind %d or fwhm_s <= 0", (int)p->kind);
        return nan;
    }
    // the fraction of the pulse in [a, b) is (erfc(z(a)) - erfc(z(b))) / 2 with
    // z(t) = (t - peak) / (sigma sqrt 2); a = -infinity for step 0 (erfc = 2)
    const double sigma = p->fwhm_s / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const double peak = 3.0 * sigma, w = sigma * std::sqrt(2.0);
    const double hi = std::erfc(((double)(step + 1) * dt_s - peak) / w);
    const double lo = step == 0 ? 2.0 : std::erfc(((double)step * dt_s - peak) / w);
    return 0.5 * (lo - hi);
}

int drts_direction_set(int32_t directions, double *unit, double *weight)
{
    if (directions == DRTS_DIRS_LEBEDEV86) {
        lebedev86(unit, weight);
        return 86;
    }
    if (directions != DRTS_DIRS_LATTICE26) return set_error(DRTS_E_INVALID, "unknown directions %d", directions);
    for (int d = 0; d < kDirs; ++d) {
        const int e[3] = {dir_dx(d), dir_dy(d), dir_dz(d)};
        const double len = std::sqrt((double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
        for (int i = 0; i < 3 && unit; ++i) unit[3 * d + i] = (double)e[i] / len;
        if (weight) weight[d] = 1.0 / kDirs;
    }
    return kDirs;
}

int drts_matrix_info(const drts_matrix_t *A, int64_t *n_states, int64_t *n_escape, int64_t *nnz, int64_t *bytes,
                     double *dt_s)
{
    if (!A) return set_error(DRTS_E_INVALID, "matrix is NULL");
    if (n_states) *n_states = A->m.model.n_states;
    if (n_escape) *n_escape = A->m.model.n_escape;
    if (nnz) *nnz = A->m.nnz;
    if (bytes) *bytes = A->m.bytes();
    if (dt_s) *dt_s = A->m.model.dt_s;
    return DRTS_OK;
}

int drts_matrix_groups(const drts_matrix_t *A, drts_groups_info_t *info)
{
    if (!A || !info) return set_error(DRTS_E_INVALID, "NULL argument");
    if (A->m.n_groups < 0) return set_error(DRTS_E_STATE, "the row groups are not built (no grouped step has run)");
    const bool g = A->m.n_groups > 0;
    info->n_groups = A->m.n_groups;
    info->n_fast = g ? A->m.n_fast : 0;
    info->n_vox2_rows = g ? A->m.n_vox2 : 0;
    info->n_list_rows = g ? A->m.n_slow : 0;
    info->n_list_entries = g ? A->m.n_slow_nnz : 0;
    info->value_tables = g ? A->m.vi_ntab : 0;
    return DRTS_OK;
}

int64_t drts_matrix_row_of(const drts_matrix_t *A, int64_t state, int32_t escape)
{
    if (!A || state < 0 || state >= A->m.model.n_states) return -1;
    if (!escape) return state;
    const auto &es = A->m.model.escape_state;
    auto it = std::lower_bound(es.begin(), es.end(), state);
    if (it == es.end() || *it != state) return -1;
    return A->m.model.n_states + (int64_t)(it - es.begin());
}

int drts_matrix_export_rows(const drts_matrix_t *A, int64_t row0, int64_t n_rows, int64_t *row_ptr, int32_t *col,
                            void *val)
{
    if (!A || !row_ptr) return set_error(DRTS_E_INVALID, "matrix or row_ptr is NULL");
    const Matrix &M = A->m;
    if (!M.has_csr) return set_error(DRTS_E_STATE, "the matrix was built without its CSR arrays");
    if (row0 < 0 || n_rows < 0 || row0 + n_rows > M.model.n_rows) return set_error(DRTS_E_RANGE, "rows out of range");
    hipStream_t s = M.dev.stream;
    if (M.rp64) {
        DRTS_HIP(hipMemcpyAsync(row_ptr, M.row_ptr.as<int64_t>() + row0, (size_t)(n_rows + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
        DRTS_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<int32_t> tmp((size_t)n_rows + 1);
        DRTS_HIP(hipMemcpyAsync(tmp.data(), M.row_ptr.as<int32_t>() + row0, (size_t)(n_rows + 1) * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
        DRTS_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < tmp.size(); ++i) row_ptr[i] = tmp[i];
    }
    const int64_t b = row_ptr[0], n = row_ptr[n_rows] - row_ptr[0];
    const size_t vs = M.model.value_type == DRTS_F64 ? 8 : 4;
    if (col && n) DRTS_HIP(hipMemcpyAsync(col, M.col.as<int32_t>() + b, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    if (val && n)
        DRTS_HIP(hipMemcpyAsync(val, (const char *)M.val.ptr + (size_t)b * vs, (size_t)n * vs, hipMemcpyDeviceToHost, s));
    DRTS_HIP(hipStreamSynchronize(s));
    return DRTS_OK;
}

void drts_matrix_destroy(drts_matrix_t *A) { delete A; }

int drts_solver_create(const drts_matrix_t *A, int32_t n_rhs, const drts_detectors_t *det, int64_t max_steps,
                       const drts_device_t *dev, drts_solver_t **out)
{
    if (!out || !A) return set_error(DRTS_E_INVALID, "NULL argument");
    *out = nullptr;
    if (n_rhs < 1 || n_rhs > 64) return set_error(DRTS_E_INVALID, "n_rhs must be in 1..64");
    if (n_rhs > 1 && A->m.model.value_type != DRTS_F32)
        return set_error(DRTS_E_INVALID, "several right-hand sides need an FP32 matrix");
    if (max_steps < 1) return set_error(DRTS_E_INVALID, "max_steps must be >= 1");
    if (n_rhs == 1) {
        // the single-rhs step kernels gather x with 32-bit byte offsets (the
        // SpMM kernel addresses X with 64-bit offsets)
        const uint64_t vb = A->m.model.value_type == DRTS_F64 ? 8 : 4;
        if ((uint64_t)A->m.model.n_rows * vb >= 0xffffffffull)
            return set_error(DRTS_E_RANGE, "a state vector of %lld rows exceeds 4 GiB",
                             (long long)A->m.model.n_rows);
    }
    drts_solver *S = new (std::nothrow) drts_solver;
    if (!S) return set_error(DRTS_E_NOMEM, "host allocation failed");
    S->dev = make_device(dev);
    S->A = A;
    S->n_rhs = n_rhs;
    S->max_steps = max_steps;
    S->opt = default_options(S);
    const Model &M = A->m.model;
    int rc = DRTS_OK;
    try {
        S->smax_h.reserve((size_t)n_rhs);
        if (det && det->n_det > 0) {
            const int nd_max = n_rhs > 1 ? 32 : 256;
            if (det->n_det > nd_max) rc = set_error(DRTS_E_INVALID, "at most %d detectors", nd_max);
            if (!rc && (!det->det_ptr || !det->state || !det->F)) rc = set_error(DRTS_E_INVALID, "detector arrays");
            for (int d = 0; !rc && d < det->n_det; ++d) {
                for (int64_t i = det->det_ptr[d]; i < det->det_ptr[d + 1]; ++i) {
                    const bool esc = det->escape && det->escape[i];
                    const int64_t r = drts_matrix_row_of(A, det->state[i], esc ? 1 : 0);
                    if (r < 0) {
                        rc = set_error(DRTS_E_INVALID, "detector %d entry %lld: state %lld has no %s row", d,
                                       (long long)i, (long long)det->state[i], esc ? "escape" : "state");
                        break;
                    }
                    S->dets.push_back({r, d, det->F[i]});
                }
            }
            S->n_det = det->n_det;
            std::stable_sort(S->dets.begin(), S->dets.end(),
                             [](const DetEntry &a, const DetEntry &b) { return a.row < b.row; });
        }
        const size_t st = (size_t)M.n_rows * n_rhs * (M.value_type == DRTS_F64 ? 8 : 4);
        // kStatePad entries past the state: aligned 16-byte loads of a run of
        // x that ends near the last row stay in the buffer
        const size_t st_alloc = st + (size_t)kStatePad * n_rhs * (M.value_type == DRTS_F64 ? 8 : 4);
        Device &dv = S->dev;
        if (!rc) rc = S->buf0.allocate(&dv, st_alloc);
        if (!rc) rc = S->buf1.allocate(&dv, st_alloc);
        if (!rc) rc = S->ctl_t.allocate(&dv, n_rhs * sizeof(int64_t));
        if (!rc) rc = S->ctl_E.allocate(&dv, n_rhs * sizeof(int32_t));
        if (!rc) rc = S->ctl_M.allocate(&dv, n_rhs * sizeof(double));
        if (!rc) rc = S->ctl_abs.allocate(&dv, n_rhs * sizeof(double));
        if (!rc) rc = S->t_end.allocate(&dv, sizeof(int64_t));
        if (!rc) rc = S->queue.allocate(&dv, sizeof(int32_t));
        if (!rc) rc = S->ser_tot.allocate(&dv, (size_t)max_steps * 3 * n_rhs * sizeof(double));
        if (!rc) rc = S->ser_det.allocate(&dv, (size_t)max_steps * std::max(S->n_det, 1) * n_rhs * sizeof(double));
        if (!rc) rc = S->ser_exp.allocate(&dv, (size_t)max_steps * n_rhs * sizeof(int32_t));
        if (!rc) rc = S->ser_abs_exp.allocate(&dv, (size_t)max_steps * n_rhs * sizeof(int32_t));
        if (!rc) rc = S->smax.allocate(&dv, (size_t)max_steps * n_rhs * sizeof(double));
        if (!rc) rc = S->amp.allocate(&dv, 16);
        if (!rc) {
            std::vector<int64_t> r(S->dets.size());
            std::vector<int32_t> id(S->dets.size());
            std::vector<double> F(S->dets.size());
            for (size_t i = 0; i < S->dets.size(); ++i) {
                r[i] = S->dets[i].row;
                id[i] = S->dets[i].id;
                F[i] = S->dets[i].F;
            }
            rc = upload_vec(dv, S->det_row, r);
            if (!rc) rc = upload_vec(dv, S->det_id, id);
            if (!rc) rc = upload_vec(dv, S->det_F, F);
            std::vector<int64_t> none;
            if (!rc) rc = upload_vec(dv, S->src_row, none);
            std::vector<int32_t> none32;
            if (!rc) rc = upload_vec(dv, S->src_id, none32);
            if (!rc) rc = upload_vec(dv, S->src_rhs, none32);
            std::vector<double> noned;
            if (!rc) rc = upload_vec(dv, S->src_w, noned);
        }
        if (!rc) {
            hipStream_t s = dv.stream;
            if (hipMemsetAsync(S->buf0.ptr, 0, st_alloc, s) != hipSuccess ||
                hipMemsetAsync(S->buf1.ptr, 0, st_alloc, s) != hipSuccess ||
                hipMemsetAsync(S->ctl_t.ptr, 0, n_rhs * sizeof(int64_t), s) != hipSuccess ||
                hipMemsetAsync(S->ctl_E.ptr, 0, n_rhs * sizeof(int32_t), s) != hipSuccess ||
                hipMemsetAsync(S->ctl_M.ptr, 0, n_rhs * sizeof(double), s) != hipSuccess ||
                hipMemsetAsync(S->ctl_abs.ptr, 0, n_rhs * sizeof(double), s) != hipSuccess ||
                hipMemsetAsync(S->queue.ptr, 0, sizeof(int32_t), s) != hipSuccess ||
                hipMemsetAsync(S->smax.ptr, 0, S->smax.bytes, s) != hipSuccess ||
                hipMemsetAsync(S->ser_tot.ptr, 0, S->ser_tot.bytes, s) != hipSuccess ||
                hipMemsetAsync(S->ser_det.ptr, 0, S->ser_det.bytes, s) != hipSuccess ||
                hipMemcpyAsync(S->t_end.ptr, &S->max_steps, sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess)
                rc = set_error(DRTS_E_HIP, "initialising solver buffers failed");
        }
        if (!rc) rc = prepare(S);
    } catch (const std::bad_alloc &) {
        rc = set_error(DRTS_E_NOMEM, "host allocation failed");
    }
    if (rc) {
        drts_solver_destroy(S);
        return rc;
    }
    *out = S;
    return DRTS_OK;
}

int drts_solver_get_options(const drts_solver_t *S, drts_options_t *opt)
{
    if (!S || !opt) return set_error(DRTS_E_INVALID, "NULL argument");
    *opt = S->opt;
    return DRTS_OK;
}

int drts_solver_set_options(drts_solver_t *S, const drts_options_t *opt)
{
    if (!S || !opt) return set_error(DRTS_E_INVALID, "NULL argument");
    int rc = check_options(S, opt);
    if (rc) return rc;
    if (S->n_rhs > 1 && opt->kernel == DRTS_KERNEL_CSR && opt->variant == DRTS_SPMM_GROUPED_F64SUM) {
        // decided now, so that a matrix whose rows do not group leaves the
        // options as they were
        const Matrix &A = S->A->m;
        if (!long_rows(A) && A.n_groups < 0 && (rc = row_groups(A))) return rc;
        if (long_rows(A) || A.n_groups <= 0)
            return set_error(DRTS_E_INVALID, "DRTS_SPMM_GROUPED_F64SUM needs rows that group (and are not "
                                             "several hundred entries long)");
    }
    S->opt = *opt;
    return prepare(S);
}

int drts_step(drts_solver_t *S, const drts_source_table_t *src)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    if (S->t_host + 1 > S->max_steps) return set_error(DRTS_E_RANGE, "step %lld beyond max_steps", (long long)S->t_host);
    int rc = set_sources(S, src);
    if (!rc) rc = settle_groups(S);
    if (!rc) rc = upload_amplitudes(S, src, S->t_host, 1);
    if (!rc) rc = launch_one(S, S->dev.stream);
    if (rc) return rc;
    S->t_host += 1;
    return DRTS_OK;
}

}  // extern "C"

// ---- the step without allocation ----------------------------------------------
//
// drts_step_noalloc takes the step's scratch memory -- the device copy of the
// step descriptor, the counter of the dynamic walk and the per-chunk FP64
// partials with their finalize segments -- from this file-scope array instead
// of the solver's buffers.  Every device that runs it holds one copy of the
// array until the process ends; its address on a device comes from
// hipGetSymbolAddress (the array's name in host code is not a device address).
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr size_t kScratchInstOff = 0;      // StepInst (well under 1 KiB)
constexpr size_t kScratchQueueOff = 1024;  // int32 work counter
constexpr size_t kScratchPartOff = 4096;   // FP64 partials, then the finalize segments
static_assert(sizeof(StepInst) <= kScratchQueueOff, "step descriptor fits its scratch slot");
constexpr int kScratchMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kScratchMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_on_current_device(unsigned char **out)
{
    int dev = -1;
    DRTS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchMaxDevices) return set_error(DRTS_E_RANGE, "device %d beyond %d", dev, kScratchMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(DRTS_E_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hip_name(e));
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_dev[dev]);
    return DRTS_OK;
}

// Writes the step descriptor into the scratch slot and clears the work counter
// (a kernel, not a memset or a pageable copy: plain stream-ordered writes).
__global__ void stage_step_scratch(StepInst inst, StepInst *dst, int32_t *queue)
{
    if (threadIdx.x == 0) {
        *dst = inst;
        *queue = 0;
    }
}

}  // namespace

extern "C" {

int drts_step_noalloc(drts_solver_t *S, const drts_source_table_t *src)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    if (S->t_host + 1 > S->max_steps) return set_error(DRTS_E_RANGE, "step %lld beyond max_steps", (long long)S->t_host);
    // staging another source table allocates: only the staged one is accepted
    const bool staged = (!src || src->n_src <= 0) ? (S->n_src == 0 && S->src_key == nullptr)
                                                  : (src == S->src_key && src->ctx == S->src_ctx_key &&
                                                     src->n_src == S->n_src);
    if (!staged)
        return set_error(DRTS_E_STATE, "drts_step_noalloc: the source table is not the one staged in the solver "
                                       "(hand it to drts_step or drts_run once first)");
    const StepInst &I0 = S->inst_h;
    const size_t part_bytes = partials_bytes(S->n_det, S->n_rhs, I0.n_chunks);
    if (part_bytes > kScratchBytes - kScratchPartOff)
        return set_error(DRTS_E_RANGE,
                         "drts_step_noalloc: the step needs %zu bytes of partials, the scratch array holds %zu "
                         "(fewer chunks: more tiles per chunk; or use drts_step)",
                         part_bytes, kScratchBytes - kScratchPartOff);
    unsigned char *base = nullptr;
    int rc = scratch_on_current_device(&base);
    if (rc) return rc;
    // amplitudes of this step: host vectors sized when the table was staged
    if ((rc = upload_amplitudes(S, src, S->t_host, 1))) return rc;
    StepInst I = I0;
    I.partials = reinterpret_cast<double *>(base + kScratchPartOff);
    StepInst *inst_dev = reinterpret_cast<StepInst *>(base + kScratchInstOff);
    int32_t *queue = reinterpret_cast<int32_t *>(base + kScratchQueueOff);
    hipLaunchKernelGGL(stage_step_scratch, dim3(1), dim3(64), 0, S->dev.stream, I, inst_dev, queue);
    DRTS_HIP(hipGetLastError());
    if ((rc = launch_one(S, S->dev.stream, inst_dev, queue))) return rc;
    S->t_host += 1;
    return DRTS_OK;
}

int drts_run(drts_solver_t *S, const drts_source_table_t *src, int64_t n_steps)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    if (n_steps < 0 || S->t_host + n_steps > S->max_steps)
        return set_error(DRTS_E_RANGE, "steps %lld..%lld beyond max_steps %lld", (long long)S->t_host,
                         (long long)(S->t_host + n_steps), (long long)S->max_steps);
    // a run of zero steps only stages the source table (and lays the solver
    // out for its step)
    int rc = set_sources(S, src);
    if (!rc) rc = settle_groups(S);
    if (rc || n_steps == 0) return rc;
    rc = upload_amplitudes(S, src, S->t_host, n_steps);
    if (rc) return rc;
    const int K = S->opt.graph_steps;
    int64_t done = 0;
    if (K > 0 && !S->profile && n_steps >= K) {
        if ((rc = ensure_graph(S, K))) return rc;
        for (; done + K <= n_steps; done += K) DRTS_HIP(hipGraphLaunch(S->graph, S->dev.stream));
    }
    for (; done < n_steps; ++done)
        if ((rc = launch_one(S, S->dev.stream))) return rc;
    S->t_host += n_steps;
    return DRTS_OK;
}

int drts_solver_time(const drts_solver_t *S, int64_t *t)
{
    if (!S || !t) return set_error(DRTS_E_INVALID, "NULL argument");
    DRTS_HIP(hipMemcpyAsync(t, S->ctl_t.ptr, sizeof(int64_t), hipMemcpyDeviceToHost, S->dev.stream));
    DRTS_HIP(hipStreamSynchronize(S->dev.stream));
    return DRTS_OK;
}

int drts_detector_readout(const drts_solver_t *S, int64_t first, int64_t count, double *series, int32_t *exp2,
                          double *totals)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    if (first < 0 || count < 0 || first + count > S->max_steps) return set_error(DRTS_E_RANGE, "steps out of range");
    if (count == 0) return DRTS_OK;
    const int nr = S->n_rhs;
    hipStream_t s = S->dev.stream;
    std::vector<int32_t> e((size_t)count * nr), ea((size_t)count * nr);
    DRTS_HIP(hipMemcpyAsync(e.data(), S->ser_exp.as<int32_t>() + first * nr, e.size() * 4, hipMemcpyDeviceToHost, s));
    DRTS_HIP(hipMemcpyAsync(ea.data(), S->ser_abs_exp.as<int32_t>() + first * nr, ea.size() * 4, hipMemcpyDeviceToHost, s));
    if (series && S->n_det > 0)
        DRTS_HIP(hipMemcpyAsync(series, S->ser_det.as<double>() + first * S->n_det * nr,
                                (size_t)count * S->n_det * nr * sizeof(double), hipMemcpyDeviceToHost, s));
    if (totals)
        DRTS_HIP(hipMemcpyAsync(totals, S->ser_tot.as<double>() + first * 3 * nr, (size_t)count * 3 * nr * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    DRTS_HIP(hipStreamSynchronize(s));
    if (totals) {
        // absorbed(t) was summed from x_t (exponent E_t); express it in E_{t+1}
        for (int64_t i = 0; i < count; ++i)
            for (int k = 0; k < nr; ++k) {
                double &a = totals[(i * 3 + 2) * nr + k];
                a = std::ldexp(a, ea[(size_t)(i * nr + k)] - e[(size_t)(i * nr + k)]);
            }
    }
    if (exp2) memcpy(exp2, e.data(), e.size() * 4);
    return DRTS_OK;
}

int drts_detector_window(const drts_solver_t *S, const double *taps, int32_t n_taps, int32_t tap0, int64_t first,
                         int64_t count, double *out, int32_t *out_exp)
{
    if (!S || !taps || !out || !out_exp) return set_error(DRTS_E_INVALID, "NULL argument");
    if (S->n_det < 1) return set_error(DRTS_E_INVALID, "the solver has no detectors");
    if (n_taps < 1 || n_taps > 65536) return set_error(DRTS_E_INVALID, "n_taps must be in 1..65536");
    if (first < 0 || count < 0 || first + count > S->max_steps) return set_error(DRTS_E_RANGE, "steps out of range");
    if (count == 0) return DRTS_OK;
    Device &dev = const_cast<drts_solver *>(S)->dev;
    const size_t n_out = (size_t)count * S->n_det * S->n_rhs;
    Buffer dtaps, dout, dexp;
    int rc;
    if ((rc = dtaps.allocate(&dev, (size_t)S->n_det * n_taps * sizeof(double)))) return rc;
    if ((rc = dout.allocate(&dev, n_out * sizeof(double)))) return rc;
    if ((rc = dexp.allocate(&dev, n_out * sizeof(int32_t)))) return rc;
    DRTS_HIP(hipMemcpyAsync(dtaps.ptr, taps, (size_t)S->n_det * n_taps * sizeof(double), hipMemcpyHostToDevice,
                            dev.stream));
    WindowArgs a;
    a.ser_det = S->ser_det.as<double>();
    a.ser_exp = S->ser_exp.as<int32_t>();
    a.taps = dtaps.as<double>();
    a.n_det = S->n_det;
    a.n_rhs = S->n_rhs;
    a.n_taps = n_taps;
    a.tap0 = tap0;
    a.first = first;
    a.count = count;
    a.t_done = S->t_host;
    a.out = dout.as<double>();
    a.out_exp = dexp.as<int32_t>();
    hipError_t e = launch_detector_window(a, dev.stream);
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "window launch failed: %s", hipGetErrorString(e));
    DRTS_HIP(hipMemcpyAsync(out, dout.ptr, n_out * sizeof(double), hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipMemcpyAsync(out_exp, dexp.ptr, n_out * sizeof(int32_t), hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    return DRTS_OK;
}

int drts_state_read(const drts_solver_t *S, void *host_x, int32_t *exp2, int64_t *t)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    hipStream_t s = S->dev.stream;
    int64_t tt = 0;
    DRTS_HIP(hipMemcpyAsync(&tt, S->ctl_t.ptr, sizeof tt, hipMemcpyDeviceToHost, s));
    DRTS_HIP(hipStreamSynchronize(s));
    const Matrix &A = S->A->m;
    const size_t st = (size_t)A.model.n_rows * S->n_rhs * (A.model.value_type == DRTS_F64 ? 8 : 4);
    if (host_x)
        DRTS_HIP(hipMemcpyAsync(host_x, (tt & 1) ? S->buf1.ptr : S->buf0.ptr, st, hipMemcpyDeviceToHost, s));
    if (exp2) DRTS_HIP(hipMemcpyAsync(exp2, S->ctl_E.ptr, S->n_rhs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DRTS_HIP(hipStreamSynchronize(s));
    if (t) *t = tt;
    return DRTS_OK;
}

int drts_state_write(drts_solver_t *S, const void *host_x, const int32_t *exp2, int64_t t)
{
    if (!S || !host_x || !exp2) return set_error(DRTS_E_INVALID, "NULL argument");
    if (t < 0 || t > S->max_steps) return set_error(DRTS_E_RANGE, "t out of range");
    const Matrix &A = S->A->m;
    const Model &M = A.model;
    const int nr = S->n_rhs;
    const bool f64 = M.value_type == DRTS_F64;
    std::vector<double> mx((size_t)nr, 0.0), ab((size_t)nr, 0.0);
    for (int64_t r = 0; r < M.n_states; ++r) {
        const double a = M.absorb[M.mat_of_voxel[(size_t)(r / M.n_dir)]];
        for (int k = 0; k < nr; ++k) {
            const double v = f64 ? ((const double *)host_x)[r * nr + k] : (double)((const float *)host_x)[r * nr + k];
            mx[(size_t)k] = std::max(mx[(size_t)k], v);
            ab[(size_t)k] += a * v;
        }
    }
    std::vector<int64_t> tv((size_t)nr, t);
    hipStream_t s = S->dev.stream;
    const size_t st = (size_t)M.n_rows * nr * (f64 ? 8 : 4);
    DRTS_HIP(hipMemcpyAsync((t & 1) ? S->buf1.ptr : S->buf0.ptr, host_x, st, hipMemcpyHostToDevice, s));
    DRTS_HIP(hipMemcpyAsync(S->ctl_t.ptr, tv.data(), nr * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DRTS_HIP(hipMemcpyAsync(S->ctl_E.ptr, exp2, nr * sizeof(int32_t), hipMemcpyHostToDevice, s));
    DRTS_HIP(hipMemcpyAsync(S->ctl_M.ptr, mx.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
    DRTS_HIP(hipMemcpyAsync(S->ctl_abs.ptr, ab.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
    DRTS_HIP(hipStreamSynchronize(s));
    S->t_host = t;
    return DRTS_OK;
}

int drts_solver_profile(drts_solver_t *S, int32_t enable)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    int rc = collect_profile(S);
    if (rc) return rc;
    S->profile = enable != 0;
    S->prof_launches = 0;
    S->prof_ms = 0.0;
    return DRTS_OK;
}

int drts_solver_profile_stats(drts_solver_t *S, int64_t *launches, double *total_ms)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    int rc = collect_profile(S);
    if (rc) return rc;
    if (launches) *launches = S->prof_launches;
    if (total_ms) *total_ms = S->prof_ms;
    return DRTS_OK;
}

void drts_solver_destroy(drts_solver_t *S)
{
    if (!S) return;
    if (S->dev.stream) (void)hipStreamSynchronize(S->dev.stream);
    drop_graph(S);
    if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
    for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
    delete S;
}

}  // extern "C"

// ---- uneven batch ------------------------------------------------------------------

namespace {

// Every instance's step limit back to its solver's max_steps (stream-ordered,
// after the batch's launches).
__global__ void restore_t_end(const StepInst *insts, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *const_cast<int64_t *>(insts[i].t_end) = insts[i].max_steps;
}

void release_spent(drts_batch *B)
{
    for (hipGraphExec_t g : B->spent) (void)hipGraphExecDestroy(g);
    B->spent.clear();
}

int batch_launch(drts_batch *B, int64_t n_work, int n_inst, int rows_per_tile, hipStream_t stream,
                 int64_t n_xwork = 0)
{
    const drts_solver *S0 = B->solvers[(size_t)B->lead];
    const int grid = B->grid > 0 ? B->grid : device_cu_count() * 16;
    int32_t *queue = (B->mode == 0 && S0->opt.queue) ? B->queue.as<int32_t>() : nullptr;
    hipError_t e;
    if (B->mode != 0)
        e = launch_structured_batch(B->sas_dev.as<StructArgs>(), B->inst_dev.as<StepInst>(),
                                    B->work_dev.as<WorkItem>(), n_work, B->xwork_dev.as<WorkItem>(), n_xwork, B->mode,
                                    grid, stream);
    else
        e = launch_step(B->inst_dev.as<StepInst>(), B->work_dev.as<WorkItem>(), n_work, n_inst, 1, 0,
                        S0->A->m.rp64 ? 1 : 0, 0, grid,
                        ((long_rows(S0->A->m) ? kVariantLongRows
                                              : (S0->opt.variant == DRTS_SPMV_GROUPED ? DRTS_SPMV_LDS
                                                                                      : S0->opt.variant)) & 15) << 1, nullptr,
                        rows_per_tile, 0, queue, stream);
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "batch step launch failed: %s", hipGetErrorString(e));
    e = launch_finalize(B->inst_dev.as<StepInst>(), n_inst, 1, 0, queue, stream);
    if (e != hipSuccess) return set_error(DRTS_E_HIP, "batch finalize launch failed: %s", hipGetErrorString(e));
    return DRTS_OK;
}

// A member that runs its own grouped step (its rows group and its options ask
// for that step); the others share the batch's launch.
bool batch_own(const drts_solver *S)
{
    return !S->no_group && (S->grouped || S->group_pending);
}

}  // namespace

extern "C" {

int drts_batch_create(drts_solver_t *const *solvers, int32_t n, const drts_device_t *dev, drts_batch_t **out)
{
    if (!out || !solvers || n < 1) return set_error(DRTS_E_INVALID, "need at least one solver");
    *out = nullptr;
    const bool rp64 = solvers[0] && solvers[0]->A->m.rp64;
    for (int i = 0; i < n; ++i) {
        const drts_solver *S = solvers[i];
        if (!S) return set_error(DRTS_E_INVALID, "solver %d is NULL", i);
        if (S->n_rhs != 1 || S->A->m.model.value_type != DRTS_F32)
            return set_error(DRTS_E_INVALID, "solver %d: batches take single-rhs FP32 solvers", i);
        if (S->A->m.rp64 != rp64) return set_error(DRTS_E_INVALID, "solver %d: mixed row-pointer widths", i);
        for (int j = 0; j < i; ++j)
            if (solvers[j] == S) return set_error(DRTS_E_INVALID, "solver %d appears twice", i);
    }
    // small members take the tiled step (their instances share one launch);
    // members large enough to fill the device keep the step by row groups
    for (int i = 0; i < n; ++i) {
        drts_solver *S = solvers[i];
        const bool no_group = S->A->m.model.n_rows < kBatchOwnRows;
        if (S->no_group != no_group) {
            S->no_group = no_group;
            const int e = prepare(S);
            if (e) return e;
        }
    }
    drts_batch *B = new (std::nothrow) drts_batch;
    if (!B) return set_error(DRTS_E_NOMEM, "host allocation failed");
    B->dev = make_device(dev);
    B->solvers.assign(solvers, solvers + n);
    int rc = B->queue.allocate(&B->dev, sizeof(int32_t));
    if (!rc && hipMemsetAsync(B->queue.ptr, 0, sizeof(int32_t), B->dev.stream) != hipSuccess)
        rc = set_error(DRTS_E_HIP, "hipMemsetAsync failed");
    if (!rc && hipStreamSynchronize(B->dev.stream) != hipSuccess) rc = set_error(DRTS_E_HIP, "sync failed");
    if (rc) {
        delete B;
        return rc;
    }
    *out = B;
    return DRTS_OK;
}

int drts_batch_run(drts_batch_t *B, const drts_source_table_t *const *src, const int64_t *n_steps)
{
    if (!B || !n_steps) return set_error(DRTS_E_INVALID, "NULL argument");
    const int n = (int)B->solvers.size();
    std::vector<int> order, own;   // members of the shared launch; members with their own grouped step
    int rc;
    // every member runs the CSR step (step -1), or every member the
    // matrix-free step in the same direction-major mode (1 or 2)
    auto step_of = [](const drts_solver *S) { return structured_of(S) ? structured_mode(S) : -1; };
    const int kind = step_of(B->solvers[0]);
    if (kind != -1 && kind != 1 && kind != 2)
        return set_error(DRTS_E_INVALID, "solver 0: a batch takes the matrix-free step only in modes 1 and 2 "
                                         "(FP32, nearest-rounded values or FP64 row sums, at most %d materials)",
                         kStructMatLdsHost);
    const int mode = kind == -1 ? 0 : kind;
    for (int i = 0; i < n; ++i) {
        drts_solver *S = B->solvers[i];
        if (step_of(S) != kind)
            return set_error(DRTS_E_INVALID, "solver %d: every batch member needs the same step (kernel option)", i);
        if (mode != 0 && (S->sa.seg_len != kStructDmSeg || S->sa.n_mat > kStructMatLdsHost))
            return set_error(DRTS_E_INVALID, "solver %d: matrix-free tiles of another shape", i);
        if (mode == 0 && !S->A->m.has_csr)
            return set_error(DRTS_E_STATE, "solver %d: the CSR step needs the matrix's CSR arrays", i);
        if (n_steps[i] < 0 || S->t_host + n_steps[i] > S->max_steps)
            return set_error(DRTS_E_RANGE, "solver %d: steps beyond max_steps", i);
    }
    // the members of the shared launch need one shape: the first one's
    int lead = -1;
    for (int i = 0; i < n; ++i) {
        const drts_solver *S = B->solvers[i];
        if (mode == 0 && batch_own(S)) continue;
        if (lead < 0) {
            lead = i;
            continue;
        }
        const drts_solver *L = B->solvers[(size_t)lead];
        if (mode == 0 && S->opt.rows_per_tile != L->opt.rows_per_tile)
            return set_error(DRTS_E_INVALID, "solver %d: every batch member needs the same rows_per_tile", i);
        if (mode == 0 && long_rows(S->A->m) != long_rows(L->A->m))
            return set_error(DRTS_E_INVALID, "solver %d: a batch takes either long-row (Lebedev) members or "
                                             "lattice members", i);
    }
    for (int i = 0; i < n; ++i) {
        drts_solver *S = B->solvers[i];
        if (n_steps[i] == 0) continue;
        if ((rc = set_sources(S, src ? src[i] : nullptr))) return rc;
        const bool mine = mode == 0 && batch_own(S);
        if (mine && (rc = settle_groups(S))) return rc;
        if ((rc = upload_amplitudes(S, src ? src[i] : nullptr, S->t_host, n_steps[i]))) return rc;
        // a member whose rows turned out not to group joins the shared launch
        // when it has the shared shape
        if (mine && !S->grouped && lead >= 0 &&
            S->opt.rows_per_tile != B->solvers[(size_t)lead]->opt.rows_per_tile)
            return set_error(DRTS_E_INVALID, "solver %d: every batch member needs the same rows_per_tile", i);
        (mine && S->grouped ? own : order).push_back(i);
    }
    if (order.empty() && own.empty()) return DRTS_OK;
    auto longer = [&](int a, int b) { return n_steps[a] > n_steps[b]; };
    std::stable_sort(order.begin(), order.end(), longer);
    std::stable_sort(own.begin(), own.end(), longer);
    B->lead = order.empty() ? 0 : order[0];
    const int rpt = B->solvers[(size_t)B->lead]->opt.rows_per_tile;
    // instances: the shared launch's (0..P-1), then the own-step members'
    // (their step limits are restored with the others')
    const int P = (int)order.size(), Q = (int)own.size(), T = P + Q;
    std::vector<drts_solver *> all;
    for (int i : order) all.push_back(B->solvers[(size_t)i]);
    for (int i : own) all.push_back(B->solvers[(size_t)i]);
    std::vector<StepInst> insts((size_t)T);
    std::vector<StructArgs> sas;
    std::vector<WorkItem> work, xwork;
    std::vector<int64_t> prefix((size_t)P), xprefix((size_t)P), tend((size_t)T), len_of((size_t)T);
    for (int j = 0; j < T; ++j) {
        drts_solver *S = all[(size_t)j];
        insts[(size_t)j] = S->inst_h;
        len_of[(size_t)j] = n_steps[j < P ? order[(size_t)j] : own[(size_t)(j - P)]];
        tend[(size_t)j] = S->t_host + len_of[(size_t)j];
        if (j >= P) continue;
        for (int64_t c = 0; c < S->n_chunks; ++c) work.push_back({j, (int32_t)c});
        if (mode != 0) {
            sas.push_back(S->sa);
            const int64_t items = (S->sa.n_xrows + kStructXRows - 1) / kStructXRows;
            for (int64_t k = 0; k < items; ++k) xwork.push_back({j, (int32_t)k});
        }
        prefix[(size_t)j] = (int64_t)work.size();
        xprefix[(size_t)j] = (int64_t)xwork.size();
    }
    B->mode = mode;
    Device &dev = B->dev;
    hipStream_t s = dev.stream;
    for (int j = 0; j < T; ++j) {
        drts_solver *S = all[(size_t)j];
        // every solver's own stream work (uploads) must be done before the batch stream uses it
        DRTS_HIP(hipStreamSynchronize(S->dev.stream));
        DRTS_HIP(hipMemcpyAsync(S->t_end.ptr, &tend[(size_t)j], sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    if ((rc = upload_vec(dev, B->inst_dev, insts))) return rc;
    if ((rc = upload_vec(dev, B->work_dev, work))) return rc;
    if (mode != 0) {
        if ((rc = upload_vec(dev, B->sas_dev, sas))) return rc;
        if ((rc = upload_vec(dev, B->xwork_dev, xwork))) return rc;
    }
    DRTS_HIP(hipStreamSynchronize(s));
    release_spent(B);   // the previous run's graphs are done
    if (Q > 0 && !B->fork) {
        DRTS_HIP(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
        for (int a = 0; a < kBatchAuxStreams; ++a) {
            DRTS_HIP(hipStreamCreateWithFlags(&B->aux[a], hipStreamNonBlocking));
            DRTS_HIP(hipEventCreateWithFlags(&B->join[a], hipEventDisableTiming));
        }
    }

    // launches: while step < the length of the j-th longest, the first j+1
    // members of each list are active
    const int K = 25;
    hipStream_t cap = nullptr;
    int64_t step = 0;
    const int64_t n_max = std::max(P ? len_of[0] : 0, Q ? len_of[(size_t)P] : 0);
    while (step < n_max) {
        int active = 0, active_own = 0;
        while (active < P && len_of[(size_t)active] > step) ++active;
        while (active_own < Q && len_of[(size_t)(P + active_own)] > step) ++active_own;
        // both active sets stay constant until the first of their members ends
        int64_t seg_end = n_max;
        if (active) seg_end = std::min(seg_end, len_of[(size_t)active - 1]);
        if (active_own) seg_end = std::min(seg_end, len_of[(size_t)(P + active_own - 1)]);
        const int64_t n_work = active ? prefix[(size_t)active - 1] : 0;
        const int64_t n_xwork = active ? xprefix[(size_t)active - 1] : 0;
        // count steps: the shared launches on st, each large member's steps
        // on an auxiliary stream forked from st and joined back (member j on
        // stream j mod kBatchAuxStreams), so their launch gaps overlap
        const int n_aux = std::min(active_own, kBatchAuxStreams);
        auto steps_on = [&](hipStream_t st, int64_t count) {
            int r = DRTS_OK;
            if (n_aux > 0 && hipEventRecord(B->fork, st) != hipSuccess)
                return set_error(DRTS_E_HIP, "hipEventRecord failed");
            for (int a = 0; a < n_aux; ++a)
                if (hipStreamWaitEvent(B->aux[a], B->fork, 0) != hipSuccess)
                    return set_error(DRTS_E_HIP, "hipStreamWaitEvent failed");
            for (int64_t k = 0; k < count && r == DRTS_OK; ++k) {
                if (active) r = batch_launch(B, n_work, active, rpt, st, n_xwork);
                for (int j = 0; j < active_own && r == DRTS_OK; ++j)
                    r = launch_one(all[(size_t)(P + j)], B->aux[j % kBatchAuxStreams]);
            }
            // joined also after a failed launch: a capture ends only joined
            for (int a = 0; a < n_aux; ++a)
                if (hipEventRecord(B->join[a], B->aux[a]) != hipSuccess ||
                    hipStreamWaitEvent(st, B->join[a], 0) != hipSuccess)
                    if (r == DRTS_OK) r = set_error(DRTS_E_HIP, "stream join failed");
            return r;
        };
        int64_t len = seg_end - step;
        // graph segments only for a batch without own-step members; one with
        // them launches eagerly
        if (len >= 2 * K && Q == 0) {
            if (!cap) DRTS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            DRTS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            rc = steps_on(cap, K);
            hipError_t e = hipStreamEndCapture(cap, &g);
            if (rc == DRTS_OK && e != hipSuccess) rc = set_error(DRTS_E_HIP, "capture: %s", hipGetErrorString(e));
            if (rc == DRTS_OK && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
                rc = set_error(DRTS_E_HIP, "graph instantiate failed");
            if (g) (void)hipGraphDestroy(g);
            for (; rc == DRTS_OK && len >= K; len -= K, step += K)
                if (hipGraphLaunch(ge, s) != hipSuccess) rc = set_error(DRTS_E_HIP, "graph launch failed");
            // destroyed once the stream has run it (next run, or the batch's destruction)
            if (ge) B->spent.push_back(ge);
            if (rc) break;
        }
        if (len > 0) {
            rc = steps_on(s, len);
            step += len;
        }
        if (rc) break;
    }
    if (cap) (void)hipStreamDestroy(cap);
    if (rc) {
        // some steps ran: bring every member back to a consistent state (its
        // own step limit, its step count as the device has it)
        (void)hipStreamSynchronize(s);
        release_spent(B);
        for (drts_solver *S : all) {
            int64_t tt = S->t_host;
            (void)hipMemcpy(S->t_end.ptr, &S->max_steps, sizeof(int64_t), hipMemcpyHostToDevice);
            if (hipMemcpy(&tt, S->ctl_t.ptr, sizeof(int64_t), hipMemcpyDeviceToHost) == hipSuccess) S->t_host = tt;
        }
        return rc;
    }
    for (int j = 0; j < T; ++j) all[(size_t)j]->t_host += len_of[(size_t)j];
    // the solvers' own step limits come back after the batch's launches, in
    // stream order: the call returns without waiting for the steps
    hipLaunchKernelGGL(restore_t_end, dim3((unsigned)((T + 63) / 64)), dim3(64), 0, s, B->inst_dev.as<StepInst>(), T);
    DRTS_HIP(hipGetLastError());
    // work a member's own stream takes later (readout, its own steps) waits for
    // the batch
    if (!B->done) DRTS_HIP(hipEventCreateWithFlags(&B->done, hipEventDisableTiming));
    DRTS_HIP(hipEventRecord(B->done, s));
    for (drts_solver *S : all)
        if (S->dev.stream != s) DRTS_HIP(hipStreamWaitEvent(S->dev.stream, B->done, 0));
    return DRTS_OK;
}

int drts_batch_autotune(drts_batch_t *B, drts_options_t *chosen)
{
    if (!B) return set_error(DRTS_E_INVALID, "batch is NULL");
    const int n = (int)B->solvers.size();
    for (int i = 0; i < n; ++i) {
        if (B->solvers[(size_t)i]->t_host != 0) return set_error(DRTS_E_STATE, "autotune before the first step");
        if (B->solvers[(size_t)i]->opt.kernel != DRTS_KERNEL_CSR)
            return set_error(DRTS_E_INVALID, "solver %d: the batch autotuner takes CSR members", i);
    }
    B->mode = 0;
    Device &dev = B->dev;
    hipStream_t s = dev.stream;
    // members with their own grouped step keep their options: the shape is
    // chosen for the shared launch (groups built now, so that the split is
    // final)
    int rc = DRTS_OK;
    std::vector<int> shared;
    for (int i = 0; i < n; ++i) {
        drts_solver *S = B->solvers[(size_t)i];
        if (batch_own(S) && (rc = settle_groups(S))) return rc;
        if (!(batch_own(S) && S->grouped)) shared.push_back(i);
    }
    const int cus = device_cu_count();
    if (shared.empty()) {
        if (chosen) {
            *chosen = B->solvers[0]->opt;
            chosen->grid = B->grid > 0 ? B->grid : cus * 16;
        }
        return DRTS_OK;
    }
    // every member's state and control words (exponent, maximum, absorbed
    // sum at t = 0), restored afterwards
    std::vector<Buffer> save((size_t)n);
    std::vector<int32_t> save_E((size_t)n);
    std::vector<double> save_M((size_t)n), save_abs((size_t)n);
    for (int i = 0; i < n && !rc; ++i) {
        drts_solver *S = B->solvers[(size_t)i];
        DRTS_HIP(hipStreamSynchronize(S->dev.stream));
        const size_t st = (size_t)S->A->m.model.n_rows * 4;
        if ((rc = save[(size_t)i].allocate(&dev, st))) break;
        DRTS_HIP(hipMemcpyAsync(save[(size_t)i].ptr, S->buf0.ptr, st, hipMemcpyDeviceToDevice, s));
        DRTS_HIP(hipMemcpyAsync(&save_E[(size_t)i], S->ctl_E.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DRTS_HIP(hipMemcpyAsync(&save_M[(size_t)i], S->ctl_M.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
        DRTS_HIP(hipMemcpyAsync(&save_abs[(size_t)i], S->ctl_abs.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (rc) return rc;
    DRTS_HIP(hipStreamSynchronize(s));
    B->lead = shared[0];
    const drts_solver *S0 = B->solvers[(size_t)B->lead];
    int64_t min_steps = INT64_MAX;
    for (const drts_solver *S : B->solvers) min_steps = std::min(min_steps, S->max_steps);
    const int steps = (int)std::max<int64_t>(1, std::min<int64_t>(3, min_steps - 1));
    struct Cand {
        int rpt, tpc, variant, grid;
    };
    std::vector<Cand> cands;
    for (int r : {64, 128, 256})
        for (int c : {1, 2, 4, 8, 16})
            for (int v : {(int)DRTS_SPMV_ROW, (int)DRTS_SPMV_LDS})
                for (int g : {16, 64}) {
                    cands.push_back({r, c, v, cus * g});
                }
    const std::vector<drts_options_t> orig = [&] {
        std::vector<drts_options_t> o;
        for (const drts_solver *S : B->solvers) o.push_back(S->opt);
        return o;
    }();
    // one candidate's options on every member of the shared launch, its lists
    const int n_sh = (int)shared.size();
    std::vector<StepInst> insts((size_t)n_sh);
    std::vector<WorkItem> work;
    auto apply = [&](const Cand &c) -> int {
        work.clear();
        for (int j = 0; j < n_sh; ++j) {
            const int i = shared[(size_t)j];
            drts_solver *S = B->solvers[(size_t)i];
            drts_options_t o = orig[(size_t)i];
            o.rows_per_tile = c.rpt;
            o.tiles_per_chunk = c.tpc;
            o.variant = c.variant;
            o.xcd_remap = 0;
            int e = check_options(S, &o);
            if (e) return e;
            S->opt = o;
            if ((e = prepare(S))) return e;
            insts[(size_t)j] = S->inst_h;
            for (int64_t k = 0; k < S->n_chunks; ++k) work.push_back({j, (int32_t)k});
        }
        B->grid = c.grid;
        int e = upload_vec(dev, B->inst_dev, insts);
        if (!e) e = upload_vec(dev, B->work_dev, work);
        return e;
    };
    std::vector<int64_t> zero_t((size_t)n, 0);
    auto reset_t = [&]() -> int {
        for (int i : shared)
            DRTS_HIP(hipMemcpyAsync(B->solvers[(size_t)i]->ctl_t.ptr, &zero_t[(size_t)i], sizeof(int64_t),
                                    hipMemcpyHostToDevice, s));
        return DRTS_OK;
    };
    hipEvent_t e0, e1;
    DRTS_HIP(hipEventCreate(&e0));
    DRTS_HIP(hipEventCreate(&e1));
    float best_ms = INFINITY;
    Cand best = {S0->opt.rows_per_tile, S0->opt.tiles_per_chunk, S0->opt.variant, cus * 16};
    for (const Cand &c : cands) {
        if ((rc = apply(c))) break;
        const int64_t n_work = (int64_t)work.size();
        if ((rc = reset_t())) break;
        if ((rc = batch_launch(B, n_work, n_sh, c.rpt, s))) break;   // warm-up
        if ((rc = reset_t())) break;
        if (hipEventRecord(e0, s) != hipSuccess) {
            rc = set_error(DRTS_E_HIP, "hipEventRecord failed");
            break;
        }
        for (int k = 0; k < steps && !rc; ++k) rc = batch_launch(B, n_work, n_sh, c.rpt, s);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = set_error(DRTS_E_HIP, "event timing failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // restore every member's state and control words, then apply the choice
    for (int i = 0; i < n; ++i) {
        drts_solver *S = B->solvers[(size_t)i];
        const size_t st = (size_t)S->A->m.model.n_rows * 4;
        DRTS_HIP(hipMemcpyAsync(S->buf0.ptr, save[(size_t)i].ptr, st, hipMemcpyDeviceToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_t.ptr, &zero_t[(size_t)i], sizeof(int64_t), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_E.ptr, &save_E[(size_t)i], sizeof(int32_t), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_M.ptr, &save_M[(size_t)i], sizeof(double), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_abs.ptr, &save_abs[(size_t)i], sizeof(double), hipMemcpyHostToDevice, s));
    }
    DRTS_HIP(hipStreamSynchronize(s));
    if (rc) {
        // leave the members as they were
        for (int i : shared) {
            B->solvers[(size_t)i]->opt = orig[(size_t)i];
            (void)prepare(B->solvers[(size_t)i]);
        }
        B->grid = 0;
        return rc;
    }
    if ((rc = apply(best))) return rc;
    DRTS_HIP(hipStreamSynchronize(s));
    if (chosen) {
        *chosen = B->solvers[(size_t)B->lead]->opt;
        chosen->grid = best.grid;
    }
    return DRTS_OK;
}

void drts_batch_destroy(drts_batch_t *B)
{
    if (!B) return;
    (void)hipStreamSynchronize(B->dev.stream);
    release_spent(B);
    if (B->done) (void)hipEventDestroy(B->done);
    if (B->fork) (void)hipEventDestroy(B->fork);
    for (int a = 0; a < kBatchAuxStreams; ++a) {
        if (B->aux[a]) (void)hipStreamDestroy(B->aux[a]);
        if (B->join[a]) (void)hipEventDestroy(B->join[a]);
    }
    delete B;
}

// ---- autotuning ----------------------------------------------------------------------

static bool f64sum_spmm(const drts_solver *S)
{
    return S->n_rhs > 1 && S->opt.kernel == DRTS_KERNEL_CSR && S->opt.variant == DRTS_SPMM_GROUPED_F64SUM;
}

static std::string tune_key(const drts_solver *S)
{
    const Matrix &A = S->A->m;
    const int rows_cls = (int)std::lround(std::log2((double)std::max<int64_t>(A.model.n_rows, 1)));
    const int nnz_row = (int)std::lround((double)A.nnz / std::max<int64_t>(A.model.n_rows, 1));
    char buf[128];
    // the FP64-sum SpMM gives other results: its shapes are cached apart
    snprintf(buf, sizeof buf, "drts2:rhs%d:f%d%s:rows2^%d:nnzrow%d:cu%d", S->n_rhs,
             A.model.value_type == DRTS_F64 ? 64 : 32, f64sum_spmm(S) ? "s64" : "", rows_cls, nnz_row,
             device_cu_count());
    return buf;
}

int drts_autotune(drts_solver_t *S, const char *cache_path, drts_options_t *chosen)
{
    if (!S) return set_error(DRTS_E_INVALID, "solver is NULL");
    if (S->t_host != 0) return set_error(DRTS_E_STATE, "autotune before the first step");
    // the grouped candidates need the matrix's row groups
    if (!S->no_group && S->opt.kernel == DRTS_KERNEL_CSR && S->A->m.model.value_type == DRTS_F32) {
        int rg = row_groups(S->A->m);
        if (rg) return rg;
    }
    const std::string key = tune_key(S);
    drts_options_t best = S->opt;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char k[128];
            int r, c, g, x, pl;
            bool hit = false;
            while (fscanf(f, "%127s %d %d %d %d %d", k, &r, &c, &g, &x, &pl) == 6) {
                if (key == k) {
                    best.rows_per_tile = r;
                    best.tiles_per_chunk = c;
                    best.grid = g;
                    best.xcd_remap = x;
                    best.variant = f64sum_spmm(S) ? DRTS_SPMM_GROUPED_F64SUM : pl;
                    hit = true;
                }
            }
            fclose(f);
            if (hit && check_options(S, &best) == DRTS_OK) {
                S->opt = best;
                int rc = prepare(S);
                if (!rc && chosen) *chosen = best;
                return rc;
            }
        }
    }
    const Matrix &A = S->A->m;
    hipStream_t s = S->dev.stream;
    const size_t st = (size_t)A.model.n_rows * S->n_rhs * (A.model.value_type == DRTS_F64 ? 8 : 4);
    Buffer save;
    int rc = save.allocate(&S->dev, st);
    if (rc) return rc;
    DRTS_HIP(hipMemcpyAsync(save.ptr, S->buf0.ptr, st, hipMemcpyDeviceToDevice, s));
    const int cus = device_cu_count();
    std::vector<drts_options_t> cands;
    const bool spmm = spmm_of(S);
    const int rows_opts[] = {64, 128, 256};
    const int chunk_opts[] = {2, 4, 16};
    const int grid_mult[] = {4, 8, 16, 32, 64};
    for (int r : rows_opts)
        for (int c : chunk_opts)
            for (int g : grid_mult)
                for (int x = 0; x < 3; ++x)
                    for (int pl = 0; pl <= (spmm ? 0 : DRTS_SPMV_GROUPED); ++pl) {
                        if (pl == DRTS_SPMV_GROUPED && (A.model.value_type == DRTS_F64 || S->no_group)) continue;
                        if (pl == DRTS_SPMV_LDS && A.model.value_type == DRTS_F64) continue;
                        drts_options_t o = S->opt;
                        o.rows_per_tile = r;
                        o.tiles_per_chunk = spmm ? c * 32 : c;
                        o.grid = cus * (spmm ? g / 2 : g);
                        o.xcd_remap = x;
                        o.variant = f64sum_spmm(S) ? DRTS_SPMM_GROUPED_F64SUM : pl;
                        cands.push_back(o);
                    }
    const int steps = (int)std::min<int64_t>(4, S->max_steps);
    hipEvent_t e0, e1;
    DRTS_HIP(hipEventCreate(&e0));
    DRTS_HIP(hipEventCreate(&e1));
    const bool prof = S->profile;
    S->profile = false;
    float best_ms = INFINITY;
    const int64_t zero_t[64] = {0};
    for (const drts_options_t &o : cands) {
        S->opt = o;
        if ((rc = prepare(S))) break;
        DRTS_HIP(hipMemcpyAsync(S->ctl_t.ptr, zero_t, S->n_rhs * sizeof(int64_t), hipMemcpyHostToDevice, s));
        if ((rc = launch_one(S, s))) break;   // warm-up
        DRTS_HIP(hipMemcpyAsync(S->ctl_t.ptr, zero_t, S->n_rhs * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < steps && !rc; ++k) rc = launch_one(S, s);
        DRTS_HIP(hipEventRecord(e1, s));
        DRTS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        DRTS_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = o;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    S->profile = prof;
    // restore the state and control words
    DRTS_HIP(hipMemcpyAsync(S->buf0.ptr, save.ptr, st, hipMemcpyDeviceToDevice, s));
    {
        std::vector<int32_t> z32((size_t)S->n_rhs, 0);
        std::vector<double> zd((size_t)S->n_rhs, 0.0);
        DRTS_HIP(hipMemcpyAsync(S->ctl_t.ptr, zero_t, S->n_rhs * sizeof(int64_t), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_E.ptr, z32.data(), S->n_rhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_M.ptr, zd.data(), S->n_rhs * sizeof(double), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipMemcpyAsync(S->ctl_abs.ptr, zd.data(), S->n_rhs * sizeof(double), hipMemcpyHostToDevice, s));
        DRTS_HIP(hipStreamSynchronize(s));
    }
    if (rc) return rc;
    S->opt = best;
    if ((rc = prepare(S))) return rc;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "a")) {
            fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), best.rows_per_tile, best.tiles_per_chunk, best.grid,
                    best.xcd_remap, best.variant);
            fclose(f);
        }
    }
    if (chosen) *chosen = best;
    return DRTS_OK;
}

}  // extern "C"
