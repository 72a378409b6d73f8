// Serving loop: continuous batching of independent DRTS solves.
//
// A client of the library's own C ABI: each admitted request owns a matrix
// and a single-rhs solver; a tick groups every admitted solver into one
// uneven batch (one launch per step for all of them) and runs a quantum of
// steps.  Admission is by device footprint against a budget; retirement
// copies the series to host memory and frees the request's device memory.
// Submission builds the request's host model outside the server's lock, so
// clients may submit from other threads while a tick runs on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "drts.h"
#include "drts_internal.h"
#include "drts_step.h"

using namespace drts;

namespace {

struct Request {
    int64_t id = 0;
    int64_t n_steps = 0, done = 0;
    int skips = 0;
    // deep copy of the medium
    drts_medium_t med{};
    std::vector<drts_material_t> mats;
    std::vector<uint8_t> map;
    std::vector<int32_t> layer_z0;
    // detectors
    int32_t n_det = 0;
    std::vector<int64_t> det_ptr, det_state;
    std::vector<uint8_t> det_esc;
    std::vector<double> det_F;
    const drts_source_table_t *src = nullptr;
    int64_t est_base = 0;    // footprint bound before assembly, without the CSR arrays
    int64_t est_csr = 0;     // bound of the CSR arrays (built for the CSR step only)
    int64_t est_grp = 0;     // bound of the row groups (CSR step, requests of kBatchOwnRows rows or more)
    int64_t bytes = 0;       // footprint held while admitted
    double work = 0;         // entries of [A; L] (bound) x steps: the shortest-first key
    Model model;             // host model, built once at submission, moved into the matrix
    drts_matrix_t *A = nullptr;
    drts_solver_t *S = nullptr;
    int32_t kernel = DRTS_KERNEL_CSR;   // the step it runs, fixed at admission
    bool batched_mf = false;            // matrix-free with direction-major tiles: joins the matrix-free batch
    bool finished = false;
    // results, copied at retirement
    std::vector<double> series, totals;
    std::vector<int32_t> exp2;

    void free_device()
    {
        if (S) drts_solver_destroy(S);
        if (A) drts_matrix_destroy(A);
        S = nullptr;
        A = nullptr;
    }
    ~Request() { free_device(); }
};

// Device bytes of a solver besides its matrix: two state buffers, the series,
// the amplitude table and the per-chunk partials (bounded by the rows).
int64_t solver_bytes(int64_t n_rows, int64_t n_steps, int32_t n_det, int32_t n_src)
{
    const int64_t series = n_steps * (8 * (3 + std::max(n_det, 1)) + 8);
    const int64_t amp = n_steps * 8 * (std::max(n_src, 1) + 1);
    const int64_t partials = (n_rows / 64 + 256 + 64) * 8 * (4 + n_det);
    return 2 * 4 * n_rows + series + amp + partials + (1 << 20);
}

}  // namespace

struct drts_server {
    drts_device_t dev{};
    hipStream_t build_stream = nullptr;   // admissions assemble here while a quantum runs
    int64_t budget = 0, used = 0;
    int32_t quantum = 0, max_active = 0, max_skips = 0, policy = 0;
    int32_t kernel = DRTS_KERNEL_CSR;   // the step of requests admitted from now on
    // guards next_id and everything below: submissions may run on other
    // threads concurrently with the other calls
    mutable std::mutex mu;
    int64_t next_id = 1;
    std::deque<Request *> waiting;   // ascending id (submission order)
    std::vector<Request *> active;
    std::map<int64_t, std::unique_ptr<Request>> all;
    std::deque<int64_t> unreported;
    drts_batch_t *batch = nullptr;      // the admitted CSR requests
    drts_batch_t *mf_batch = nullptr;   // the admitted matrix-free requests
    bool batch_dirty = true;

    ~drts_server()
    {
        if (batch) drts_batch_destroy(batch);
        if (mf_batch) drts_batch_destroy(mf_batch);
        if (build_stream) {
            (void)hipStreamSynchronize(build_stream);
            (void)hipStreamDestroy(build_stream);
        }
    }
};

namespace {

int copy_request(Request &q, const drts_medium_t *m, const drts_detectors_t *det)
{
    q.med = *m;
    if (m->n_mat < 1 || m->n_mat > 255 || !m->mat) return set_error(DRTS_E_INVALID, "medium materials");
    if (m->grid.nx < 1 || m->grid.ny < 1 || m->grid.nz < 1) return set_error(DRTS_E_INVALID, "grid size");
    q.mats.assign(m->mat, m->mat + m->n_mat);
    q.med.mat = q.mats.data();
    if (m->mat_of_voxel) {
        const size_t nv = (size_t)m->grid.nx * m->grid.ny * m->grid.nz;
        q.map.assign(m->mat_of_voxel, m->mat_of_voxel + nv);
        q.med.mat_of_voxel = q.map.data();
    }
    if (m->geom.kind == DRTS_GEOM_LAYERS_Z && m->geom.n_layers > 0) {
        if (!m->geom.layer_z0) return set_error(DRTS_E_INVALID, "layer_z0 is NULL");
        q.layer_z0.assign(m->geom.layer_z0, m->geom.layer_z0 + m->geom.n_layers);
        q.med.geom.layer_z0 = q.layer_z0.data();
    }
    if (det && det->n_det > 0) {
        if (!det->det_ptr || !det->state || !det->F) return set_error(DRTS_E_INVALID, "detector arrays");
        q.n_det = det->n_det;
        q.det_ptr.assign(det->det_ptr, det->det_ptr + det->n_det + 1);
        const int64_t ne = q.det_ptr.back();
        if (ne < 0) return set_error(DRTS_E_INVALID, "detector entries");
        q.det_state.assign(det->state, det->state + ne);
        q.det_F.assign(det->F, det->F + ne);
        if (det->escape) q.det_esc.assign(det->escape, det->escape + ne);
        else q.det_esc.assign((size_t)ne, 0);
    }
    return DRTS_OK;
}

// Large CSR requests on their own step by row groups inside the server's
// batch: off.  A replay of the full 256-request sphere stream with it on ended
// in a host segmentation fault after 70 requests, whose cause is not known;
// every CSR request takes the shared tiled launch.
constexpr bool kServeOwnGrouped = false;

// Upper bound of the request's device footprint, from the medium alone.  The
// CSR arrays: a row holds at most 26 entries per move group (the plain move
// and each irregular move), every entry 8 bytes (FP32 value, int32 column),
// plus the row pointers.  The tables every step reads or the assembly needs:
// the material map, the direction blocks (FP64 and FP32), the irregular-move
// and escape lists with the row bitmap, and the matrix-free solver's row lists
// (about 32 bytes per irregular or escape row, one bit per row).  A request
// of kBatchOwnRows rows or more takes the CSR step by row groups, whose
// arrays hold the values once more in group order and the two-voxel rows'
// copy (at most 8 bytes per entry in all) and per row at most 117 bytes of
// descriptors, members' rows and materials, row lists, value-indexed slots
// and bricks; the bound adds 64 bytes per row for the sort buffers of their
// construction.
int estimate_bytes(Request &q, int32_t kernel = DRTS_KERNEL_CSR)
{
    Model &M = q.model;
    int rc = build_model(&q.med, &M);
    if (rc) return rc;
    const int64_t n_irr = (int64_t)M.irr_row.size();
    const int64_t nnz_ub = (int64_t)kDirs * (M.n_rows + n_irr);
    q.est_csr = 8 * (nnz_ub + 4) + 8 * (M.n_rows + 1);
    q.est_grp = kServeOwnGrouped && M.n_rows >= kBatchOwnRows ? 8 * nnz_ub + (117 + 64) * M.n_rows + (1 << 20) : 0;
    const int64_t tables = M.n_vox + (int64_t)M.mats.size() * kDirs * kDirs * 12 + 28 * n_irr + 8 * M.n_escape +
                           M.n_states / 8 + 32 * (n_irr + M.n_escape) + M.n_rows / 8 + (1 << 20);
    const int32_t n_src = q.src ? q.src->n_src : 0;
    q.est_base = tables + solver_bytes(M.n_rows, q.n_steps, q.n_det, n_src);
    (void)kernel;
    q.work = (double)nnz_ub * (double)q.n_steps;
    return DRTS_OK;
}

// The footprint bound of a request admitted with `kernel` as its step.
int64_t bound_for(const Request &q, int32_t kernel)
{
    return q.est_base + (kernel == DRTS_KERNEL_CSR ? q.est_csr + q.est_grp : 0);
}

// Assembles an admitted request's matrix (only the tables the matrix-free
// steps read, when it takes one) and creates its solver, on the server's build
// stream -- so that admission overlaps a quantum running on the server's
// stream -- then moves the solver to the server's stream.
int admit(drts_server *Q, Request &q)
{
    // the host model built at submission goes into the matrix (rebuilt if an
    // earlier admission attempt consumed it)
    int rc = DRTS_OK;
    if (!Q->build_stream && hipStreamCreateWithFlags(&Q->build_stream, hipStreamNonBlocking) != hipSuccess)
        return set_error(DRTS_E_HIP, "creating the build stream failed");
    drts_device_t bdev = Q->dev;
    bdev.stream = (void *)Q->build_stream;
    if (q.model.n_states == 0) rc = build_model(&q.med, &q.model);
    if (!rc) rc = build_matrix_from_model(std::move(q.model), &bdev, &q.A, Q->kernel == DRTS_KERNEL_CSR);
    if (rc) return rc;
    drts_detectors_t det{};
    det.n_det = q.n_det;
    det.det_ptr = q.det_ptr.data();
    det.state = q.det_state.data();
    det.escape = q.det_esc.data();
    det.F = q.det_F.data();
    // a large request keeps the step by row groups (on its own in the batch):
    // its groups are built now, so that its footprint counts them (switched
    // off: see kServeOwnGrouped)
    int64_t n_st = 0, n_esc = 0;
    drts_matrix_info(q.A, &n_st, &n_esc, nullptr, nullptr, nullptr);
    const bool own = kServeOwnGrouped && Q->kernel == DRTS_KERNEL_CSR && n_st + n_esc >= kBatchOwnRows;
    if (own) rc = matrix_row_groups(q.A);
    if (!rc) rc = drts_solver_create(q.A, 1, q.n_det > 0 ? &det : nullptr, q.n_steps, &bdev, &q.S);
    if (!rc && Q->kernel == DRTS_KERNEL_CSR && !own) {
        // small requests share the batch's launch: the tiled step (LDS
        // layout, 4 tiles per chunk)
        drts_options_t o{};
        rc = drts_solver_get_options(q.S, &o);
        if (!rc) {
            o.variant = DRTS_SPMV_LDS;
            o.tiles_per_chunk = 4;
            rc = drts_solver_set_options(q.S, &o);
        }
    }
    if (!rc && Q->kernel != DRTS_KERNEL_CSR) {
        // the matrix-free step with its measured launch shape: 8 tiles per
        // chunk, 16 workgroups per CU
        int dev = 0, cus = 0;
        drts_options_t o{};
        rc = drts_solver_get_options(q.S, &o);
        if (!rc && (hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess))
            rc = set_error(DRTS_E_HIP, "device attributes");
        if (!rc) {
            o.kernel = Q->kernel;
            o.tiles_per_chunk = 8;
            o.grid = 16 * std::max(cus, 1);
            rc = drts_solver_set_options(q.S, &o);
        }
    }
    if (!rc) rc = solver_set_stream(q.S, (hipStream_t)Q->dev.stream);
    if (rc) {
        q.free_device();
        return rc;
    }
    q.kernel = Q->kernel;
    if (q.kernel != DRTS_KERNEL_CSR) {
        // the direction-major modes batch: FP64 row sums, or exact values when
        // nearest-rounded, with at most 8 materials
        const bool f64sum = q.kernel == DRTS_KERNEL_STRUCTURED_F64SUM;
        q.batched_mf = q.med.n_mat <= kStructMatLdsHost && (f64sum || q.med.rounding == DRTS_ROUND_NEAREST);
    }
    int64_t n_states = 0, n_escape = 0;
    drts_matrix_info(q.A, &n_states, &n_escape, nullptr, nullptr, nullptr);
    const int32_t n_src = q.src ? q.src->n_src : 0;
    q.bytes = matrix_device_bytes(q.A) + 32 * n_escape + (n_states + n_escape) / 8 +
              solver_bytes(n_states + n_escape, q.n_steps, q.n_det, n_src);
    return DRTS_OK;
}

int retire(drts_server *Q, Request &q)
{
    const int64_t T = q.n_steps;
    q.series.assign((size_t)T * std::max(q.n_det, 1), 0.0);
    q.totals.assign((size_t)T * 3, 0.0);
    q.exp2.assign((size_t)T, 0);
    int rc = drts_detector_readout(q.S, 0, T, q.series.data(), q.exp2.data(), q.totals.data());
    if (rc) return rc;
    q.free_device();
    Q->used -= q.bytes;
    q.bytes = 0;
    q.finished = true;
    Q->unreported.push_back(q.id);
    return DRTS_OK;
}

}  // namespace

extern "C" {

int drts_serve_create(const drts_device_t *dev, int64_t budget_bytes, int32_t quantum, int32_t max_active,
                      int32_t max_skips, int32_t policy, drts_server_t **out)
{
    if (!out) return set_error(DRTS_E_INVALID, "out is NULL");
    if (policy != DRTS_SERVE_ARRIVAL && policy != DRTS_SERVE_SHORTEST)
        return set_error(DRTS_E_INVALID, "unknown admission policy %d", policy);
    *out = nullptr;
    if (budget_bytes <= 0) return set_error(DRTS_E_INVALID, "budget_bytes must be positive");
    if (quantum < 1 || quantum > 100000) return set_error(DRTS_E_INVALID, "quantum in 1..100000");
    if (max_active < 1 || max_active > 4096) return set_error(DRTS_E_INVALID, "max_active in 1..4096");
    if (max_skips < 0) return set_error(DRTS_E_INVALID, "max_skips must be >= 0");
    drts_server *Q = new (std::nothrow) drts_server;
    if (!Q) return set_error(DRTS_E_NOMEM, "host allocation failed");
    if (dev) Q->dev = *dev;
    Q->budget = budget_bytes;
    Q->quantum = quantum;
    Q->max_active = max_active;
    Q->max_skips = max_skips;
    Q->policy = policy;
    *out = Q;
    return DRTS_OK;
}

int drts_serve_set_step(drts_server_t *Q, int32_t kernel)
{
    if (!Q) return set_error(DRTS_E_INVALID, "server is NULL");
    if (kernel != DRTS_KERNEL_CSR && kernel != DRTS_KERNEL_STRUCTURED && kernel != DRTS_KERNEL_STRUCTURED_F64SUM)
        return set_error(DRTS_E_INVALID, "unknown kernel %d", kernel);
    std::lock_guard<std::mutex> lk(Q->mu);
    Q->kernel = kernel;
    return DRTS_OK;
}

int drts_serve_submit(drts_server_t *Q, const drts_medium_t *medium, const drts_source_table_t *src,
                      const drts_detectors_t *det, int64_t n_steps, int64_t *request_id)
{
    if (!Q || !medium || !request_id) return set_error(DRTS_E_INVALID, "NULL argument");
    if (medium->value_type != DRTS_F32) return set_error(DRTS_E_INVALID, "served solves take FP32 media");
    if (medium->directions != DRTS_DIRS_LATTICE26)
        return set_error(DRTS_E_INVALID, "served solves take the 26 lattice directions");
    if (n_steps < 1) return set_error(DRTS_E_INVALID, "n_steps must be >= 1");
    std::unique_ptr<Request> q;
    int rc;
    int64_t id;
    int32_t kernel;
    {
        // the id fixes the request's place in submission order
        std::lock_guard<std::mutex> lk(Q->mu);
        id = Q->next_id++;
        kernel = Q->kernel;
    }
    try {
        // host work (copy, model): outside the lock
        q.reset(new Request);
        q->id = id;
        q->n_steps = n_steps;
        q->src = src;
        q->kernel = kernel;
        rc = copy_request(*q, medium, det);
        if (!rc) rc = estimate_bytes(*q, kernel);
    } catch (const std::bad_alloc &) {
        return set_error(DRTS_E_NOMEM, "host allocation failed");
    }
    if (rc) return rc;
    if (bound_for(*q, kernel) > Q->budget)
        return set_error(DRTS_E_NOMEM, "request needs about %lld bytes, beyond the budget of %lld",
                         (long long)bound_for(*q, kernel), (long long)Q->budget);
    std::lock_guard<std::mutex> lk(Q->mu);
    auto at = Q->waiting.end();
    while (at != Q->waiting.begin() && (*(at - 1))->id > id) --at;
    Q->waiting.insert(at, q.get());
    *request_id = id;
    Q->all[id] = std::move(q);
    return DRTS_OK;
}

int drts_serve_footprint(const drts_medium_t *medium, const drts_source_table_t *src, const drts_detectors_t *det,
                         int64_t n_steps, int64_t *bytes)
{
    if (!medium || !bytes) return set_error(DRTS_E_INVALID, "NULL argument");
    if (n_steps < 1) return set_error(DRTS_E_INVALID, "n_steps must be >= 1");
    int rc;
    try {
        Request q;
        q.n_steps = n_steps;
        q.src = src;
        rc = copy_request(q, medium, det);
        if (!rc) rc = estimate_bytes(q, DRTS_KERNEL_CSR);
        if (!rc) *bytes = bound_for(q, DRTS_KERNEL_CSR);
    } catch (const std::bad_alloc &) {
        return set_error(DRTS_E_NOMEM, "host allocation failed");
    }
    return rc;
}

int drts_serve_tick(drts_server_t *Q, int32_t *n_active, int32_t *n_waiting, int32_t *n_finished,
                    int64_t *bytes_in_use)
{
    if (!Q) return set_error(DRTS_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(Q->mu);
    int rc = DRTS_OK;
    int32_t finished = 0;
    // admission: first fit in the policy's order; a request passed over
    // max_skips times blocks the ones behind it
    auto admission = [&]() -> int {
        if (Q->policy == DRTS_SERVE_SHORTEST)
            // least work first; ties keep arrival order
            std::stable_sort(Q->waiting.begin(), Q->waiting.end(),
                             [](const Request *a, const Request *b) { return a->work < b->work; });
        std::vector<Request *> passed;   // earlier requests that did not fit this tick
        for (auto it = Q->waiting.begin(); it != Q->waiting.end() && (int)Q->active.size() < Q->max_active;) {
            Request &q = **it;
            if (Q->used + bound_for(q, Q->kernel) <= Q->budget) {
                int r = admit(Q, q);
                if (r) return r;
                Q->used += q.bytes;
                Q->active.push_back(&q);
                Q->batch_dirty = true;
                for (Request *p : passed) ++p->skips;
                it = Q->waiting.erase(it);
                continue;
            }
            if (q.skips >= Q->max_skips) break;
            passed.push_back(&q);
            ++it;
        }
        return DRTS_OK;
    };
    // 1. with nothing running, admit first; otherwise the admissions below
    //    assemble on the build stream while this tick's quantum runs
    const bool admit_first = Q->active.empty();
    if (admit_first && (rc = admission())) return rc;
    // 2. one quantum for every request admitted before: the CSR ones as one
    //    batch, the matrix-free ones of the batched kind (direction-major
    //    tiles) as another (one launch per kernel and step each), any other
    //    matrix-free one with its own graph-replayed run, all in turn on the
    //    server's stream; the launches return without waiting for the steps
    std::vector<Request *> ran = Q->active;
    if (!ran.empty()) {
        std::vector<Request *> csr, mf, solo;
        for (Request *q : ran) {
            if (q->kernel == DRTS_KERNEL_CSR) csr.push_back(q);
            else if (q->batched_mf) mf.push_back(q);
            else solo.push_back(q);
        }
        if (Q->batch_dirty) {
            for (drts_batch_t **b : {&Q->batch, &Q->mf_batch}) {
                if (*b) drts_batch_destroy(*b);
                *b = nullptr;
            }
            for (int k = 0; k < 2; ++k) {
                std::vector<drts_solver_t *> ss;
                for (Request *q : (k == 0 ? csr : mf)) ss.push_back(q->S);
                if (!ss.empty() && (rc = drts_batch_create(ss.data(), (int32_t)ss.size(), &Q->dev,
                                                           k == 0 ? &Q->batch : &Q->mf_batch)))
                    return rc;
            }
            Q->batch_dirty = false;
        }
        for (int k = 0; k < 2; ++k) {
            std::vector<Request *> &group = k == 0 ? csr : mf;
            if (group.empty()) continue;
            std::vector<const drts_source_table_t *> tabs;
            std::vector<int64_t> steps;
            for (Request *q : group) {
                tabs.push_back(q->src);
                steps.push_back(std::min<int64_t>(Q->quantum, q->n_steps - q->done));
            }
            if ((rc = drts_batch_run(k == 0 ? Q->batch : Q->mf_batch, tabs.data(), steps.data()))) return rc;
            for (size_t i = 0; i < group.size(); ++i) group[i]->done += steps[i];
        }
        for (Request *q : solo) {
            const int64_t n = std::min<int64_t>(Q->quantum, q->n_steps - q->done);
            if ((rc = drts_run(q->S, q->src, n))) return rc;
            q->done += n;
        }
    }
    // 3. admissions overlapping the quantum (they join the next one)
    if (!admit_first && (rc = admission())) return rc;
    if (!ran.empty()) DRTS_HIP(hipStreamSynchronize((hipStream_t)Q->dev.stream));
    // 4. retirement
    bool retired = false;
    std::vector<Request *> keep;
    for (Request *q : Q->active) {
        if (q->done >= q->n_steps) {
            if ((rc = retire(Q, *q))) return rc;
            ++finished;
            retired = true;
        } else {
            keep.push_back(q);
        }
    }
    Q->active.swap(keep);
    if (retired) {
        // the batches refer to retired solvers: drop them before anything else runs
        Q->batch_dirty = true;
        for (drts_batch_t **b : {&Q->batch, &Q->mf_batch}) {
            if (*b) drts_batch_destroy(*b);
            *b = nullptr;
        }
    }
    if (n_active) *n_active = (int32_t)Q->active.size();
    if (n_waiting) *n_waiting = (int32_t)Q->waiting.size();
    if (n_finished) *n_finished = finished;
    if (bytes_in_use) *bytes_in_use = Q->used;
    return DRTS_OK;
}

int drts_serve_poll(drts_server_t *Q, int64_t *ids, int32_t cap, int32_t *n_out)
{
    if (!Q || !n_out || (cap > 0 && !ids)) return set_error(DRTS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(Q->mu);
    int32_t n = 0;
    while (n < cap && !Q->unreported.empty()) {
        ids[n++] = Q->unreported.front();
        Q->unreported.pop_front();
    }
    *n_out = n;
    return DRTS_OK;
}

int drts_serve_result(const drts_server_t *Q, int64_t request_id, double *series, int32_t *exp2, double *totals)
{
    if (!Q) return set_error(DRTS_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(Q->mu);
    auto it = Q->all.find(request_id);
    if (it == Q->all.end()) return set_error(DRTS_E_INVALID, "unknown request %lld", (long long)request_id);
    const Request &q = *it->second;
    if (!q.finished) return set_error(DRTS_E_STATE, "request %lld has not finished", (long long)request_id);
    if (series && q.n_det > 0) memcpy(series, q.series.data(), (size_t)q.n_steps * q.n_det * sizeof(double));
    if (exp2) memcpy(exp2, q.exp2.data(), (size_t)q.n_steps * sizeof(int32_t));
    if (totals) memcpy(totals, q.totals.data(), (size_t)q.n_steps * 3 * sizeof(double));
    return DRTS_OK;
}

int drts_serve_release(drts_server_t *Q, int64_t request_id)
{
    if (!Q) return set_error(DRTS_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(Q->mu);
    auto it = Q->all.find(request_id);
    if (it == Q->all.end()) return set_error(DRTS_E_INVALID, "unknown request %lld", (long long)request_id);
    if (!it->second->finished) return set_error(DRTS_E_STATE, "request %lld has not finished", (long long)request_id);
    Q->all.erase(it);
    return DRTS_OK;
}

void drts_serve_destroy(drts_server_t *Q) { delete Q; }

}  // extern "C"
