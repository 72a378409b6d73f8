// DRTS time step on gfx950: J(t+1) = A J(t) + B P(t) (Eq. (26)) with the
// one-step detector sums of Eq. (27), for one or many solvers per launch.
//
// Single right-hand side (SpMV).  A persistent grid walks a list of work items
// (instance, chunk of row tiles).  For every tile of R rows the workgroup
// streams the tile's contiguous run of (value, column) pairs with 16-byte
// nontemporal loads (the matrix is read once per step and must not evict the
// state from L2/MALL), gathers x for each entry, stages the products in LDS
// and lets one thread per row sum its own run in ascending column order.  The
// epilogue of the same tile applies the power-of-two rescale, injects the
// step's source photons, stores y, and accumulates FP64 totals (photons in
// the grid, escaped, to be absorbed next step), the FP32 maximum for the next
// rescale and the detector sums.  Per-chunk partials are reduced by the
// finalize kernel in a fixed order, so results do not depend on scheduling.
//
// Many right-hand sides (SpMM).  Same work list; each wavefront owns a row at
// a time and its 64 lanes are the right-hand sides (X is [rows][rhs], so one
// column of A touches a contiguous 4*n_rhs-byte row of X); the column index
// and value of an entry are uniform across the wavefront.
//
// XCD-aware order: with xcd_remap the work list is cut into 8 contiguous
// ranges and the workgroups dispatched to one XCD (round robin by workgroup
// id) walk one range, so each XCD's L2 holds one moving window of x.
#include <type_traits>

#include "drts_internal.h"
#include "drts_step.h"

namespace drts {
namespace {

constexpr int kNT = 256;     // threads per workgroup
constexpr int kXcds = 8;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Pointers into device memory are marked as global (address space 1): the
// descriptors are read from memory, so the compiler would otherwise emit flat
// accesses, which may alias LDS and serialise every gather behind the LDS
// stores.
#define GLB __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const GLB T *gp(const T *p) { return (const GLB T *)p; }
template <typename T> __device__ __forceinline__ GLB T *gpw(T *p) { return (GLB T *)p; }
// Data that no kernel of the step writes (coefficient tables): marked
// constant, so loads at wave-uniform addresses go through the scalar cache
// into SGPRs and feed vector instructions without a broadcast.
#define CST __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ const CST T *cst(const T *p) { return (const CST T *)p; }

template <typename VT> struct Quad;
template <> struct Quad<float> {
    f4 v;
    __device__ __forceinline__ void load(const GLB float *p) { v = __builtin_nontemporal_load((const GLB f4 *)p); }
    __device__ __forceinline__ float operator[](int j) const { return v[j]; }
};
template <> struct Quad<double> {
    d2 a, b;
    __device__ __forceinline__ void load(const GLB double *p)
    {
        a = __builtin_nontemporal_load((const GLB d2 *)p);
        b = __builtin_nontemporal_load((const GLB d2 *)(p + 2));
    }
    __device__ __forceinline__ double operator[](int j) const { return j < 2 ? a[j] : b[j - 2]; }
};

struct Scale {
    int k;   // x_t is multiplied by 2^-k
    int En;  // exponent of x_{t+1}
};

// Exponent bookkeeping shared by the step and the finalize kernels: the step
// scales x_t by 2^-k so that max(x_t, s_t 2^-E_t) 2^-k lies in [0.5, 1).
__device__ __forceinline__ Scale step_scale(const StepInst &I, int rhs, int64_t t)
{
    const int E = I.E[rhs];
    int k = 0;
    if (I.rescale) {
        double want = I.M[rhs];
        const double sx = ldexp(I.smax[t * I.n_rhs + rhs], -E);
        if (sx > want) want = sx;
        if (want > 0.0) (void)frexp(want, &k);
        if (k < -126) k = -126;
    }
    return {k, E + k};
}

template <int NT = kNT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <int NT = kNT>
__device__ __forceinline__ double block_max(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Butterfly sum / max over a wavefront; lane 0's result has a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <typename IT>
__device__ __forceinline__ int lower_bound_rows(const int64_t *rows, int lo, int hi, int64_t key)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rows[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Work-list order: plain grid stride, or 8 contiguous ranges (one per XCD).
struct Walk {
    int64_t begin, end, stride;
};
__device__ __forceinline__ Walk walk_of(int64_t n_work, int xcd_remap, const int64_t *xcd_bounds)
{
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (xcd_remap && G % kXcds == 0 && G >= kXcds) {
        // workgroups are dispatched to the XCDs round robin: b % kXcds is b's XCD
        const int64_t x = b % kXcds, local = b / kXcds, per = G / kXcds;
        const int64_t lo = xcd_bounds ? xcd_bounds[x] : x * n_work / kXcds;
        const int64_t hi = xcd_bounds ? xcd_bounds[x + 1] : (x + 1) * n_work / kXcds;
        return {lo + local, hi, per};
    }
    return {b, n_work, G};
}

// ---------------------------------------------------------------------------
// SpMV step (one right-hand side)
//
// One row per thread (NT rows per tile).  Per chunk, the tile bounds
// (row_ptr at tile starts), the per-tile source/detector offsets and the
// absorption table go to LDS once, so a tile needs two dependent round trips
// only: {values, columns, own row pointers, material} issued together, then
// the x gathers.  The stage holds 32 entries per row; a tile with more
// entries (rare: long rows) takes the multi-pass path.
// ---------------------------------------------------------------------------
constexpr int kChunkMax = 64;   // tiles per chunk staged in LDS
constexpr int kMatMax = 256;

// Buffer resources (gfx9 layout: 64-bit base, byte range, 0x00020000) let the
// streaming loads use 32-bit offsets from a scalar base instead of a 64-bit
// address per lane, and return zero for an offset past the range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint64_t bytes)
{
    const uint32_t n = bytes >= 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}
// A value every lane holds the same, made a scalar: loads of control words
// from device memory land in vector registers, and anything derived from
// them (the state buffer chosen by the step's parity, the buffer descriptors
// built on it) would otherwise need a per-lane descriptor loop at every use.
__device__ __forceinline__ int64_t scalar_i64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

constexpr int kStream = 2;  // cache policy bits of a buffer load: nontemporal
// s_waitcnt immediate (gfx9 encoding): vmcnt <= 1, expcnt and lgkmcnt not waited on
constexpr int kWaitVm1 = 0x0F71;

template <typename VT> struct BufQuad;
template <> struct BufQuad<float> {
    __device__ static Quad<float> load(__amdgpu_buffer_rsrc_t rs, uint32_t off)
    {
        Quad<float> q;
        q.v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kStream));
        return q;
    }
    __device__ static float gather(__amdgpu_buffer_rsrc_t rs, int32_t c)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, c * 4, 0, 0));
    }
};
template <> struct BufQuad<double> {
    __device__ static Quad<double> load(__amdgpu_buffer_rsrc_t rs, uint32_t off)
    {
        Quad<double> q;
        q.a = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kStream));
        q.b = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off + 16, 0, kStream));
        return q;
    }
    __device__ static double gather(__amdgpu_buffer_rsrc_t rs, int32_t c)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, c * 8, 0, 0));
    }
};

// Entries of one tile held in registers between their loads and the gathers.
template <typename VT, typename IT, int U> struct TileRegs {
    Quad<VT> qv[U];
    i4 qc[U];
    uint32_t qo[U];   // entry offset of each quad from a0
    IT a0, b, e;
    IT mylo, myhi;
    int q;
};

template <typename VT, typename IT, int NT, int U, int R>
__device__ __forceinline__ void issue_tile(TileRegs<VT, IT, U> &T, const GLB IT *rp, const GLB int32_t *col,
                                           const GLB VT *val, const GLB uint8_t *mat, IT b, IT e, int64_t r0,
                                           int nr, int64_t n_states, uint64_t vmul, int64_t nnz)
{
    const int tid = threadIdx.x;
    const int64_t r = r0 + tid;
    T.b = b;
    T.e = e;
    T.mylo = 0;
    T.myhi = 0;
    T.q = 0;
    if (tid < nr && tid < R) {
        T.mylo = rp[r];
        T.myhi = rp[r + 1];
        if (r < n_states) T.q = mat[vox_of(r, vmul)];
    }
    // Every lane runs U quads without branches: a quad index at or past e is
    // clamped to the last quad holding entries of the tile, so the lane
    // re-reads cached data and rewrites the same products into the same LDS
    // slots.  Entries of a loaded quad outside [b, e) belong to neighbouring
    // tiles or to the zero padding: their columns are valid state indices
    // and their products land in LDS slots no row of this tile reads.
    T.a0 = b & ~(IT)3;
    const uint32_t last = e > T.a0 ? (uint32_t)(((e - 1 - T.a0) >> 2) << 2) : 0u;   // an empty tile re-reads its first quad
    const uint32_t span = (uint32_t)(e - T.a0);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint32_t i = 4u * (uint32_t)(tid + k * NT);
        T.qo[k] = i < span ? i : last;
    }
    const int64_t base = (int64_t)T.a0;
    const uint64_t left = (uint64_t)(nnz + 4 - base);
    const __amdgpu_buffer_rsrc_t rc = make_rsrc((const void *)(col + base), left * 4);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc((const void *)(val + base), left * sizeof(VT));
#pragma unroll
    for (int k = 0; k < U; ++k) {
        T.qc[k] = __builtin_amdgcn_raw_buffer_load_b128(rc, (int)(T.qo[k] * 4), 0, kStream);
        T.qv[k] = BufQuad<VT>::load(rv, T.qo[k] * (uint32_t)sizeof(VT));
    }
}

// gathers x, stages the products, sums each thread's row in column order
template <typename VT, typename IT, int NT, int U, int R>
__device__ __forceinline__ VT finish_tile(const TileRegs<VT, IT, U> &T, __amdgpu_buffer_rsrc_t rx, VT *s_prod)
{
    VT xv[U][4];
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) xv[k][jj] = BufQuad<VT>::gather(rx, T.qc[k][jj]);
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) s_prod[T.qo[k] + jj] = T.qv[k][jj] * xv[k][jj];
    __syncthreads();
    VT acc = 0;
    IT jj = T.mylo;
    for (; jj + 4 <= T.myhi; jj += 4) {
        const VT p0 = s_prod[jj - T.a0], p1 = s_prod[jj - T.a0 + 1];
        const VT p2 = s_prod[jj - T.a0 + 2], p3 = s_prod[jj - T.a0 + 3];
        acc += p0;
        acc += p1;
        acc += p2;
        acc += p3;
    }
    for (; jj < T.myhi; ++jj) acc += s_prod[jj - T.a0];
    return acc;
}

// Quad layout with the values loaded straight into LDS (gfx950 buffer loads
// with the lds flag): the data of lane l of a wave instruction lands at
// M0 + 16 l, so quad q = tid + k NT of the tile lands at entries 4q .. 4q+3 of
// the stage, exactly where its products go.  Only the columns pass through
// registers (28 fewer VGPRs than the quad layout: five resident workgroups
// per CU instead of four).  Each lane later reads back only the quads it
// loaded itself, so the product step needs no barrier.
template <typename IT, int U> struct TileRegsL {
    i4 qc[U];
    IT b, e;
    IT mylo, myhi, a0;
    int q;
};

template <typename IT, int NT, int U, int R>
__device__ __forceinline__ void issue_tile_l(TileRegsL<IT, U> &T, const GLB IT *rp, const GLB int32_t *col,
                                             const GLB float *val, const GLB uint8_t *mat, IT b, IT e, int64_t r0,
                                             int nr, int64_t n_states, uint64_t vmul, int64_t nnz, float *s_prod)
{
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t r = r0 + tid;
    T.b = b;
    T.e = e;
    T.mylo = 0;
    T.myhi = 0;
    T.q = 0;
    if (tid < nr && tid < R) {
        T.mylo = rp[r];
        T.myhi = rp[r + 1];
        if (r < n_states) T.q = mat[vox_of(r, vmul)];
    }
    // quads past the tile re-read its last quad (in bounds, as in the quad
    // layout) into slots no row of the tile reads
    T.a0 = b & ~(IT)3;
    const uint32_t last = e > T.a0 ? (uint32_t)(((e - 1 - T.a0) >> 2) << 2) : 0u;   // an empty tile re-reads its first quad
    const uint32_t span = (uint32_t)(e - T.a0);
    const int64_t base = (int64_t)T.a0;
    const uint64_t left = (uint64_t)(nnz + 4 - base);
    const __amdgpu_buffer_rsrc_t rc = make_rsrc((const void *)(col + base), left * 4);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc((const void *)(val + base), left * 4);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const uint32_t i = 4u * (uint32_t)(tid + k * NT);
        const uint32_t o = i < span ? i : last;
        T.qc[k] = __builtin_amdgcn_raw_buffer_load_b128(rc, (int)(o * 4), 0, kStream);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, (__attribute__((address_space(3))) void *)(s_prod + 4 * (64 * wave + k * NT)),
                                                 16, (int)(o * 4), 0, 0, kStream);
    }
}

// after_gathers runs once the gathers are issued; when it issues one store
// from this wave (stored), the wait leaves that store, the newest memory
// operation, in flight
template <typename IT, int NT, int U, int R, typename F>
__device__ __forceinline__ float finish_tile_l(const TileRegsL<IT, U> &T, __amdgpu_buffer_rsrc_t rx, float *s_prod,
                                               F after_gathers, bool stored)
{
    const int tid = threadIdx.x;
    float xv[U][4];
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) xv[k][jj] = BufQuad<float>::gather(rx, T.qc[k][jj]);
    after_gathers();
    // the values of this lane's quads are in LDS once every load of the lane
    // has completed (the compiler does not order LDS reads after
    // LDS-destination loads by itself)
    if (stored) __builtin_amdgcn_s_waitcnt(kWaitVm1);
    else __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        f4 *slot = (f4 *)(s_prod + 4 * (tid + k * NT));
        f4 v = *slot;
        v[0] = v[0] * xv[k][0];
        v[1] = v[1] * xv[k][1];
        v[2] = v[2] * xv[k][2];
        v[3] = v[3] * xv[k][3];
        *slot = v;
    }
    __syncthreads();
    float acc = 0;
    IT jj = T.mylo;
    for (; jj + 4 <= T.myhi; jj += 4) {
        const float p0 = s_prod[jj - T.a0], p1 = s_prod[jj - T.a0 + 1];
        const float p2 = s_prod[jj - T.a0 + 2], p3 = s_prod[jj - T.a0 + 3];
        acc += p0;
        acc += p1;
        acc += p2;
        acc += p3;
    }
    for (; jj < T.myhi; ++jj) acc += s_prod[jj - T.a0];
    return acc;
}

// R threads stream the entries of R rows, one row per thread and 7 quads of
// entries per thread.  LAY = 0: quads through registers; LAY = 2: the values
// loaded straight into LDS (FP32 values only).
template <typename VT, typename IT, int R, int LAY>
__global__ void __launch_bounds__(R, (LAY == 2 && sizeof(VT) == 4 && sizeof(IT) == 4 && R >= 128 ? 5 : 1)) step_spmv(const StepInst *__restrict__ insts,
                                                 const WorkItem *__restrict__ work, int64_t n_work,
                                                 int xcd_remap, const int64_t *__restrict__ xcd_bounds,
                                                 int32_t *__restrict__ queue)
{
    constexpr int NT = R;
    constexpr int NW = NT / 64;
    __shared__ int64_t s_wi;
    __shared__ double s_wred[4][NW];
    constexpr int U = 7;                 // quads of entries per thread
    constexpr int CAP = 4 * U * NT;      // entries staged per pass (28 per row)
    static_assert(U >= 1 && CAP >= 28 * R, "tile shape");
    constexpr int LAYV = (LAY == 2 && sizeof(VT) != 4) ? 0 : LAY;   // FP64 values: quads
    __shared__ __attribute__((aligned(16))) VT s_prod[CAP];
    __shared__ IT s_tb[kChunkMax + 1];
    __shared__ int32_t s_src[kChunkMax + 1];
    __shared__ int32_t s_det[kChunkMax + 1];
    __shared__ double s_abs[kMatMax];
    __shared__ VT s_y[R];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    // LDS layout: a tile's y values are stored only after the next tile's
    // gathers have been issued, so the wait for those gathers (and for the
    // values landing in LDS) need not wait for the store as well.  The pending
    // tile: its y, first row and row count (uniform), each lane's value.
    GLB VT *pend_y = nullptr;
    int64_t pend_r0 = 0;
    int pend_nr = 0;
    VT pend_v = 0;
    auto flush = [&]() {
        if (pend_y) {
            // a buffer store: the tile's base in SGPRs, each lane's 32-bit offset
            if (threadIdx.x < pend_nr && (int)threadIdx.x < R) {
                if constexpr (sizeof(VT) == 4)
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __builtin_bit_cast(uint32_t, pend_v),
                        make_rsrc((const void *)(pend_y + pend_r0), (uint64_t)pend_nr * 4), (int)(4 * threadIdx.x), 0, 0);
                else
                    pend_y[pend_r0 + threadIdx.x] = pend_v;
            }
            pend_y = nullptr;
        }
    };
    // work items come from a global counter (dynamic balance) or a fixed walk
    int64_t wi = wk.begin;
    int cached = -1;
    int64_t t = 0;
    bool live = false;
    Scale sc{0, 0};
    VT scale = 1;
    for (;; wi += wk.stride) {
        if (queue) {
            if (tid == 0) s_wi = atomicAdd(queue, 1);
            __syncthreads();
            wi = s_wi;
            __syncthreads();   // every thread has read s_wi before thread 0 may write it again
        }
        if (wi >= (queue ? n_work : wk.end)) break;
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        if (item.inst != cached) {
            // per-instance constants of this launch, read once per workgroup
            cached = item.inst;
            t = I.t[0];
            live = t < *I.t_end;
            if (live) {
                sc = step_scale(I, 0, t);
                scale = (VT)ldexp(1.0, -sc.k);
            }
        }
        if (!live) continue;
        const GLB IT *rp = gp((const IT *)I.row_ptr);
        const GLB int32_t *col = gp(I.col);
        const GLB VT *val = gp((const VT *)I.val);
        const GLB VT *x = gp((const VT *)((t & 1) ? I.buf1 : I.buf0));
        const __amdgpu_buffer_rsrc_t rx = make_rsrc((const void *)x, (uint64_t)I.n_rows * sizeof(VT));
        GLB VT *y = gpw((VT *)((t & 1) ? I.buf0 : I.buf1));
        const GLB uint8_t *mat = gp(I.mat);
        const int64_t n_rows = I.n_rows, n_states = I.n_states;
        const uint64_t vmul = I.vox_mul;
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int ntc = (int)min((int64_t)I.tiles_per_chunk, I.n_tiles - tile0);

        // chunk prologue
        for (int j = tid; j <= ntc; j += NT) {
            s_tb[j] = rp[min((tile0 + j) * R, n_rows)];
            s_src[j] = gp(I.src_tile)[tile0 + j];
            s_det[j] = gp(I.det_tile)[tile0 + j];
        }
        for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
        __syncthreads();

        double sN = 0.0, sE = 0.0, sA = 0.0, dsum = 0.0;
        VT mx = 0;
        auto fits = [&](int j) { return s_tb[j + 1] - s_tb[j] <= (IT)CAP - 3; };
        auto rows_of = [&](int j) { return (int)min((int64_t)R, n_rows - (tile0 + j) * R); };
        for (int j = 0; j < ntc; ++j) {
            const int64_t r0 = (tile0 + j) * R;
            const int nr = rows_of(j);
            const int64_t r = r0 + tid;
            const bool own = tid < nr && tid < R;
            VT acc = 0;
            int q = 0;
            if (LAYV == 2 && fits(j)) {
                if constexpr (sizeof(VT) == 4) {
                    TileRegsL<IT, U> tl;
                    issue_tile_l<IT, NT, U, R>(tl, rp, col, (const GLB float *)val, mat, s_tb[j], s_tb[j + 1], r0, nr,
                                               n_states, vmul, I.nnz, (float *)s_prod);
                    // the previous tile's store goes out after this tile's
                    // gathers; a wave that issued it then waits for all but it
                    const bool mine = pend_y != nullptr && 64 * wave < pend_nr;
                    acc = finish_tile_l<IT, NT, U, R>(tl, rx, (float *)s_prod, [&]() { flush(); }, mine);
                    q = tl.q;
                }
            } else if (fits(j)) {
                TileRegs<VT, IT, U> tr;
                issue_tile<VT, IT, NT, U, R>(tr, rp, col, val, mat, s_tb[j], s_tb[j + 1], r0, nr, n_states, vmul, I.nnz);
                acc = finish_tile<VT, IT, NT, U, R>(tr, rx, s_prod);
                q = tr.q;
            } else {
                // long rows: several passes over the tile
                const IT b = s_tb[j], e = s_tb[j + 1];
                IT mylo = 0, myhi = 0;
                if (own) {
                    mylo = rp[r];
                    myhi = rp[r + 1];
                    if (r < n_states) q = mat[vox_of(r, vmul)];
                }
                for (IT a = b & ~(IT)3; a < e; a += CAP) {
                    const IT cs = a < b ? b : a;
                    const IT ce = (e - a < (IT)CAP) ? e : a + (IT)CAP;
                    for (IT i = a + 4 * tid; i < ce; i += 4 * NT) {
                        const i4 c4 = __builtin_nontemporal_load((const GLB i4 *)(col + i));
                        Quad<VT> v4;
                        v4.load(val + i);
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const IT idx = i + jj;
                            if (idx >= cs && idx < ce) s_prod[idx - a] = v4[jj] * x[c4[jj]];
                        }
                    }
                    __syncthreads();
                    const IT lo = mylo > cs ? mylo : cs;
                    const IT hi = myhi < ce ? myhi : ce;
                    for (IT jj = lo; jj < hi; ++jj) acc += s_prod[jj - a];
                    __syncthreads();
                }
            }

            // epilogue: rescale, sources, store, FP64 totals
            constexpr bool kDefer = LAYV == 2 && sizeof(VT) == 4;
            if (kDefer) flush();   // a store still pending (a multi-pass tile did not issue it)
            if (own) {
                VT v = acc * scale;
                const int sb = s_src[j], se = s_src[j + 1];
                if (sb < se) {
                    const GLB int64_t *srow = gp(I.src_row);
                    int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && srow[e2] == r; ++e2) {
                        s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                        any = true;
                    }
                    if (any) v += (VT)ldexp(s, -sc.En);
                }
                if (kDefer) pend_v = v;
                else y[r] = v;
                s_y[tid] = v;
                if (r < n_states) {
                    sN += (double)v;
                    sA += s_abs[q] * (double)v;
                    mx = v > mx ? v : mx;
                } else {
                    sE += (double)v;
                }
            }
            if (kDefer) {
                pend_y = y;
                pend_r0 = r0;
                pend_nr = nr;
            }
            __syncthreads();
            const int db = s_det[j], de = s_det[j + 1];
            if (db < de && tid < I.n_det) {
                for (int e2 = db; e2 < de; ++e2)
                    if (gp(I.det_id)[e2] == tid) dsum += gp(I.det_F)[e2] * (double)s_y[gp(I.det_row)[e2] - r0];
            }
        }
        // chunk partials: wave butterflies, then the waves in order
        const int64_t nc = I.n_chunks, c = item.chunk;
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            s_wred[0][wave] = wN;
            s_wred[1][wave] = wE;
            s_wred[2][wave] = wA;
            s_wred[3][wave] = wM;
        }
        __syncthreads();
        GLB double *part = gpw(I.partials);
        if (tid < 4) {
            double a = s_wred[tid][0];
            for (int w = 1; w < NW; ++w) a = (tid == 3) ? fmax(a, s_wred[tid][w]) : a + s_wred[tid][w];
            part[(int64_t)tid * nc + c] = a;
        }
        if (tid < I.n_det) part[(int64_t)(kSlotDet + tid) * nc + c] = dsum;
    }
    flush();
}

// ---------------------------------------------------------------------------
// SpMV step for long rows (several hundred entries, as the multi-voxel
// weights of Lebedev media give): one wave per row while summing
//
// A workgroup takes a tile of R rows.  Each wave sums every fourth row of the
// tile: lane l multiplies entries lo + l, lo + l + 64, ... -- the row's
// columns and values are requested at once (up to 768 entries per pass, 12
// loads in flight per lane and array), then all the gathers -- and adds them
// in that order; a butterfly then adds the 64 lane sums in a fixed order.
// The tile's sums go to LDS and the epilogue (rescale, sources, y store, FP64
// totals and detectors, chunk partials) is the one of the tile kernels, a
// thread per row.  Results are reproducible run to run; they are not the
// tile kernels' sequential row sums bit for bit.
// ---------------------------------------------------------------------------
constexpr int kLongJ = 12;   // entries per lane requested at once (768 per wave)

template <typename VT, typename IT>
__global__ void __launch_bounds__(kNT) step_spmv_long(const StepInst *__restrict__ insts,
                                                       const WorkItem *__restrict__ work, int64_t n_work,
                                                       int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    constexpr int NT = kNT, NW = NT / 64;
    __shared__ double s_wred[4][NW];
    __shared__ IT s_tb[kChunkMax + 1];
    __shared__ int32_t s_src[kChunkMax + 1];
    __shared__ int32_t s_det[kChunkMax + 1];
    __shared__ double s_abs[kMatMax];
    __shared__ VT s_y[NT];
    __shared__ VT s_acc[NT];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    int cached = -1;
    int64_t t = 0;
    bool live = false;
    Scale sc{0, 0};
    VT scale = 1;
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        if (item.inst != cached) {
            cached = item.inst;
            t = I.t[0];
            live = t < *I.t_end;
            if (live) {
                sc = step_scale(I, 0, t);
                scale = (VT)ldexp(1.0, -sc.k);
            }
        }
        if (!live) continue;
        const int R = I.rows_per_tile;
        const GLB IT *rp = gp((const IT *)I.row_ptr);
        const GLB int32_t *col = gp(I.col);
        const GLB VT *val = gp((const VT *)I.val);
        const GLB VT *x = gp((const VT *)((t & 1) ? I.buf1 : I.buf0));
        GLB VT *y = gpw((VT *)((t & 1) ? I.buf0 : I.buf1));
        const GLB uint8_t *mat = gp(I.mat);
        const int64_t n_rows = I.n_rows, n_states = I.n_states;
        const uint64_t vmul = I.vox_mul;
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int ntc = (int)min((int64_t)I.tiles_per_chunk, I.n_tiles - tile0);
        for (int j = tid; j <= ntc; j += NT) {
            s_tb[j] = rp[min((tile0 + j) * R, n_rows)];
            s_src[j] = gp(I.src_tile)[tile0 + j];
            s_det[j] = gp(I.det_tile)[tile0 + j];
        }
        for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
        __syncthreads();
        double sN = 0.0, sE = 0.0, sA = 0.0, dsum = 0.0;
        VT mx = 0;
        for (int j = 0; j < ntc; ++j) {
            const int64_t r0 = (tile0 + j) * R;
            const int nr = (int)min((int64_t)R, n_rows - r0);
            // row sums, a wave per row: all of a row's columns and values are
            // requested at once (clamped into the row, so every load is in
            // bounds), then all its gathers, then the products in entry order
            for (int rr = wave; rr < nr; rr += NW) {
                const IT lo = rp[r0 + rr], hi = rp[r0 + rr + 1];
                VT a = 0;
                for (IT base = lo; base < hi; base += 64 * kLongJ) {
                    int32_t c[kLongJ];
                    VT v[kLongJ], xv[kLongJ];
#pragma unroll
                    for (int u = 0; u < kLongJ; ++u) {
                        const IT kk = base + lane + 64 * u;
                        const IT kc = kk < hi ? kk : hi - 1;
                        c[u] = __builtin_nontemporal_load(col + kc);
                        v[u] = __builtin_nontemporal_load(val + kc);
                    }
#pragma unroll
                    for (int u = 0; u < kLongJ; ++u) xv[u] = x[c[u]];
#pragma unroll
                    for (int u = 0; u < kLongJ; ++u)
                        if (base + lane + 64 * u < hi) a += v[u] * xv[u];
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
                if (lane == 0) s_acc[rr] = a;
            }
            __syncthreads();
            // epilogue: a thread per row
            const int64_t r = r0 + tid;
            const bool own = tid < nr;
            if (own) {
                VT v = s_acc[tid] * scale;
                const int sb = s_src[j], se = s_src[j + 1];
                if (sb < se) {
                    const GLB int64_t *srow = gp(I.src_row);
                    int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && srow[e2] == r; ++e2) {
                        s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                        any = true;
                    }
                    if (any) v += (VT)ldexp(s, -sc.En);
                }
                y[r] = v;
                s_y[tid] = v;
                if (r < n_states) {
                    sN += (double)v;
                    sA += s_abs[mat[vox_of(r, vmul)]] * (double)v;
                    mx = v > mx ? v : mx;
                } else {
                    sE += (double)v;
                }
            }
            __syncthreads();
            const int db = s_det[j], de = s_det[j + 1];
            if (db < de && tid < I.n_det) {
                for (int e2 = db; e2 < de; ++e2)
                    if (gp(I.det_id)[e2] == tid) dsum += gp(I.det_F)[e2] * (double)s_y[gp(I.det_row)[e2] - r0];
            }
        }
        // chunk partials: wave butterflies, then the waves in order
        const int64_t nc = I.n_chunks, c = item.chunk;
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            s_wred[0][wave] = wN;
            s_wred[1][wave] = wE;
            s_wred[2][wave] = wA;
            s_wred[3][wave] = wM;
        }
        __syncthreads();
        GLB double *part = gpw(I.partials);
        if (tid < 4) {
            double a = s_wred[tid][0];
            for (int w = 1; w < NW; ++w) a = (tid == 3) ? fmax(a, s_wred[tid][w]) : a + s_wred[tid][w];
            part[(int64_t)tid * nc + c] = a;
        }
        if (tid < I.n_det) part[(int64_t)(kSlotDet + tid) * nc + c] = dsum;
        __syncthreads();   // s_tb, s_src, s_det and s_wred are rewritten by the next item
    }
}

// value of lane l (uniform l) of a 64-bit per-lane value
__device__ __forceinline__ int64_t lane_i64(int64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// SpMM step (n_rhs right-hand sides, FP32), lanes = right-hand sides
//
// X is [rows][n_rhs]: one column index gives n_rhs contiguous values, so the
// gather of one entry is a single coalesced load of the whole wave.  A wave
// takes every fourth row of its chunk.  The row pointers of 64 of its rows
// come with one load (lane l holds row l's bounds); per row, lanes 0..n-1 load
// the row's columns and values with one coalesced load each, every lane reads
// entry k's column and value back by readlane, and all gathers of the row are
// issued before the first product.  The next row's columns and values are
// requested before the current row's gathers, so both round trips overlap.
// Products are added in column order, one rounding each, as the single-rhs
// step adds them: every column of the result equals that step's bit for bit.
// ---------------------------------------------------------------------------
constexpr int kSpmmUnroll = 26;   // entries of a plain row, gathered fully unrolled

// A chunk's per-wave sums (lane = rhs) combined in a fixed wave order and
// written as the chunk's partials; the workgroup's waves all call it.
__device__ __forceinline__ void spmm_chunk_partials(const StepInst &I, int64_t c, int wave, int lane, double sN,
                                                    double sE, double sA, float mx, double (*s_w)[4][64],
                                                    const double *s_det)
{
    const int nrhs = I.n_rhs, nd = I.n_det;
    s_w[0][wave][lane] = sN;
    s_w[1][wave][lane] = sE;
    s_w[2][wave][lane] = sA;
    s_w[3][wave][lane] = (double)mx;
    __syncthreads();
    const int64_t nc = I.n_chunks;
    if (wave == 0 && lane < nrhs) {
        const double N = ((s_w[0][0][lane] + s_w[0][1][lane]) + s_w[0][2][lane]) + s_w[0][3][lane];
        const double Es = ((s_w[1][0][lane] + s_w[1][1][lane]) + s_w[1][2][lane]) + s_w[1][3][lane];
        const double A = ((s_w[2][0][lane] + s_w[2][1][lane]) + s_w[2][2][lane]) + s_w[2][3][lane];
        const double M = fmax(fmax(s_w[3][0][lane], s_w[3][1][lane]), fmax(s_w[3][2][lane], s_w[3][3][lane]));
        I.partials[((int64_t)kSlotN * nrhs + lane) * nc + c] = N;
        I.partials[((int64_t)kSlotEsc * nrhs + lane) * nc + c] = Es;
        I.partials[((int64_t)kSlotAbs * nrhs + lane) * nc + c] = A;
        I.partials[((int64_t)kSlotMax * nrhs + lane) * nc + c] = M;
        for (int d = 0; d < nd; ++d) {
            const double D = ((s_det[(0 * nd + d) * 64 + lane] + s_det[(1 * nd + d) * 64 + lane]) +
                              s_det[(2 * nd + d) * 64 + lane]) +
                             s_det[(3 * nd + d) * 64 + lane];
            I.partials[((int64_t)(kSlotDet + d) * nrhs + lane) * nc + c] = D;
        }
    }
    __syncthreads();
}

template <typename IT>
__global__ void __launch_bounds__(kNT) step_spmm(const StepInst *__restrict__ insts,
                                                  const WorkItem *__restrict__ work, int64_t n_work,
                                                  int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    extern __shared__ double s_det[];   // [4 waves][n_det][64]
    __shared__ double s_w[4][4][64];     // per-wave totals for the fixed-order combine
    __shared__ double s_abs[kMatMax];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);

    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        const int64_t t = I.t[0];
        if (t >= *I.t_end) continue;
        const int nrhs = I.n_rhs, nd = I.n_det;
        const bool active = lane < nrhs;
        const int xl = min(lane, nrhs - 1);   // lanes past n_rhs gather a valid element, then drop it
        Scale sc{0, 0};
        if (active) sc = step_scale(I, lane, t);
        const float scale = ldexpf(1.0f, -sc.k);
        const GLB IT *rp = gp((const IT *)I.row_ptr);
        const GLB int32_t *col = gp(I.col);
        const GLB float *val = gp((const float *)I.val);
        const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
        GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
        const GLB uint8_t *mat = gp(I.mat);
        double *my_det = s_det + (int64_t)wave * nd * 64;
        for (int d = 0; d < nd; ++d) my_det[d * 64 + lane] = 0.0;
        for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
        __syncthreads();

        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        const int R = I.rows_per_tile;
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int64_t tile1 = min(tile0 + (int64_t)I.tiles_per_chunk, I.n_tiles);
        const int64_t row_b = tile0 * R, row_e = min(tile1 * R, I.n_rows);
        // sources and detectors are rare: look them up only in chunks that have them
        const bool any_src = gp(I.src_tile)[tile1] > gp(I.src_tile)[tile0];
        const bool any_det = nd > 0 && gp(I.det_tile)[tile1] > gp(I.det_tile)[tile0];

        for (int64_t rb = row_b + wave; rb < row_e; rb += 4 * 64) {
            // bounds of this wave's next 64 rows rb, rb + 4, ...
            const int nb = (int)min((int64_t)64, (row_e - rb + 3) / 4);
            const int64_t my_r = rb + 4 * (int64_t)min(lane, nb - 1);
            const int64_t v_lo = (int64_t)rp[my_r], v_hi = (int64_t)rp[my_r + 1];
            // columns and values of row 0 (lanes 0 .. n-1)
            int64_t lo = lane_i64(v_lo, 0), hi = lane_i64(v_hi, 0);
            const int64_t j0 = lo + min((int64_t)lane, max(hi - lo - 1, (int64_t)0));
            int32_t c_cur = col[j0];
            float v_cur = val[j0];
            for (int i = 0; i < nb; ++i) {
                const int64_t r = rb + 4 * (int64_t)i;
                const int n = (int)(hi - lo);
                // the next row's entries are requested right after this row's
                // gathers: loads return in order, so the gathers are waited
                // for without waiting for them, and they arrive meanwhile
                int64_t lo_n = 0, hi_n = 0;
                int32_t c_nxt = 0;
                float v_nxt = 0.0f;
                auto prefetch = [&]() {
                    // unconditional, at an index clamped into the row (an empty
                    // row reads the padding after the last entry): the wait
                    // counts stay exact; lanes past the row's length are unused
                    const int inx = min(i + 1, nb - 1);
                    lo_n = lane_i64(v_lo, inx);
                    hi_n = lane_i64(v_hi, inx);
                    const int64_t j = lo_n + min((int64_t)lane, max(hi_n - lo_n - 1, (int64_t)0));
                    c_nxt = col[j];
                    v_nxt = val[j];
                };
                float acc = 0.0f;
                if (n == kSpmmUnroll) {
                    float xv[kSpmmUnroll];
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k) {
                        const int ck = __builtin_amdgcn_readlane(c_cur, k);
                        xv[k] = X[(int64_t)ck * nrhs + xl];
                    }
                    prefetch();
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k)
                        acc += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v_cur), k)) * xv[k];
                } else {
                    prefetch();
                    // any length, in windows of 64 entries
                    for (int64_t wb = lo; wb < hi; wb += 64) {
                        int32_t cw = c_cur;
                        float vw = v_cur;
                        if (wb != lo) {
                            cw = 0;
                            vw = 0.0f;
                            if (wb + lane < hi) {
                                cw = col[wb + lane];
                                vw = val[wb + lane];
                            }
                        }
                        const int m = (int)min((int64_t)64, hi - wb);
                        int k = 0;
                        for (; k + 8 <= m; k += 8) {
                            float xv[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const int ck = __builtin_amdgcn_readlane(cw, k + u);
                                xv[u] = X[(int64_t)ck * nrhs + xl];
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                acc += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vw), k + u)) * xv[u];
                        }
                        for (; k < m; ++k) {
                            const int ck = __builtin_amdgcn_readlane(cw, k);
                            const float xk = X[(int64_t)ck * nrhs + xl];
                            acc += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vw), k)) * xk;
                        }
                    }
                }
                float v = acc * scale;
                if (any_src) {
                    const int64_t tile = r / R;
                    const int sb = gp(I.src_tile)[tile], se = gp(I.src_tile)[tile + 1];
                    if (sb < se) {
                        int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                        double s = 0.0;
                        bool any = false;
                        for (; e2 < se && I.src_row[e2] == r; ++e2) {
                            if (I.src_rhs[e2] == lane) {
                                s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                                any = true;
                            }
                        }
                        if (any) v += (float)ldexp(s, -sc.En);
                    }
                }
                if (active) {
                    Y[r * nrhs + lane] = v;
                    if (r < I.n_states) {
                        sN += (double)v;
                        sA += s_abs[mat[vox_of(r, I.vox_mul)]] * (double)v;
                        mx = fmaxf(mx, v);
                    } else {
                        sE += (double)v;
                    }
                    if (any_det) {
                        const int64_t tile = r / R;
                        const int db = gp(I.det_tile)[tile], de = gp(I.det_tile)[tile + 1];
                        if (db < de) {
                            int e2 = lower_bound_rows<IT>(I.det_row, db, de, r);
                            for (; e2 < de && I.det_row[e2] == r; ++e2)
                                my_det[I.det_id[e2] * 64 + lane] += I.det_F[e2] * (double)v;
                        }
                    }
                }
                lo = lo_n;
                hi = hi_n;
                c_cur = c_nxt;
                v_cur = v_nxt;
            }
        }
        spmm_chunk_partials(I, item.chunk, wave, lane, sN, sE, sA, mx, s_w, s_det);
    }
}

// A group descriptor read field by field (a struct copy from the global or
// constant address space has no constructor)
template <typename P> __device__ __forceinline__ GroupDesc load_desc(P p)
{
    GroupDesc D;
    D.voff = p->voff;
    D.coff = p->coff;
    D.m0 = p->m0;
    D.nm = p->nm;
    D.n = p->n;
    D.cstart = p->cstart;
    return D;
}

// ---------------------------------------------------------------------------
// SpMM step by row groups (n_rhs right-hand sides, FP32, one solver), lanes = rhs
//
// Rows whose column lists are equal form a group: in a lattice matrix, the
// rows that pull from one source voxel (one per direction, state or escape
// row) all hold that voxel's whole state.  The matrix keeps, beside its CSR,
// the values in group order and each member's row and material, so every
// array the step reads of a group is contiguous, and one descriptor per
// group (read through the scalar cache).  A wave takes a group at a time:
// lane j fetches member j's row and material; the X rows of the group's
// columns are gathered once into registers (one coalesced 4*n_rhs-byte row
// per column; a group whose columns are one run needs no column load at
// all); lane m of load k holds member m's entry k, and member m's row is
// formed from those registers by readlane.  Each X row is then fetched about
// once per step instead of once per entry.  A member is formed with the same
// products in the same column order as in the row-by-row kernel and the
// single-rhs step, so every column of the result equals theirs bit for bit.
// With F64S each member's row is instead summed in FP64 (one fma per term, in
// column order: the products of two FP32 numbers are exact in FP64) and
// rounded once to FP32, which keeps the FP32 accumulation error from building
// up over long runs.
// With VI (taken with F64S) the fast groups' values come from their
// value-indexed slots (lane j reads member j's 32-byte slot and takes its 26
// values from the dictionary in LDS: the same FP32 values, from a quarter of
// the bytes).
// Groups whose rows are not kSpmmUnroll long are formed row by row (windows
// of 64 entries).  Sources are looked up only in groups the solver flagged.
//
// Work item c takes groups c * n_groups / n_work onwards, a quarter of them
// (contiguous) to each wave; a wave's totals over its quarter are the
// partials of index 4c + wave, so the sums do not depend on which workgroup
// takes which item.  The detector sums are left to spmm_detectors, which
// reads the stored rows.
// ---------------------------------------------------------------------------
template <typename IT, bool F64S, bool VI>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(F64S ? 4 : 5, 8))) step_spmm_grouped(const StepInst *__restrict__ insts,
                                                          const WorkItem *__restrict__ work, int64_t n_work,
                                                          int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    extern __shared__ float s_dict[];   // VI: [vi_ntab][kViDict]
    __shared__ double s_abs[kMatMax];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const int nrhs = I.n_rhs;
    const bool active = lane < nrhs;
    const int xl = min(lane, nrhs - 1);   // lanes past n_rhs gather a valid element, then drop it
    Scale sc{0, 0};
    if (active) sc = step_scale(I, lane, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB int32_t *col = gp(I.col);
    const GLB float *val = gp(I.grp_val);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB uint8_t *gmat = gp(I.grp_mat);
    const GLB int32_t *grow = gp(I.grp_row);
    const GLB int32_t *src_tile = gp(I.src_tile);
    const CST GroupDesc *grp = cst(I.grp);
    const CST uint32_t *gsrc = cst(I.grp_src);
    const CST int32_t *gfo = cst(I.vi_fast_of);
    const GLB uint8_t *vidx = gp(I.vi_idx);
    for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
    if constexpr (VI)
        for (int q = threadIdx.x; q < I.vi_ntab * kViDict; q += kNT) s_dict[q] = gp(I.vi_dict)[q];
    __syncthreads();

    const int R = I.rows_per_tile;
    const int64_t G = I.n_groups, nc = I.n_chunks;
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const int64_t c = work[wi].chunk;
        const int64_t c_b = c * G / n_work, c_e = (c + 1) * G / n_work;
        const int64_t g_b = c_b + wave * (c_e - c_b) / 4, g_e = c_b + (wave + 1) * (c_e - c_b) / 4;
        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        for (int64_t g = g_b; g < g_e; ++g) {
            const GroupDesc D = load_desc(grp + g);
            const bool g_src = (gsrc[g >> 5] >> (g & 31)) & 1u;
            const int m0 = D.m0, nm = D.nm, n = D.n;
            // lane j (< nm): member j
            const int jl = min(lane, nm - 1);
            const int32_t my_r = grow[m0 + jl];
            const int my_mat = gmat[m0 + jl];
            int my_tile = 0;
            uint64_t src_mask = 0;

            // member m's result: rescale, sources, store, totals
            auto emit = [&](int m, float acc) {
                const int64_t r = __builtin_amdgcn_readlane(my_r, m);
                float v = acc * scale;
                if ((src_mask >> m) & 1) {
                    const int tile = __builtin_amdgcn_readlane(my_tile, m);
                    const int sb = src_tile[tile], se = src_tile[tile + 1];
                    int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && I.src_row[e2] == r; ++e2) {
                        if (I.src_rhs[e2] == lane) {
                            s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                            any = true;
                        }
                    }
                    if (any) v += (float)ldexp(s, -sc.En);
                }
                if (active) {
                    Y[r * nrhs + lane] = v;
                    if (r < I.n_states) {
                        sN += (double)v;
                        sA += s_abs[__builtin_amdgcn_readlane(my_mat, m)] * (double)v;
                        mx = fmaxf(mx, v);
                    } else {
                        sE += (double)v;
                    }
                }
            };
            auto flag_sources = [&]() {
                if (g_src) {
                    my_tile = my_r / R;
                    src_mask = __builtin_amdgcn_ballot_w64(src_tile[my_tile + 1] > src_tile[my_tile]);
                }
            };

            if (n == kSpmmUnroll) {
                float xv[kSpmmUnroll];
                if (D.cstart >= 0) {
                    // one run of columns: a buffer at its first X row, the
                    // rows at scalar offsets
                    const __amdgpu_buffer_rsrc_t rx =
                        make_rsrc((const void *)(X + (int64_t)D.cstart * nrhs), (uint64_t)kSpmmUnroll * nrhs * 4);
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k)
                        xv[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, xl * 4, k * nrhs * 4, 0));
                } else {
                    const int32_t cl = col[D.coff + min(lane, kSpmmUnroll - 1)];
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k)
                        xv[k] = X[(int64_t)__builtin_amdgcn_readlane(cl, k) * nrhs + xl];
                }
                // vk[k]: lane m holds member m's entry k (a buffer at the
                // group's values, entry k at a scalar offset; or, value-
                // indexed, member m's slot and the dictionary)
                float vk[kSpmmUnroll];
                bool indexed = false;
                if constexpr (VI) {
                    const int32_t f = gfo[g];
                    if (f >= 0) {
                        const GLB u32x4 *slot = (const GLB u32x4 *)(vidx + (int64_t)f * kViBlock + (int64_t)jl * kViSlot);
                        const u32x4 s0 = __builtin_nontemporal_load(slot), s1 = __builtin_nontemporal_load(slot + 1);
                        const uint32_t wd[8] = {s0[0], s0[1], s0[2], s0[3], s1[0], s1[1], s1[2], s1[3]};
                        const float *tab =
                            s_dict + ((wd[kViTabByte >> 2] >> (8 * (kViTabByte & 3))) & 0xff) * kViDict;
#pragma unroll
                        for (int k = 0; k < kSpmmUnroll; ++k) vk[k] = tab[(wd[k >> 2] >> (8 * (k & 3))) & 0xff];
                        indexed = true;
                    }
                }
                if (!indexed) {
                    const __amdgpu_buffer_rsrc_t rv =
                        make_rsrc((const void *)(val + D.voff), (uint64_t)kSpmmUnroll * nm * 4);
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k)
                        vk[k] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(rv, jl * 4, k * nm * 4, kStream));
                }
                flag_sources();
                if constexpr (F64S) {
                    double xd[kSpmmUnroll];
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k) xd[k] = (double)xv[k];
#pragma unroll
                    for (int m = 0; m < kGroupMax; ++m) {
                        if (m < nm) {
                            double acc = 0.0;
#pragma unroll
                            for (int k = 0; k < kSpmmUnroll; ++k)
                                acc = __builtin_fma(
                                    (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(vk[k]), m)), xd[k],
                                    acc);
                            emit(m, (float)acc);
                        }
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < kGroupMax; ++m) {
                        if (m < nm) {
                            float acc = 0.0f;
#pragma unroll
                            for (int k = 0; k < kSpmmUnroll; ++k)
                                acc += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vk[k]), m)) * xv[k];
                            emit(m, acc);
                        }
                    }
                }
            } else {
                flag_sources();
                for (int m = 0; m < nm; ++m) {
                    std::conditional_t<F64S, double, float> acc = 0;
                    for (int wb = 0; wb < n; wb += 64) {
                        int32_t cw = 0;
                        float vw = 0.0f;
                        if (wb + lane < n) {
                            cw = col[D.coff + wb + lane];
                            vw = val[D.voff + (int64_t)(wb + lane) * nm + m];
                        }
                        const int w = min(64, n - wb);
                        int k = 0;
                        for (; k + 8 <= w; k += 8) {
                            float xw[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                xw[u] = X[(int64_t)__builtin_amdgcn_readlane(cw, k + u) * nrhs + xl];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                const float vu = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vw), k + u));
                                if constexpr (F64S) acc = __builtin_fma((double)vu, (double)xw[u], acc);
                                else acc += vu * xw[u];
                            }
                        }
                        for (; k < w; ++k) {
                            const float xk = X[(int64_t)__builtin_amdgcn_readlane(cw, k) * nrhs + xl];
                            const float vu = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vw), k));
                            if constexpr (F64S) acc = __builtin_fma((double)vu, (double)xk, acc);
                            else acc += vu * xk;
                        }
                    }
                    emit(m, (float)acc);
                }
            }
        }
        if (active) {
            const int64_t b = 4 * c + wave;
            I.partials[((int64_t)kSlotN * nrhs + lane) * nc + b] = sN;
            I.partials[((int64_t)kSlotEsc * nrhs + lane) * nc + b] = sE;
            I.partials[((int64_t)kSlotAbs * nrhs + lane) * nc + b] = sA;
            I.partials[((int64_t)kSlotMax * nrhs + lane) * nc + b] = (double)mx;
        }
    }
}

// Detector sums of the step by row groups (Eq. (27)): block (p, d) forms the
// sum F * y over part p of detector d's entries (kDetParts equal parts of its
// row-ordered list) from the stored rows of y -- lanes = rhs, the four waves
// take every fourth entry, then combine in a fixed order -- and writes it to
// the direct sums, which the finalize adds in part order.
__global__ void __launch_bounds__(kNT) spmm_detectors(const StepInst *__restrict__ insts)
{
    __shared__ double s_d[4][64];
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const int p = blockIdx.x, d = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nrhs = I.n_rhs;
    const int xl = min(lane, nrhs - 1);
    const GLB float *Y = gp((const float *)((t & 1) ? I.buf0 : I.buf1));
    const int64_t b = I.ddet_ptr[d], n = I.ddet_ptr[d + 1] - b;
    const int64_t pb = b + p * n / kDetParts, pe = b + (p + 1) * n / kDetParts;
    double acc = 0.0;
#pragma unroll 4
    for (int64_t k = pb + wave; k < pe; k += 4) acc += I.ddet_F[k] * (double)Y[I.ddet_row[k] * nrhs + xl];
    s_d[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && lane < nrhs)
        det_direct_sums(I.partials, I.n_det, nrhs, I.n_chunks)[((int64_t)d * kDetParts + p) * nrhs + lane] =
            ((s_d[0][lane] + s_d[1][lane]) + s_d[2][lane]) + s_d[3][lane];
}

// ---------------------------------------------------------------------------
// SpMV step by row groups (one rhs, FP32, one solver)
//
// The row groups and the group-order arrays of the many-rhs step.  The fast
// groups -- full lattice rows, kSpmmUnroll columns in one run, nearly every
// group -- go to step_spmv_grouped_vi when their values are value-indexed,
// else to step_spmv_grouped, whose lanes are the members: each half-wave
// takes a group (lane m of the half is member m), so a wave forms a pair of
// groups per half-wave pass; it issues the loads of kGroupPairs pairs before
// it forms the first (more bytes in flight per wave), and the descriptors of
// its next pairs load while the current ones are formed.  Lane m loads x at
// column m of the run into LDS, then its own entries with one load per k (the
// group's values are column-major, so a group's k-th entries are one
// contiguous run) and adds entry * x over k in column order: the CSR step's
// products in its order, so y equals its y bit for bit.  The matrix stream
// is the values alone (no columns) and x is read once per group.  Two-voxel
// rows (interface rows whose entries come from two voxels) go to
// step_spmv_vox2, every other row to step_spmv_rowlist, a thread per row.
// Work items of the fast groups are split among the waves as in the many-rhs
// step (partials of index 4c + wave), those of the row list and of the
// two-voxel rows follow; the detector sums are left to spmv_detectors.
// ---------------------------------------------------------------------------
constexpr int kGroupPairs = 2;   // pairs of groups a wave forms per iteration

template <int NP>
__global__ void __launch_bounds__(kNT) step_spmv_grouped(const StepInst *__restrict__ insts,
                                                          const WorkItem *__restrict__ work, int64_t n_work,
                                                          int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    constexpr int NG = 2 * NP;        // groups a wave forms at once: NP pairs, a half-wave each
    __shared__ float s_x[4][NG][32];  // per wave and group: x at the group's columns
    __shared__ double s_abs[kMatMax];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, m = lane & 31;
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const Scale sc = step_scale(I, 0, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB float *val = gp(I.grp_val);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB uint8_t *gmat = gp(I.grp_mat);
    const GLB int32_t *grow = gp(I.grp_row);
    const GLB int32_t *src_tile = gp(I.src_tile);
    const CST GroupDesc *grp = cst(I.grp);
    const CST int32_t *gfast = cst(I.grp_fast);
    const CST uint32_t *gsrc = cst(I.grp_src);
    const int64_t nv = I.nnz + 4;   // entries of the group-order values (with the padding)
    for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
    __syncthreads();

    const int R = I.rows_per_tile;
    const int64_t G = I.n_fast;
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const int64_t c = work[wi].chunk;
        const int64_t c_b = c * G / n_work, c_e = (c + 1) * G / n_work;
        const int64_t g_b = c_b + wave * (c_e - c_b) / 4, g_e = c_b + (wave + 1) * (c_e - c_b) / 4;
        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        if (g_b < g_e) {
            // the wave's NG groups (past the end of its range: its last group
            // again, formed but not stored), descriptors and source bits
            // through the scalar cache; the next NG's load while these form
            int64_t id[NG];
            GroupDesc D[NG];
            uint32_t w[NG];
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                id[q] = gfast[min(g_b + q, g_e - 1)];
                D[q] = load_desc(grp + id[q]);
                w[q] = gsrc[id[q] >> 5];
            }
            for (int64_t g2 = g_b; g2 < g_e; g2 += NG) {
                int64_t ci[NG];
                GroupDesc C[NG];
                uint32_t cw[NG];
#pragma unroll
                for (int q = 0; q < NG; ++q) {
                    ci[q] = id[q];
                    C[q] = D[q];
                    cw[q] = w[q];
                }
                if (g2 + NG < g_e) {
#pragma unroll
                    for (int q = 0; q < NG; ++q) {
                        id[q] = gfast[min(g2 + NG + q, g_e - 1)];
                        D[q] = load_desc(grp + id[q]);
                        w[q] = gsrc[id[q] >> 5];
                    }
                }
                // every pair's loads first (x at the run, members' rows and
                // materials, NP x 26 values), then the sums in pair order
                float vk[NP][kSpmmUnroll];
                float xm[NP];
                int32_t r[NP];
                int mt[NP], nmv[NP];
                bool gsb[NP];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    const GroupDesc &A0 = C[2 * p], &A1 = C[2 * p + 1];
                    const int nm = h ? A1.nm : A0.nm;
                    const int m0 = h ? A1.m0 : A0.m0, cstart = h ? A1.cstart : A0.cstart;
                    const int64_t voff = h ? A1.voff : A0.voff;
                    gsb[p] = h ? ((cw[2 * p + 1] >> (ci[2 * p + 1] & 31)) & 1u) : ((cw[2 * p] >> (ci[2 * p] & 31)) & 1u);
                    nmv[p] = nm;
                    const int jm = min(m, nm - 1);
                    r[p] = grow[m0 + jm];
                    mt[p] = gmat[m0 + jm];
                    xm[p] = X[cstart + min(m, kSpmmUnroll - 1)];
                    // a buffer at the lower of the pair's value offsets; each
                    // lane's entries at 32-bit offsets from it (the pair's
                    // groups are neighbours in the fast list, a few thousand
                    // entries apart)
                    const int64_t vb = min(A0.voff, A1.voff);
                    const __amdgpu_buffer_rsrc_t rv = make_rsrc((const void *)(val + vb), (uint64_t)(nv - vb) * 4);
                    const uint32_t o0 = (uint32_t)(voff - vb + jm) * 4, st = (uint32_t)nm * 4;
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k)
                        vk[p][k] = __builtin_bit_cast(
                            float, __builtin_amdgcn_raw_buffer_load_b32(rv, (int)(o0 + k * st), 0, kStream));
                }
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    float *sx = s_x[wave][2 * p + h];
                    sx[m] = xm[p];
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < kSpmmUnroll; ++k) acc += vk[p][k] * sx[k];
                    if (g2 + 2 * p + h < g_e && m < nmv[p]) {
                        const int32_t rr = r[p];
                        float v = acc * scale;
                        if (gsb[p]) {
                            const int tile = rr / R;
                            const int sb = src_tile[tile], se = src_tile[tile + 1];
                            if (sb < se) {
                                int e2 = lower_bound_rows<int32_t>(I.src_row, sb, se, rr);
                                double s = 0.0;
                                bool any = false;
                                for (; e2 < se && I.src_row[e2] == rr; ++e2) {
                                    s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                                    any = true;
                                }
                                if (any) v += (float)ldexp(s, -sc.En);
                            }
                        }
                        Y[rr] = v;
                        if (rr < I.n_states) {
                            sN += (double)v;
                            sA += s_abs[mt[p]] * (double)v;
                            mx = fmaxf(mx, v);
                        } else {
                            sE += (double)v;
                        }
                    }
                }
            }
        }
        // the wave's totals over its groups, in a fixed butterfly
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            const int64_t nc = I.n_chunks, b = 4 * c + wave;
            I.partials[(int64_t)kSlotN * nc + b] = wN;
            I.partials[(int64_t)kSlotEsc * nc + b] = wE;
            I.partials[(int64_t)kSlotAbs * nc + b] = wA;
            I.partials[(int64_t)kSlotMax * nc + b] = wM;
        }
    }
}

// The fast groups with value-indexed values, by bricks.  Lane m reads its
// member's slot (kViSlot bytes: its entries as one-byte indices, the
// dictionary's number, the group's position in its brick, its row) with two
// 16-byte loads and takes each value from the dictionary in LDS -- the same FP32
// values, so the same products, order and y bit for bit, from a quarter of
// the bytes.  A work item is a range of bricks; the workgroup forms one brick
// at a time (its groups split among the waves, two pairs of groups issued per
// pass) and stages every state row (u + e_m, m) of its groups -- all inside
// the brick's window of kWin^3 voxels -- in LDS, with a presence bit; after a
// barrier it writes the window out in address order (consecutive lanes,
// consecutive rows: few lines per store), then the next brick.  Escape rows
// and rows whose index is not (u + e_m, m) are stored directly.  SRC: some
// fast group holds a source row (else the source code is left out).
constexpr int kGroupPairsVi = 2;   // pairs of groups a wave forms per pass

template <int NP, bool SRC>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(5, 8))) step_spmv_grouped_vi(const StepInst *__restrict__ insts,
                                                             const WorkItem *__restrict__ work, int64_t n_work,
                                                             int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    constexpr int NG = 2 * NP;
    constexpr int kHasWords = (kWinSlots + 31) / 32;
    extern __shared__ float s_tab[];            // [vi_ntab][kViDict]
    __shared__ float s_win[kWinSlots];          // the brick's staged rows
    __shared__ uint32_t s_has[2][kHasWords];    // presence bits, by brick parity
    __shared__ float s_x[4][NG][32];
    __shared__ double s_abs[kViTabs];           // value indexing: at most kViTabs materials
    // index tables: per direction d its voxel offset in the grid and in the
    // window; per position in the brick its voxel in the window; per window
    // voxel its offset in the grid from the window's first voxel
    __shared__ int32_t s_goff[26], s_doff[26], s_pb[kBrick * kBrick * kBrick], s_woff[kWin * kWin * kWin];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, m = lane & 31;
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const Scale sc = step_scale(I, 0, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB uint8_t *gmat = gp(I.grp_mat);
    const GLB uint8_t *vidx = gp(I.vi_idx);
    const GLB int32_t *src_tile = gp(I.src_tile);
    const GLB i4 *fd4 = (const GLB i4 *)gp(I.vi_fdesc);
    const GLB uint32_t *srcf = gp(I.grp_src_f);
    const CST int32_t *bptr = cst(I.brick_ptr);
    const CST int32_t *borg = cst(I.brick_org);
    const int32_t nx = I.grid_nx, ny = I.grid_ny;
    const int64_t plane = (int64_t)nx * ny;
    for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
    for (int q = threadIdx.x; q < I.vi_ntab * kViDict; q += kNT) s_tab[q] = gp(I.vi_dict)[q];
    for (int q = threadIdx.x; q < 2 * kHasWords; q += kNT) (&s_has[0][0])[q] = 0u;
    // (the bricks' guard keeps a plane, and so every offset here, within int32)
    for (int q = threadIdx.x; q < 26; q += kNT) {
        const int kk = q + (q >= 13 ? 1 : 0);
        const int ex = kk % 3 - 1, ey = (kk / 3) % 3 - 1, ez = kk / 9 - 1;
        s_goff[q] = ex + ey * nx + ez * (int32_t)plane;
        s_doff[q] = (ez * kWin + ey) * kWin + ex;
    }
    for (int q = threadIdx.x; q < kBrick * kBrick * kBrick; q += kNT)
        s_pb[q] = ((q / (kBrick * kBrick) + 1) * kWin + (q / kBrick) % kBrick + 1) * kWin + q % kBrick + 1;
    for (int q = threadIdx.x; q < kWin * kWin * kWin; q += kNT)
        s_woff[q] = q % kWin + ((q / kWin) % kWin) * nx + (q / (kWin * kWin)) * (int32_t)plane;
    // this thread's first window slot s = threadIdx.x as (window voxel, direction)
    const int vw0 = threadIdx.x / 26, dd0 = threadIdx.x - 26 * (threadIdx.x / 26);
    __syncthreads();

    const int R = I.rows_per_tile;
    const int64_t NB = I.n_brick;
    int parity = 0;
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const int64_t c = work[wi].chunk;
        const int64_t b_b = c * NB / n_work, b_e = (c + 1) * NB / n_work;
        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        for (int64_t bk = b_b; bk < b_e; ++bk) {
            uint32_t *has = s_has[parity];
            const int64_t f0 = bptr[bk], f1 = bptr[bk + 1];
            const int64_t per = (f1 - f0 + 3) / 4;
            const int64_t g_b = f0 + wave * per, g_e = min(g_b + per, f1);
            // the window's first voxel: the brick's origin - (1, 1, 1)
            const int64_t w0 = (int64_t)borg[bk] - 1 - nx - plane;
            if (g_b < g_e) {
                // per pass, the NG groups' {first member, member count, first
                // column, group} (lane q holds group q mod NG) and the
                // source-bit words of fast indices g2 (even lanes) and
                // g2 + NG - 1 (odd lanes), by vector loads issued a pass
                // ahead: no scalar loads in the loop, whose waits would also
                // hold the LDS reads
                i4 nd = fd4[min(g_b + (lane % NG), g_e - 1)];
                uint32_t nsw = srcf[(g_b + ((lane & 1) ? NG - 1 : 0)) >> 5];
                for (int64_t g2 = g_b; g2 < g_e; g2 += NG) {
                    const i4 cd = nd;
                    const uint32_t csw = nsw;
                    // (unconditional: past the range it reloads the last
                    // group, so the loads need no branch and the waits count
                    // exactly)
                    nd = fd4[min(g2 + NG + (lane % NG), g_e - 1)];
                    nsw = srcf[min(g2 + NG + ((lane & 1) ? NG - 1 : 0), g_e - 1) >> 5];
                    const uint32_t sw0 = (uint32_t)__builtin_amdgcn_readlane((int)csw, 0);
                    const uint32_t sw1 = (uint32_t)__builtin_amdgcn_readlane((int)csw, 1);
                    // every pair's loads first, then the sums in pair order
                    u32x4 sl[NP][2];
                    float xm[NP];
                    int32_t r[NP];
                    int mt[NP], nmv[NP], cs[NP];
                    bool gsb[NP];
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const int m0 = h ? __builtin_amdgcn_readlane(cd[0], 2 * p + 1)
                                         : __builtin_amdgcn_readlane(cd[0], 2 * p);
                        const int nm = h ? __builtin_amdgcn_readlane(cd[1], 2 * p + 1)
                                         : __builtin_amdgcn_readlane(cd[1], 2 * p);
                        const int cstart = h ? __builtin_amdgcn_readlane(cd[2], 2 * p + 1)
                                             : __builtin_amdgcn_readlane(cd[2], 2 * p);
                        const int64_t fi = g2 + 2 * p + h;
                        const uint32_t swd = ((fi >> 5) == (g2 >> 5)) ? sw0 : sw1;
                        gsb[p] = (swd >> (fi & 31)) & 1u;
                        nmv[p] = nm;
                        cs[p] = cstart;
                        const int jm = min(m, nm - 1);
                        mt[p] = gmat[m0 + jm];
                        xm[p] = X[cstart + min(m, kSpmmUnroll - 1)];
                        // this half's group is fast group g2 + 2p + h (the
                        // last one again past the wave's range)
                        const int64_t f = min(g2 + 2 * p + h, g_e - 1);
                        const GLB u32x4 *slot = (const GLB u32x4 *)(vidx + f * kViBlock + (int64_t)jm * kViSlot);
                        sl[p][0] = __builtin_nontemporal_load(slot);
                        sl[p][1] = __builtin_nontemporal_load(slot + 1);
                        r[p] = (int32_t)sl[p][1][kViRowWord - 4];   // the member's row, from its slot
                    }
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        float *sx = s_x[wave][2 * p + h];
                        sx[m] = xm[p];
                        const uint32_t wd[8] = {sl[p][0][0], sl[p][0][1], sl[p][0][2], sl[p][0][3],
                                                sl[p][1][0], sl[p][1][1], sl[p][1][2], sl[p][1][3]};
                        const float *tab = s_tab + ((wd[kViTabByte >> 2] >> (8 * (kViTabByte & 3))) & 0xff) * kViDict;
                        float acc = 0.0f;
#pragma unroll
                        for (int k = 0; k < kSpmmUnroll; ++k)
                            acc += tab[(wd[k >> 2] >> (8 * (k & 3))) & 0xff] * sx[k];
                        if (g2 + 2 * p + h < g_e && m < nmv[p]) {
                            const int32_t rr = r[p];
                            float v = acc * scale;
                            if (SRC && gsb[p]) {
                                const int tile = rr / R;
                                const int sb = src_tile[tile], se = src_tile[tile + 1];
                                if (sb < se) {
                                    int e2 = lower_bound_rows<int32_t>(I.src_row, sb, se, rr);
                                    double s = 0.0;
                                    bool any = false;
                                    for (; e2 < se && I.src_row[e2] == rr; ++e2) {
                                        s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                                        any = true;
                                    }
                                    if (any) v += (float)ldexp(s, -sc.En);
                                }
                            }
                            bool staged = false;
                            if (rr < I.n_states) {
                                sN += (double)v;
                                sA += s_abs[mt[p]] * (double)v;
                                mx = fmaxf(mx, v);
                                // the row (u + e_d, d) of source voxel u, d = rr mod 26:
                                // its slot in the brick's window (u at position pos of
                                // the brick, so the slot is in the window for any d)
                                const int32_t vd = rr / 26, d = rr - 26 * vd;
                                const int32_t u = cs[p] / 26;
                                if (vd == u + s_goff[d]) {
                                    const int pos = (wd[kViPosByte >> 2] >> (8 * (kViPosByte & 3))) &
                                                    (kBrick * kBrick * kBrick - 1);
                                    const int slot = (s_pb[pos] + s_doff[d]) * 26 + d;
                                    s_win[slot] = v;
                                    atomicOr(&has[slot >> 5], 1u << (slot & 31));
                                    staged = true;
                                }
                            } else {
                                sE += (double)v;
                            }
                            if (!staged) Y[rr] = v;
                        }
                    }
                }
            }
            __syncthreads();
            // the window in address order: slot s is row 26 v + d of window
            // voxel v (s = 26 v + d, stepped by kNT = 9 * 26 + 22 per pass);
            // clear the other parity's bits for the next brick
            uint32_t *nxt = s_has[parity ^ 1];
            for (int q = threadIdx.x; q < kHasWords; q += kNT) nxt[q] = 0u;
            GLB float *Yw = Y + w0 * 26;
            int vw = vw0, dd = dd0;
            for (int s = threadIdx.x; s < kWinSlots; s += kNT) {
                if ((has[s >> 5] >> (s & 31)) & 1u) Yw[s_woff[vw] * 26 + dd] = s_win[s];
                vw += kNT / 26;
                dd += kNT % 26;
                if (dd >= 26) {
                    dd -= 26;
                    ++vw;
                }
            }
            __syncthreads();
            parity ^= 1;
        }
        // the wave's totals over its groups, in a fixed butterfly
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            const int64_t nc = I.n_chunks, b = 4 * c + wave;
            I.partials[(int64_t)kSlotN * nc + b] = wN;
            I.partials[(int64_t)kSlotEsc * nc + b] = wE;
            I.partials[(int64_t)kSlotAbs * nc + b] = wA;
            I.partials[(int64_t)kSlotMax * nc + b] = wM;
        }
    }
}

// The rows of the groups step_spmv_grouped does not take, a thread per row:
// work item j (blockIdx.x, then every gridDim.x-th) is rows kRowListItem j
// onwards of the list; each row's entries are added in column order (the
// tiled step's order), eight requested at a time; its partials are those of
// index slow_part + 4j + wave.
constexpr int kRowListWin = 8;

template <typename IT>
__global__ void __launch_bounds__(kNT) step_spmv_rowlist(const StepInst *__restrict__ insts)
{
    __shared__ double s_abs[kMatMax];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const Scale sc = step_scale(I, 0, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB IT *rp = gp((const IT *)I.row_ptr);
    const GLB int32_t *col = gp(I.col);
    const GLB float *val = gp((const float *)I.val);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB uint8_t *mat = gp(I.mat);
    const GLB int32_t *src_tile = gp(I.src_tile);
    for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
    __syncthreads();
    const int R = I.rows_per_tile;
    const int64_t n_items = (I.n_slow + kRowListItem - 1) / kRowListItem;
    for (int64_t j = blockIdx.x; j < n_items; j += gridDim.x) {
        const int64_t i = j * kRowListItem + threadIdx.x;
        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        if (i < I.n_slow) {
            const int64_t r = gp(I.slow_rows)[i];
            const int64_t lo = (int64_t)rp[r], hi = (int64_t)rp[r + 1];
            float acc = 0.0f;
            for (int64_t kb = lo; kb < hi; kb += kRowListWin) {
                float vw[kRowListWin], xw[kRowListWin];
#pragma unroll
                for (int u = 0; u < kRowListWin; ++u) {
                    const int64_t k = min(kb + u, hi - 1);
                    vw[u] = val[k];
                    xw[u] = X[col[k]];
                }
#pragma unroll
                for (int u = 0; u < kRowListWin; ++u)
                    if (kb + u < hi) acc += vw[u] * xw[u];
            }
            float v = acc * scale;
            const int tile = (int)(r / R);
            const int sb = src_tile[tile], se = src_tile[tile + 1];
            if (sb < se) {
                int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                double s = 0.0;
                bool any = false;
                for (; e2 < se && I.src_row[e2] == r; ++e2) {
                    s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                    any = true;
                }
                if (any) v += (float)ldexp(s, -sc.En);
            }
            Y[r] = v;
            if (r < I.n_states) {
                sN += (double)v;
                sA += s_abs[mat[vox_of(r, I.vox_mul)]] * (double)v;
                mx = fmaxf(mx, v);
            } else {
                sE += (double)v;
            }
        }
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            const int64_t nc = I.n_chunks, b = I.slow_part + 4 * j + wave;
            I.partials[(int64_t)kSlotN * nc + b] = wN;
            I.partials[(int64_t)kSlotEsc * nc + b] = wE;
            I.partials[(int64_t)kSlotAbs * nc + b] = wA;
            I.partials[(int64_t)kSlotMax * nc + b] = wM;
        }
    }
}

// The two-voxel rows (columns two runs of kVox2Run: the states of two
// voxels, e.g. the transmitted and the reflected part of an interface row),
// a thread per row: work item j (blockIdx.x, then every gridDim.x-th) is rows
// kVox2Item j onwards of their list.  A row's values are a 16-byte aligned
// block of their compact copy; x at a run comes as the eight aligned quads
// that hold it (the state buffers keep kStatePad entries past the last row,
// so these stay inside) and is shifted into place by the run's offset in its
// first quad, two selects per entry.  Entries are added in column order (the
// CSR step's products and order: y is equal bit for bit).  Partials of index
// vox2_part + 4j + wave.
typedef float f8 __attribute__((ext_vector_type(8)));
typedef float f16 __attribute__((ext_vector_type(16)));
typedef float f32x32 __attribute__((ext_vector_type(32)));

// x[c .. c + 32) shifted: entry k is x[c + k] (k < 29); the eight aligned
// quads from c & ~3, then whole-vector selects by the shift (vectors, not an
// indexed array, so that the selection stays in registers)
__device__ __forceinline__ f32x32 x_run(const GLB float *X, int32_t c)
{
    const int32_t c0 = c & ~3, s = c & 3;
    const GLB f4 *p = (const GLB f4 *)(X + c0);
    const f8 a = __builtin_shufflevector(p[0], p[1], 0, 1, 2, 3, 4, 5, 6, 7);
    const f8 b = __builtin_shufflevector(p[2], p[3], 0, 1, 2, 3, 4, 5, 6, 7);
    const f8 c8 = __builtin_shufflevector(p[4], p[5], 0, 1, 2, 3, 4, 5, 6, 7);
    const f8 d = __builtin_shufflevector(p[6], p[7], 0, 1, 2, 3, 4, 5, 6, 7);
    const f16 ab = __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
    const f16 cd = __builtin_shufflevector(c8, d, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
    const f32x32 F = __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17,
                                             18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31);
    const f32x32 F1 = __builtin_shufflevector(F, F, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                                              19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 31);
    const f32x32 G = (s & 1) ? F1 : F;
    const f32x32 G2 = __builtin_shufflevector(G, G, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19,
                                              20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 31, 31);
    return (s & 2) ? G2 : G;
}

__global__ void __launch_bounds__(kNT) step_spmv_vox2(const StepInst *__restrict__ insts)
{
    __shared__ double s_abs[kMatMax];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const Scale sc = step_scale(I, 0, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB int32_t *src_tile = gp(I.src_tile);
    const GLB int32_t *info = gp(I.vox2_info);
    const GLB float *v2 = gp(I.vox2_val);
    for (int q = threadIdx.x; q < I.n_mat; q += kNT) s_abs[q] = gp(I.absorb)[q];
    __syncthreads();
    const int R = I.rows_per_tile;
    const int64_t n_items = (I.n_vox2 + kVox2Item - 1) / kVox2Item;
    for (int64_t j = blockIdx.x; j < n_items; j += gridDim.x) {
        const int64_t i = j * kVox2Item + threadIdx.x;
        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        if (i < I.n_vox2) {
            const i4 in = *(const GLB i4 *)(info + 4 * i);
            const int32_t r = in[0];
            const GLB float *vr = v2 + i * kVox2Len;
            // the row's 52 values: 13 aligned quads (entry k of the second
            // run is value kVox2Run + k)
            const GLB f4 *pv = (const GLB f4 *)vr;
            f4 vq[kVox2Len / 4];
#pragma unroll
            for (int q = 0; q < kVox2Len / 4; ++q) vq[q] = pv[q];
            const f32x32 wa = x_run(X, in[1]), wb = x_run(X, in[2]);
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < kVox2Run; ++k) acc += vq[k >> 2][k & 3] * wa[k];
#pragma unroll
            for (int k = 0; k < kVox2Run; ++k) acc += vq[(kVox2Run + k) >> 2][(kVox2Run + k) & 3] * wb[k];
            float v = acc * scale;
            const int tile = r / R;
            const int sb = src_tile[tile], se = src_tile[tile + 1];
            if (sb < se) {
                int e2 = lower_bound_rows<int32_t>(I.src_row, sb, se, r);
                double sacc = 0.0;
                bool any = false;
                for (; e2 < se && I.src_row[e2] == r; ++e2) {
                    sacc += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                    any = true;
                }
                if (any) v += (float)ldexp(sacc, -sc.En);
            }
            Y[r] = v;
            if (r < I.n_states) {
                sN += (double)v;
                sA += s_abs[in[3]] * (double)v;
                mx = fmaxf(mx, v);
            } else {
                sE += (double)v;
            }
        }
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            const int64_t nc = I.n_chunks, b = I.vox2_part + 4 * j + wave;
            I.partials[(int64_t)kSlotN * nc + b] = wN;
            I.partials[(int64_t)kSlotEsc * nc + b] = wE;
            I.partials[(int64_t)kSlotAbs * nc + b] = wA;
            I.partials[(int64_t)kSlotMax * nc + b] = wM;
        }
    }
}

// Detector sums of the single-rhs step by row groups (Eq. (27)): block (p, d)
// forms the sum F * y over part p of detector d's entries (every thread every
// 256th entry, then a fixed-order block sum) from the stored y.
__global__ void __launch_bounds__(kNT) spmv_detectors(const StepInst *__restrict__ insts)
{
    __shared__ double s_red[kNT];
    const StepInst &I = insts[0];
    const int64_t t = I.t[0];
    if (t >= *I.t_end) return;
    const int p = blockIdx.x, d = blockIdx.y;
    const GLB float *Y = gp((const float *)((t & 1) ? I.buf0 : I.buf1));
    const int64_t b = I.ddet_ptr[d], n = I.ddet_ptr[d + 1] - b;
    const int64_t pb = b + p * n / kDetParts, pe = b + (p + 1) * n / kDetParts;
    double acc = 0.0;
    for (int64_t k = pb + threadIdx.x; k < pe; k += kNT) acc += I.ddet_F[k] * (double)Y[I.ddet_row[k]];
    acc = block_sum<kNT>(acc, s_red);
    if (threadIdx.x == 0) det_direct_sums(I.partials, I.n_det, 1, I.n_chunks)[(int64_t)d * kDetParts + p] = acc;
}

// ---------------------------------------------------------------------------
// finalize: fixed-order reduction of the chunk partials, series and control
// ---------------------------------------------------------------------------
// Two-level reduction of the per-chunk partials in a fixed order, in two
// kernels (the kernel boundary orders the levels; no device-scope fence).
// finalize_seg: block (seg, inst, rhs) sums the chunks of segment seg
// (contiguous, kFinSeg segments per instance) for every slot and stores one
// value per slot.  finalize_step: block (inst, rhs) sums the segments in
// ascending order, records the series and advances the control words.  The
// order of every addition depends only on the number of chunks.
__global__ void __launch_bounds__(kNT) finalize_seg(const StepInst *__restrict__ insts)
{
    constexpr int NW = kNT / 64;
    __shared__ double s_w[4][NW];
    const StepInst &I = insts[blockIdx.y];
    const int rhs = blockIdx.z;
    if (rhs >= I.n_rhs) return;
    const int64_t t = I.t[rhs];
    if (t >= scalar_i64(*I.t_end)) return;
    const int64_t nc = I.n_chunks;
    const int nseg = (int)min((int64_t)kFinSeg, nc);
    const int seg = blockIdx.x;
    if (seg >= nseg) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nr = I.n_rhs, nslot = kSlotDet + I.n_det;
    const int64_t c0 = seg * nc / nseg, c1 = (seg + 1) * nc / nseg;
    const GLB double *part = gp(I.partials);
    GLB double *segp = gpw(I.partials + (int64_t)nslot * nr * nc);   // [slot * n_rhs + rhs][kFinSeg]
    // up to four slots per pass, so their loads are in flight together
    // with direct detector sums only the totals have chunk partials
    const int nsum = I.det_direct ? kSlotDet : nslot;
    if (I.det_direct && tid < I.n_det) {
        const double *ds = det_direct_sums(I.partials, I.n_det, nr, nc);
        double v = 0.0;
        if (seg == 0)
            for (int p = 0; p < kDetParts; ++p) v += ds[((int64_t)tid * kDetParts + p) * nr + rhs];
        segp[((int64_t)(kSlotDet + tid) * nr + rhs) * kFinSeg + seg] = v;
    }
    for (int k0 = 0; k0 < nsum; k0 += 4) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t c = c0 + tid; c < c1; c += kNT) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + j;
                if (k < nsum) {
                    const double v = part[((int64_t)k * nr + rhs) * nc + c];
                    a[j] = (k == kSlotMax) ? fmax(a[j], v) : a[j] + v;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double w = (k0 + j == kSlotMax) ? wave_max(a[j]) : wave_sum(a[j]);
            if (lane == 0) s_w[j][wave] = w;
        }
        __syncthreads();
        if (tid < 4 && k0 + tid < nsum) {
            const int k = k0 + tid;
            double r = s_w[tid][0];
            for (int w = 1; w < NW; ++w) r = (k == kSlotMax) ? fmax(r, s_w[tid][w]) : r + s_w[tid][w];
            segp[((int64_t)k * nr + rhs) * kFinSeg + seg] = r;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kNT) finalize_step(const StepInst *__restrict__ insts, int32_t *queue)
{
    constexpr int NW = kNT / 64;
    __shared__ double s_fin[kSlotDet + kFinDetMax];
    // the step kernel that used the work counter has completed: reset it for
    // the next step (a kernel store, so the step loop can be graph-captured)
    if (queue && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *queue = 0;
    const StepInst &I = insts[blockIdx.x];
    const int rhs = blockIdx.y;
    if (rhs >= I.n_rhs) return;
    const int64_t t = I.t[rhs];
    if (t >= scalar_i64(*I.t_end)) return;
    const int64_t nc = I.n_chunks;
    const int nseg = (int)min((int64_t)kFinSeg, nc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nr = I.n_rhs, nslot = kSlotDet + I.n_det;
    const GLB double *segp = gp(I.partials + (int64_t)nslot * nr * nc);
    // lane l combines segments l, l + 64, ... in ascending order, then the wave
    for (int k = wave; k < nslot; k += NW) {
        const GLB double *sp = segp + ((int64_t)k * nr + rhs) * kFinSeg;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kFinSeg / 64; ++j) {
            const int sg = lane + 64 * j;
            if (sg < nseg) {
                const double u = sp[sg];
                v = (k == kSlotMax) ? fmax(v, u) : v + u;
            }
        }
        v = (k == kSlotMax) ? wave_max(v) : wave_sum(v);
        if (lane == 0) s_fin[k] = v;
    }
    __syncthreads();
    const Scale sc = step_scale(I, rhs, t);
    for (int d = tid; d < I.n_det; d += kNT) I.ser_det[(t * I.n_det + d) * nr + rhs] = s_fin[kSlotDet + d];
    if (tid == 0) {
        I.ser_tot[(t * 3 + 0) * nr + rhs] = s_fin[kSlotN];
        I.ser_tot[(t * 3 + 1) * nr + rhs] = s_fin[kSlotEsc];
        I.ser_tot[(t * 3 + 2) * nr + rhs] = I.abs_cur[rhs];
        I.ser_abs_exp[t * nr + rhs] = I.E[rhs];
        I.ser_exp[t * nr + rhs] = sc.En;
        I.abs_cur[rhs] = s_fin[kSlotAbs];
        I.M[rhs] = s_fin[kSlotMax];
        I.E[rhs] = sc.En;
        I.t[rhs] = t + 1;
    }
}

// ---------------------------------------------------------------------------
// Matrix-free (structured) step, one right-hand side
//
// Row (w, m') of a state takes the plain move of its upstream voxel
// u = w - e_m' (when u is inside and has w's refractive index) and the
// irregular moves listed for it; an escape row takes its one leaving move.
// A move (u, m, f) contributes f C_q(u)[m][n] to column 26 u + n; groups of
// moves of one voxel are merged per column in FP64 and in ascending m, and
// each entry is rounded exactly as the assembly stores it, then multiplied
// by x in ascending column order: the row value equals the CSR row value bit
// for bit, while the matrix itself never leaves the chip (per row only the
// upstream voxel's 26 states of x are read, from L2).
// ---------------------------------------------------------------------------
constexpr int kStructMatLds = kStructMatLdsHost;   // materials the direction-major kernel takes (8 x 8 index-pair mask)

__device__ __forceinline__ uint64_t mix64_dev(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// FP64 -> FP32 of a nonnegative value as the assembly stores it
__device__ __forceinline__ float round_entry(double a, int rounding, int64_t row, int64_t col)
{
    float f = (float)a;
    if (rounding == DRTS_ROUND_DITHER && (double)f != a) {
        const uint32_t bits = __float_as_uint(f);
        const float g = __uint_as_float((double)f < a ? bits + 1u : bits - 1u);
        // |g - f| is a power of two: scaling by its exponent is the exact quotient
        const double p = ldexp(fabs((double)f - a), -ilogb(fabs((double)g - (double)f)));
        const uint64_t key = ((uint64_t)row << 32) ^ (uint64_t)(uint32_t)col;
        const double u = (double)(mix64_dev(key) >> 11) * 0x1p-53;
        if (u < p) f = g;
    }
    return f;
}

template <typename VT> struct StructVals;
template <> struct StructVals<float> {
    // entry of a plain move (factor 1): the block value rounded like the CSR
    __device__ static float plain(float cf, double cd, int rounding, int64_t row, int64_t col)
    {
        return rounding == DRTS_ROUND_DITHER ? round_entry(cd, rounding, row, col) : cf;
    }
    __device__ static float merged(double a, int rounding, int64_t row, int64_t col)
    {
        return round_entry(a, rounding, row, col);
    }
};
template <> struct StructVals<double> {
    __device__ static double plain(float, double cd, int, int64_t, int64_t) { return cd; }
    __device__ static double merged(double a, int, int64_t, int64_t) { return a; }
};

// Row value from the blocks and move lists, x read from global memory.
// MODE 2 multiplies the FP64 coefficients with the FP32 x in FP64, adds the
// terms of the row in FP64 in column order (one fma each) and rounds the row
// once to FP32, so the value rounding error disappears.  Otherwise values are
// rounded as stored.
// x access of struct_row: x[c] of a single state, or X[c][lane] of a state
// with n_rhs columns (lanes past n_rhs read a valid column and drop it)
template <typename VT> struct XPlain {
    const GLB VT *x;
    __device__ __forceinline__ VT operator()(int64_t c) const { return x[c]; }
};
struct XColumn {
    const GLB float *x;
    int k, lane;
    __device__ __forceinline__ float operator()(int64_t c) const { return x[c * k + lane]; }
};

template <typename VT, int MODE, typename XA>
__device__ __forceinline__ VT struct_row_a(const StructArgs &sa, int64_t r, const XA &xa, int64_t k_first,
                                           int64_t k_end)
{
    const GLB float *Chi = gp(sa.blocks32);
    const CST double *Cd = cst(sa.blocks64);
    const GLB uint8_t *mat = gp(sa.mat);
    const GLB double *index = gp(sa.index);
    VT acc = 0;
    double acc_d = 0.0;   // MODE 2
    auto plain_group = [&](int64_t u, int m) {
        const int q = mat[u];
        const int off = (q * kDirs + m) * kDirs;
        VT xv[kDirs];
#pragma unroll
        for (int n = 0; n < kDirs; ++n) xv[n] = xa(kDirs * u + n);
#pragma unroll
        for (int n = 0; n < kDirs; ++n) {
            if (MODE == 2) {
                acc_d = __builtin_fma(Cd[off + n], (double)xv[n], acc_d);
            } else {
                const VT c = StructVals<VT>::plain(Chi[off + n], Cd[off + n], sa.rounding, r, kDirs * u + n);
                acc += c * xv[n];
            }
        }
    };
    if (r >= sa.n_states) {
        const int64_t s = gp(sa.escape_state)[r - sa.n_states];
        plain_group(s / kDirs, (int)(s % kDirs));
        return MODE == 2 ? (VT)acc_d : acc;
    }
    const int64_t w = r / kDirs;
    const int mp = (int)(r % kDirs);
    const int x0 = (int)(w % sa.nx), y0 = (int)((w / sa.nx) % sa.ny), z0 = (int)(w / ((int64_t)sa.nx * sa.ny));
    const int ux = x0 - dir_dx(mp), uy = y0 - dir_dy(mp), uz = z0 - dir_dz(mp);
    int64_t ureg = -1;
    if (ux >= 0 && ux < sa.nx && uy >= 0 && uy < sa.ny && uz >= 0 && uz < sa.nz) {
        const int64_t u = ux + (int64_t)sa.nx * (uy + (int64_t)sa.ny * uz);
        if (index[mat[u]] == index[mat[w]]) ureg = u;
    }
    int64_t k = 0, kend = 0;
    const GLB int64_t *irr_row = gp(sa.irr_row), *irr_vox = gp(sa.irr_vox);
    const GLB int32_t *irr_dir = gp(sa.irr_dir);
    const GLB double *irr_f = gp(sa.irr_f);
    if (k_first >= 0) {
        // the caller knows the row's range of the irregular-move list
        k = k_first;
        kend = k_end;
    } else if (sa.n_irr > 0 && ((gp(sa.irr_bits)[r >> 5] >> (r & 31)) & 1u)) {
        int64_t lo = 0, hi = sa.n_irr;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (irr_row[mid] < r) lo = mid + 1;
            else hi = mid;
        }
        k = lo;
        kend = k;
        while (kend < sa.n_irr && irr_row[kend] == r) ++kend;
    }
    while (k < kend || ureg >= 0) {
        const int64_t ug = k < kend ? irr_vox[k] : INT64_MAX;
        if (ureg >= 0 && ureg < ug) {
            plain_group(ureg, mp);
            ureg = -1;
            continue;
        }
        int64_t k1 = k;
        while (k1 < kend && irr_vox[k1] == ug) ++k1;
        const int q = mat[ug];
        // all loads of the group are independent of each other: x of ug and
        // each move's block row are requested at once, and the merged
        // coefficient of column n sums the moves in list order as before
        VT xv[kDirs];
#pragma unroll
        for (int n = 0; n < kDirs; ++n) xv[n] = xa(kDirs * ug + n);
        double a[kDirs];
#pragma unroll
        for (int n = 0; n < kDirs; ++n) a[n] = 0.0;
        for (int64_t kk = k; kk < k1; ++kk) {
            const double f = irr_f[kk];
            const int off = (q * kDirs + irr_dir[kk]) * kDirs;
#pragma unroll
            for (int n = 0; n < kDirs; ++n) {
                const double c = Cd[off + n];
                if (c != 0.0) a[n] = a[n] + f * c;
            }
        }
#pragma unroll
        for (int n = 0; n < kDirs; ++n) {
            if (a[n] != 0.0) {
                if (MODE == 2) acc_d = __builtin_fma(a[n], (double)xv[n], acc_d);
                else acc += StructVals<VT>::merged(a[n], sa.rounding, r, kDirs * ug + n) * xv[n];
            }
        }
        k = k1;
    }
    return MODE == 2 ? (VT)acc_d : acc;
}

template <typename VT, int MODE>
__device__ __forceinline__ VT struct_row(const StructArgs &sa, int64_t r, const GLB VT *x, int64_t k_first = -1,
                                         int64_t k_end = -1)
{
    return struct_row_a<VT, MODE>(sa, r, XPlain<VT>{x}, k_first, k_end);
}

// Plain-move value of regular row r = (w, m'), x from global memory: the
// upstream voxel's block row when that voxel lies inside and has w's
// refractive index, else zero.
template <typename VT, int MODE>
__device__ __forceinline__ VT struct_plain_row(const StructArgs &sa, int64_t r, const GLB VT *x)
{
    const GLB uint8_t *mat = gp(sa.mat);
    const GLB double *index = gp(sa.index);
    const int64_t w = r / kDirs;
    const int mp = (int)(r % kDirs);
    const int x0 = (int)(w % sa.nx), y0 = (int)((w / sa.nx) % sa.ny), z0 = (int)(w / ((int64_t)sa.nx * sa.ny));
    const int ux = x0 - dir_dx(mp), uy = y0 - dir_dy(mp), uz = z0 - dir_dz(mp);
    VT acc = 0;
    if (ux >= 0 && ux < sa.nx && uy >= 0 && uy < sa.ny && uz >= 0 && uz < sa.nz) {
        const int64_t u = ux + (int64_t)sa.nx * (uy + (int64_t)sa.ny * uz);
        const int q = mat[u];
        if (index[q] == index[mat[w]]) {
            const int off = (q * kDirs + mp) * kDirs;
            const GLB VT *xu = x + kDirs * u;
            const GLB float *Chi = gp(sa.blocks32);
            const CST double *Cd = cst(sa.blocks64);
            VT xv[kDirs];
#pragma unroll
            for (int n = 0; n < kDirs; ++n) xv[n] = xu[n];
            if (MODE == 2 || MODE == 3) {
                double a = 0.0;
#pragma unroll
                for (int n = 0; n < kDirs; ++n) a = __builtin_fma(Cd[off + n], (double)xv[n], a);
                acc = (VT)a;
            } else {
#pragma unroll
                for (int n = 0; n < kDirs; ++n) {
                    const VT c = StructVals<VT>::plain(Chi[off + n], Cd[off + n], sa.rounding, r, kDirs * u + n);
                    acc += c * xv[n];
                }
            }
        }
    }
    return acc;
}

__device__ __forceinline__ bool struct_irregular(const StructArgs &sa, int64_t r)
{
    return sa.n_irr > 0 && ((gp(sa.irr_bits)[r >> 5] >> (r & 31)) & 1u);
}

// A voxel tile: a segment of seg_len voxels of one x-line.
struct StructTile {
    int64_t row0;
    int nrows;
    int x0, len;
    int64_t line;   // y + ny z
};

// 32-bit index arithmetic throughout: a single-rhs state has fewer than 2^30
// rows (the solver refuses larger ones), so every row index fits.
__device__ __forceinline__ StructTile struct_tile(const StructArgs &sa, int64_t k)
{
    StructTile T;
    const uint32_t kk = (uint32_t)k, spl = (uint32_t)sa.segs_per_line;
    const uint32_t line = kk / spl;
    T.line = line;
    T.x0 = (int)(kk - line * spl) * sa.seg_len;
    T.len = min(sa.seg_len, sa.nx - T.x0);
    T.row0 = (int64_t)(uint32_t)(kDirs * (T.x0 + sa.nx * (int)line));
    T.nrows = kDirs * T.len;
    return T;
}

// Matrix-free step, regular rows of the voxel tiles, x gathered from global
// memory: modes 0 (exact values: FP64, or FP32 values that need the dithered
// rounding of each entry) and 3 (FP64 row sums for media with more materials
// than the direction-major kernel takes).  A tile is kStructSegLen voxels of
// one x-line, a thread per row.  Irregular rows (wall reflections, Fresnel
// splits) and escape rows are left to step_struct_x.
template <typename VT, int MODE>
__global__ void __launch_bounds__(256) step_struct(StructArgs sa, const StepInst *__restrict__ insts,
                                                    const WorkItem *__restrict__ work, int64_t n_work,
                                                    int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    static_assert(MODE == 0 || MODE == 3, "gather modes");
    constexpr int NT = 256, NW = NT / 64, L = kStructSegLen;
    constexpr int ROWS = kDirs * L;
    constexpr int NPASS = (ROWS + NT - 1) / NT;
    __shared__ int32_t s_src[kChunkMax + 1];
    __shared__ int32_t s_det[kChunkMax + 1];
    __shared__ double s_abs[kMatMax];
    __shared__ VT s_y[ROWS];
    __shared__ double s_wred[4][NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        const int64_t t = scalar_i64(I.t[0]);
        if (t >= scalar_i64(*I.t_end)) continue;
        const Scale sc = step_scale(I, 0, t);
        const VT scale = (VT)ldexp(1.0, -sc.k);
        const GLB VT *x = gp((const VT *)((t & 1) ? I.buf1 : I.buf0));
        GLB VT *y = gpw((VT *)((t & 1) ? I.buf0 : I.buf1));
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int ntc = (int)min((int64_t)I.tiles_per_chunk, I.n_tiles - tile0);
        for (int j = tid; j <= ntc; j += NT) {
            s_src[j] = gp(I.src_tile)[tile0 + j];
            s_det[j] = gp(I.det_tile)[tile0 + j];
        }
        for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
        __syncthreads();
        double sN = 0.0, sA = 0.0, dsum = 0.0;
        VT mx = 0;
        for (int j = 0; j < ntc; ++j) {
            const StructTile T = struct_tile(sa, tile0 + j);
#pragma unroll
            for (int p = 0; p < NPASS; ++p) {
                const int lr = tid + p * NT;
                if (lr >= T.nrows) continue;
                const int64_t r = T.row0 + lr;
                if (struct_irregular(sa, r)) continue;   // step_struct_x computes it
                const VT acc = struct_plain_row<VT, MODE>(sa, r, x);
                const int qw = gp(sa.mat)[r / kDirs];
                VT v = acc * scale;
                const int sb = s_src[j], se = s_src[j + 1];
                if (sb < se) {
                    int e2 = lower_bound_rows<int32_t>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && gp(I.src_row)[e2] == r; ++e2) {
                        s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                        any = true;
                    }
                    if (any) v += (VT)ldexp(s, -sc.En);
                }
                y[r] = v;
                s_y[lr] = v;
                sN += (double)v;
                sA += s_abs[qw] * (double)v;
                mx = v > mx ? v : mx;
            }
            __syncthreads();
            const int db = s_det[j], de = s_det[j + 1];
            if (db < de && tid < I.n_det) {
                for (int e2 = db; e2 < de; ++e2) {
                    if (gp(I.det_id)[e2] != tid) continue;
                    const int64_t row = gp(I.det_row)[e2];
                    if (!struct_irregular(sa, row)) dsum += gp(I.det_F)[e2] * (double)s_y[row - T.row0];
                }
            }
            __syncthreads();
        }
        const int64_t nc = I.n_chunks, c = item.chunk;
        const double wN = wave_sum(sN), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            s_wred[0][wave] = wN;
            s_wred[1][wave] = 0.0;
            s_wred[2][wave] = wA;
            s_wred[3][wave] = wM;
        }
        __syncthreads();
        GLB double *part = gpw(I.partials);
        if (tid < 4) {
            double a = s_wred[tid][0];
            for (int w = 1; w < NW; ++w) a = (tid == 3) ? fmax(a, s_wred[tid][w]) : a + s_wred[tid][w];
            part[(int64_t)tid * nc + c] = a;
        }
        if (tid < I.n_det) part[(int64_t)(kSlotDet + tid) * nc + c] = dsum;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Matrix-free step, one rhs, direction-major tiles (modes 1 and 2).
//
// A tile is a segment of up to kStructDmSeg = 64 voxels of one x-line; lane i
// of every wave is voxel x0 + i.  The rows of a direction m take x from the
// upstream voxels x0 + i - e_m, which lie on one of the 3 x 3 neighbouring
// line segments; for a fixed m they share a material inside a layer, so the
// coefficient row of (material, m) is wave-uniform and comes through the
// scalar cache into SGPRs, and LDS holds only x.  A tile runs in three
// phases, one per plane of upstream voxels (directions 17..25 read the plane
// below in z, 9..16 their own, 0..8 the plane above): each phase copies its
// three line segments (66 voxels of 26 floats each, contiguous in HBM)
// straight into LDS with LDS-destination buffer loads, and the four waves
// compute its directions (wave w every fourth one), writing each row value
// to the tile's row buffer.  A phase's halo is a third of the tile's, so five
// workgroups fit per CU and their copies overlap each other's work.  With 26
// floats per voxel, the 8-byte LDS reads of 32 lanes from consecutive voxels
// cover all 64 banks once.  The epilogue (sources, y store, FP64 sums,
// detectors) then runs a thread per row in row order.  Irregular rows are
// left to step_struct_x.  Terms are added in column order as in every other
// kernel: mode 1 with the nearest FP32 values (mul, then add), mode 2 in FP64
// (one fma per term), rounded once.
// ---------------------------------------------------------------------------
// Five waves per SIMD (96 VGPRs, a few spilled outside the row loop) beat
// four without spills on the 128^3 layered workload.
// BATCH: the work items belong to several instances, each with its own
// arguments in sas[item.inst] (an uneven batch in one launch); otherwise all
// items use sa0.
template <int MODE, bool BATCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) step_struct_dm(StructArgs sa0, const StructArgs *__restrict__ sas,
                                                       const StepInst *__restrict__ insts,
                                                       const WorkItem *__restrict__ work, int64_t n_work,
                                                       int xcd_remap, const int64_t *__restrict__ xcd_bounds)
{
    constexpr int NT = 256, NW = NT / 64, L = kStructDmSeg, HV = L + 2;
    constexpr int SEGF = HV * kDirs;        // floats per halo line segment
    constexpr int ROWS = kDirs * L;
    constexpr int BITW = ROWS / 32 + 2;     // bitmap words a tile's rows touch
    constexpr int RPT = (ROWS + NT - 1) / NT;    // epilogue rows per thread
    static_assert(SEGF % 4 == 0 && SEGF / 4 <= 2 * NT, "halo segment pieces");
    // phase ph reads upstream plane z0 + ph - 1 (halo segments 3 ph .. 3 ph + 2);
    // in the lattice order d = k - [k > 13], k = 9 (dz + 1) + 3 (dy + 1) + dx + 1,
    // its directions (dz = 1 - ph) are 17..25, 9..16 and 0..8
    static_assert(kDirs == 26, "direction order");
    extern __shared__ __attribute__((aligned(16))) float s_dm[];   // 3 SEGF halo floats, then ROWS row values
    __shared__ uint8_t s_q[9 * HV];         // material of every halo voxel, 255 outside the grid
    __shared__ uint32_t s_bits[BITW];
    __shared__ int32_t s_src[kChunkMax + 1];
    __shared__ int32_t s_det[kChunkMax + 1];
    __shared__ double s_abs[kStructMatLds];
    __shared__ double s_idx[kStructMatLds];
    __shared__ double s_wred[4][NW];
    float *s_x = s_dm;
    float *s_y = s_dm + 3 * SEGF;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // per instance: bit qu * kStructMatLds + qw of same_idx says materials qu
    // and qw have the same index; n_words is the size of the row bitmap
    uint64_t same_idx = 0;
    int64_t n_words = 0;
    int cached = -1;
    auto setup = [&](const StructArgs &s) {
        __syncthreads();   // every thread is done with the previous instance's table
        for (int q = tid; q < s.n_mat; q += NT) s_idx[q] = gp(s.index)[q];
        __syncthreads();
        same_idx = 0;
        for (int a = 0; a < s.n_mat; ++a)
            for (int b = 0; b < s.n_mat; ++b)
                if (s_idx[a] == s_idx[b]) same_idx |= 1ull << (a * kStructMatLds + b);
        n_words = (s.n_states + 31) / 32;
    };
    if (!BATCH) setup(sa0);
    const Walk wk = walk_of(n_work, xcd_remap, xcd_bounds);
    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StructArgs &sa = BATCH ? sas[item.inst] : sa0;
        if (BATCH && item.inst != cached) {
            setup(sa);
            cached = item.inst;
        }
        const StepInst &I = insts[item.inst];
        const int64_t t = scalar_i64(I.t[0]);
        if (t >= scalar_i64(*I.t_end)) continue;
        const Scale sc = step_scale(I, 0, t);
        const float scale = ldexpf(1.0f, -sc.k);
        const float *x = (const float *)((t & 1) ? I.buf1 : I.buf0);
        GLB float *y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
        const __amdgpu_buffer_rsrc_t rx = make_rsrc((const void *)x, (uint64_t)sa.n_states * 4);
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int ntc = (int)min((int64_t)I.tiles_per_chunk, I.n_tiles - tile0);
        for (int j = tid; j <= ntc; j += NT) {
            s_src[j] = gp(I.src_tile)[tile0 + j];
            s_det[j] = gp(I.det_tile)[tile0 + j];
        }
        for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
        __syncthreads();
        double sN = 0.0, sA = 0.0, dsum = 0.0;
        float mx = 0.0f;
        for (int j = 0; j < ntc; ++j) {
            const StructTile T = struct_tile(sa, tile0 + j);
            const int line = (int)T.line;
            const int zv0 = line / sa.ny, yv0 = line - zv0 * sa.ny;
            const int segf = (T.len + 2) * kDirs;   // floats the tile needs per segment
            const int segq = (segf + 3) / 4;        // their 16-byte pieces
            const int rb0 = (int)(T.row0 >> 5);
            for (int h = tid; h < 9 * HV; h += NT) {
                const int sg = h / HV, iv = h - sg * HV;
                const int xv = T.x0 - 1 + iv, yv = yv0 + sg % 3 - 1, zv = zv0 + sg / 3 - 1;
                uint8_t q = 255;
                if (xv >= 0 && xv < sa.nx && yv >= 0 && yv < sa.ny && zv >= 0 && zv < sa.nz)
                    q = gp(sa.mat)[xv + sa.nx * (yv + sa.ny * zv)];
                s_q[h] = q;
            }
            if (tid < BITW)
                s_bits[tid] = sa.n_irr > 0 ? gp(sa.irr_bits)[min(rb0 + tid, (int)n_words - 1)] : 0u;
#pragma unroll
            for (int ph = 0; ph < 3; ++ph) {
                // this phase's three segments: line (y0 + k - 1, z0 + ph - 1),
                // voxels x0 - 1 .. x0 + len.  A segment whose 16-byte pieces all
                // lie inside the state is copied straight into LDS; the others
                // (first and last line of the grid) float by float with a bounds
                // check.  Voxels outside the grid are marked in s_q, so no row
                // uses what their slots hold.
                const int zv = zv0 + ph - 1;
                const bool plane_in = zv >= 0 && zv < sa.nz;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int yv = yv0 + k - 1;
                    if (!plane_in || yv < 0 || yv >= sa.ny) continue;
                    float *seg = s_x + k * SEGF;
                    const int64_t fo = (int64_t)kDirs * (T.x0 - 1 + (int64_t)sa.nx * (yv + (int64_t)sa.ny * zv));
                    if (fo >= 0 && fo + 4 * (int64_t)segq <= sa.n_states) {
                        const uint32_t bo = (uint32_t)(4 * fo);   // 4 n_states < 2^32
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int c = u * NT + tid;
                            if (c < segq)
                                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                    rx, (__attribute__((address_space(3))) void *)(seg + 4 * (u * NT + 64 * wave)), 16,
                                    (int)(bo + 16u * (uint32_t)c), 0, 0, 0);
                        }
                    } else {
                        for (int e = tid; e < segf; e += NT) {
                            const int64_t f = fo + e;
                            seg[e] = (f >= 0 && f < sa.n_states) ? gp(x)[f] : 0.0f;
                        }
                    }
                }
                // every lane's pieces are in LDS once its loads have completed
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                const int qw = s_q[4 * HV + lane + 1];   // the row voxel (255 past the line)
                const int m0 = ph == 0 ? 17 : (ph == 1 ? 9 : 0);
                const int mn = ph == 1 ? 8 : 9;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int e = wave + NW * i;
                    if (e >= mn) continue;
                    const int m = m0 + e;
                    const int dx = dir_dx(m), dy = dir_dy(m);
                    const int k = 1 - dy, sg = 3 * ph + k, ix = lane + 1 - dx;
                    const int qu = s_q[sg * HV + ix];
                    // material bytes index the coefficient tables: only
                    // materials of the medium count as inside
                    const bool plain = qu < sa.n_mat && qw < sa.n_mat &&
                                       (qu == qw || ((same_idx >> (qu * kStructMatLds + qw)) & 1ull));
                    const uint64_t pm = __ballot(plain);
                    float v = 0.0f;
                    if (pm != 0) {
                        const int qf = __builtin_amdgcn_readlane(qu, (int)__builtin_ctzll(pm));
                        const bool uni = __ballot(plain && qu != qf) == 0;
                        const float *xs = s_x + k * SEGF + ix * kDirs;
                        if (MODE == 2) {
                            auto row_sum = [&](const CST double *C) {
                                double a = 0.0;
#pragma unroll
                                for (int n = 0; n < kDirs; ++n) a = __builtin_fma(C[n], (double)xs[n], a);
                                return (float)a;
                            };
                            v = uni ? row_sum(cst(sa.blocks64) + (qf * kDirs + m) * kDirs)
                                    : row_sum(cst(sa.blocks64) + ((plain ? qu : 0) * kDirs + m) * kDirs);
                        } else {
                            auto row_sum = [&](const CST float *C) {
                                float a = 0.0f;
#pragma unroll
                                for (int n = 0; n < kDirs; ++n) a += C[n] * xs[n];
                                return a;
                            };
                            v = uni ? row_sum(cst(sa.blocks32) + (qf * kDirs + m) * kDirs)
                                    : row_sum(cst(sa.blocks32) + ((plain ? qu : 0) * kDirs + m) * kDirs);
                        }
                        v = plain ? v * scale : 0.0f;
                    }
                    s_y[kDirs * lane + m] = v;
                }
                __syncthreads();   // the phase's halo is read before the next one lands
            }
#pragma unroll
            for (int p = 0; p < RPT; ++p) {
                const int lr = tid + p * NT;
                if (lr >= T.nrows) continue;
                const int64_t r = T.row0 + lr;
                const int r32 = (int)r;
                if ((s_bits[(r32 >> 5) - rb0] >> (r32 & 31)) & 1u) continue;   // step_struct_x computes it
                float v = s_y[lr];
                const int sb = s_src[j], se = s_src[j + 1];
                if (sb < se) {
                    int e2 = lower_bound_rows<int32_t>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && gp(I.src_row)[e2] == r; ++e2) {
                        s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                        any = true;
                    }
                    if (any) {
                        v += (float)ldexp(s, -sc.En);
                        s_y[lr] = v;
                    }
                }
                y[r] = v;
                sN += (double)v;
                sA += s_abs[s_q[4 * HV + lr / kDirs + 1]] * (double)v;
                mx = v > mx ? v : mx;
            }
            __syncthreads();
            const int db = s_det[j], de = s_det[j + 1];
            if (db < de && tid < I.n_det) {
                for (int e2 = db; e2 < de; ++e2) {
                    if (gp(I.det_id)[e2] != tid) continue;
                    const int64_t row = gp(I.det_row)[e2];
                    const int r32 = (int)row;
                    if (!((s_bits[(r32 >> 5) - rb0] >> (r32 & 31)) & 1u))
                        dsum += gp(I.det_F)[e2] * (double)s_y[row - T.row0];
                }
            }
            __syncthreads();   // before the next tile's materials, bits and rows
        }
        const int64_t nc = I.n_chunks, c = item.chunk;
        const double wN = wave_sum(sN), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            s_wred[0][wave] = wN;
            s_wred[1][wave] = 0.0;
            s_wred[2][wave] = wA;
            s_wred[3][wave] = wM;
        }
        __syncthreads();
        GLB double *part = gpw(I.partials);
        if (tid < 4) {
            double a = s_wred[tid][0];
            for (int w = 1; w < NW; ++w) a = (tid == 3) ? fmax(a, s_wred[tid][w]) : a + s_wred[tid][w];
            part[(int64_t)tid * nc + c] = a;
        }
        if (tid < I.n_det) part[(int64_t)(kSlotDet + tid) * nc + c] = dsum;
        __syncthreads();
    }
}

// Matrix-free step, the rows step_struct leaves: irregular rows and escape
// rows, listed in ascending order in sa.xrows, kStructXRows per work item.
// Each row is built from its move lists (struct_row) with x from global
// memory; its partials go to chunk sa.chunk_base + item.
template <typename VT, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) step_struct_x(StructArgs sa0, const StructArgs *__restrict__ sas,
                                                      const StepInst *__restrict__ insts,
                                                      const WorkItem *__restrict__ xwork, int64_t n_xwork)
{
    constexpr int NT = 256, NW = NT / 64, XR = kStructXRows;
    __shared__ VT s_y[XR];
    __shared__ int64_t s_r[XR];
    __shared__ double s_abs[kMatMax];
    __shared__ double s_wred[4][NW];
    __shared__ double s_red[NT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int cached = -1;
    // one instance (its work items 0 .. n_items - 1) or the batch's list of
    // (instance, item) pairs
    const int64_t n_iter = BATCH ? n_xwork : (sa0.n_xrows + XR - 1) / XR;
    for (int64_t wq = blockIdx.x; wq < n_iter; wq += gridDim.x) {
        const WorkItem it = BATCH ? xwork[wq] : WorkItem{0, (int32_t)wq};
        const StructArgs &sa = BATCH ? sas[it.inst] : sa0;
        const StepInst &I = insts[it.inst];
        const int64_t t = scalar_i64(I.t[0]);
        if (t >= scalar_i64(*I.t_end)) continue;
        if (it.inst != cached) {
            __syncthreads();   // every thread is done with the previous instance's table
            for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
            __syncthreads();
            cached = it.inst;
        }
        const Scale sc = step_scale(I, 0, t);
        const VT scale = (VT)ldexp(1.0, -sc.k);
        const GLB VT *x = gp((const VT *)((t & 1) ? I.buf1 : I.buf0));
        GLB VT *y = gpw((VT *)((t & 1) ? I.buf0 : I.buf1));
        const GLB int64_t *xrows = gp(sa.xrows);
        const int64_t j = it.chunk;
        const int64_t k0 = j * XR;
        const int n = (int)min((int64_t)XR, sa.n_xrows - k0);
        double sN = 0.0, sE = 0.0, sA = 0.0;
        VT mx = 0;
        for (int i = tid; i < n; i += NT) {
            const int64_t r = xrows[k0 + i];
            s_r[i] = r;
            // irregular rows come with their range of the irregular-move list
            const int64_t kf = gp(sa.xirr)[k0 + i], ke = gp(sa.xirr)[k0 + i + 1];
            VT v = struct_row<VT, (MODE == 2 || MODE == 3) ? 2 : 0>(sa, r, x, kf, ke) * scale;
            if (sa.n_src_entries > 0 && r < sa.n_states) {
                int e2 = gp(sa.xsrc)[k0 + i];
                double s = 0.0;
                bool any = false;
                for (; e2 < sa.n_src_entries && gp(I.src_row)[e2] == r; ++e2) {
                    s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                    any = true;
                }
                if (any) v += (VT)ldexp(s, -sc.En);
            }
            y[r] = v;
            s_y[i] = v;
            if (r < sa.n_states) {
                sN += (double)v;
                sA += s_abs[gp(sa.mat)[r / kDirs]] * (double)v;
                mx = v > mx ? v : mx;
            } else {
                sE += (double)v;
            }
        }
        __syncthreads();
        // detectors: per detector, its entries whose rows lie in this item's
        // row span (a range of its row-sorted list, found on the host),
        // shared by all threads, then a fixed-order block sum; entries of rows
        // not in the item belong to the tile kernel
        const int64_t nc = I.n_chunks, c = sa.chunk_base + j;
        GLB double *part = gpw(I.partials);
        {
            const GLB int64_t *drow = gp(sa.ddet_row);
            const GLB double *dF = gp(sa.ddet_F);
            for (int d = 0; d < I.n_det; ++d) {
                const int64_t lo = gp(sa.xdrng)[(j * I.n_det + d) * 2], hi = gp(sa.xdrng)[(j * I.n_det + d) * 2 + 1];
                double acc = 0.0;
                for (int64_t e2 = lo + tid; e2 < hi; e2 += NT) {
                    const int64_t row = drow[e2];
                    int l = 0, h = n;
                    while (l < h) {
                        const int mid = (l + h) >> 1;
                        if (s_r[mid] < row) l = mid + 1;
                        else h = mid;
                    }
                    if (l < n && s_r[l] == row) acc += dF[e2] * (double)s_y[l];
                }
                acc = block_sum<NT>(acc, s_red);
                if (tid == 0) part[(int64_t)(kSlotDet + d) * nc + c] = acc;
            }
        }
        const double wN = wave_sum(sN), wE = wave_sum(sE), wA = wave_sum(sA), wM = wave_max((double)mx);
        if (lane == 0) {
            s_wred[0][wave] = wN;
            s_wred[1][wave] = wE;
            s_wred[2][wave] = wA;
            s_wred[3][wave] = wM;
        }
        __syncthreads();
        if (tid < 4) {
            double a = s_wred[tid][0];
            for (int w = 1; w < NW; ++w) a = (tid == 3) ? fmax(a, s_wred[tid][w]) : a + s_wred[tid][w];
            part[(int64_t)tid * nc + c] = a;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Matrix-free step for n_rhs right-hand sides (lanes = right-hand sides)
//
// Push form: one wave per source voxel u.  The wave reads u's 26 rows of X
// once (a coalesced 4 n_rhs-byte load each), forms z[m] = sum_n C[m][n] X[n]
// with the block coefficients read at wave-uniform addresses through the
// scalar cache (FP64 coefficients and FP64 row sums in mode 2), and writes
// z[m] as the whole row (u + e_m, m) of Y: every regular row is written by
// exactly one voxel, so X is read once per step instead of once per using
// row; a target outside the grid is u's escape row for m.  Rows marked in
// sa.pull_bits (irregular, source and detector rows, state rows whose
// upstream voxel is outside or across an index change) are left to the pull
// kernel.  Terms are added in column order as the single-rhs kernels add
// them.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(256) step_struct_mm(StructArgs sa, const StepInst *__restrict__ insts,
                                                       const WorkItem *__restrict__ work, int64_t n_work)
{
    constexpr int NT = 256, NW = NT / 64;
    __shared__ double s_abs[kMatMax];
    __shared__ double s_w[4][NW][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const StepInst &I = insts[0];
    for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
    __syncthreads();
    const int64_t t = scalar_i64(I.t[0]);
    if (t >= scalar_i64(*I.t_end)) return;
    const int nrhs = I.n_rhs;
    const bool active = lane < nrhs;
    const int xl = min(lane, nrhs - 1);
    Scale sc{0, 0};
    if (active) sc = step_scale(I, lane, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const GLB uint8_t *mat = gp(sa.mat);
    const GLB uint32_t *pull = gp(sa.pull_bits);
    const int nvox = (int)(sa.n_states / kDirs);
    const int64_t nc = I.n_chunks;
    // one set of partials per workgroup (chunk blockIdx.x): the walk over the
    // work items is fixed, so the sums are too
    double sN = 0.0, sA = 0.0, sE = 0.0;
    float mx = 0.0f;
    for (int64_t wi = blockIdx.x; wi < n_work; wi += gridDim.x) {
        const int c = work[wi].chunk;
        const int v0 = c * kStructVoxPerChunk, v1 = min(v0 + kStructVoxPerChunk, nvox);
        for (int u = v0 + wave; u < v1; u += NW) {
            const int q = mat[u];
            const int ux = u % sa.nx, uy = (u / sa.nx) % sa.ny, uz = u / (sa.nx * sa.ny);
            float xv[kDirs];
#pragma unroll
            for (int n = 0; n < kDirs; ++n) xv[n] = X[(int64_t)(kDirs * u + n) * nrhs + xl];
            double xd[kDirs];
            if (MODE == 2) {
#pragma unroll
                for (int n = 0; n < kDirs; ++n) xd[n] = (double)xv[n];
            }
            // lane m < 26 looks up target row (u + e_m, m) once: the state row of
            // the neighbour inside the grid, or else u's escape row for m (escape
            // rows of a voxel are consecutive, in ascending m); it is written here
            // unless it is a pull row; and the target voxel's material
            bool out = false;
            int lr = 0, lq = 0;
            if (lane < kDirs) {
                const int wx = ux + dir_dx(lane), wy = uy + dir_dy(lane), wz = uz + dir_dz(lane);
                out = !(wx >= 0 && wx < sa.nx && wy >= 0 && wy < sa.ny && wz >= 0 && wz < sa.nz);
                if (!out) {
                    const int w = wx + sa.nx * (wy + sa.ny * wz);
                    lr = kDirs * w + lane;
                    lq = mat[w];
                }
            }
            const uint64_t outs = __ballot(out);
            bool lok = false;
            if (lane < kDirs) {
                // with reflecting walls nothing leaves: no escape rows, and the
                // reflected moves are irregular (pull) rows
                const bool has_row = !out || sa.n_rows > sa.n_states;
                if (out && has_row)
                    lr = (int)sa.n_states + gp(sa.esc_base)[u] + __popcll(outs & ((1ull << lane) - 1ull));
                lok = has_row && !((pull[lr >> 5] >> (lr & 31)) & 1u);
            }
            const uint64_t pushed = __ballot(lok);
            for (int m = 0; m < kDirs; ++m) {
                if (!((pushed >> m) & 1ull)) continue;
                const int r = __builtin_amdgcn_readlane(lr, m);
                const int qw = __builtin_amdgcn_readlane(lq, m);
                const bool esc = (outs >> m) & 1ull;
                const int off = (q * kDirs + m) * kDirs;
                float acc = 0.0f;
                if (MODE == 2) {
                    const CST double *Cm = cst(sa.blocks64) + off;
                    double a = 0.0;
#pragma unroll
                    for (int n = 0; n < kDirs; ++n) a = __builtin_fma(Cm[n], xd[n], a);
                    acc = (float)a;
                } else {
                    const CST float *Cm = cst(sa.blocks32) + off;
#pragma unroll
                    for (int n = 0; n < kDirs; ++n) acc += Cm[n] * xv[n];
                }
                const float v = acc * scale;
                if (active) {
                    Y[(int64_t)r * nrhs + lane] = v;
                    if (esc) {
                        sE += (double)v;
                    } else {
                        sN += (double)v;
                        sA += s_abs[qw] * (double)v;
                        mx = fmaxf(mx, v);
                    }
                }
            }
        }
    }
    s_w[0][wave][lane] = sN;
    s_w[1][wave][lane] = sA;
    s_w[2][wave][lane] = (double)mx;
    s_w[3][wave][lane] = sE;
    __syncthreads();
    const int64_t c = blockIdx.x;
    if (wave == 0 && active) {
        const double N = ((s_w[0][0][lane] + s_w[0][1][lane]) + s_w[0][2][lane]) + s_w[0][3][lane];
        const double A = ((s_w[1][0][lane] + s_w[1][1][lane]) + s_w[1][2][lane]) + s_w[1][3][lane];
        const double M = fmax(fmax(s_w[2][0][lane], s_w[2][1][lane]), fmax(s_w[2][2][lane], s_w[2][3][lane]));
        const double E = ((s_w[3][0][lane] + s_w[3][1][lane]) + s_w[3][2][lane]) + s_w[3][3][lane];
        GLB double *part = gpw(I.partials);
        part[((int64_t)kSlotN * nrhs + lane) * nc + c] = N;
        part[((int64_t)kSlotEsc * nrhs + lane) * nc + c] = E;
        part[((int64_t)kSlotAbs * nrhs + lane) * nc + c] = A;
        part[((int64_t)kSlotMax * nrhs + lane) * nc + c] = M;
        for (int d = 0; d < I.n_det; ++d) part[((int64_t)(kSlotDet + d) * nrhs + lane) * nc + c] = 0.0;
    }
}

// Pull rows of the matrix-free many-rhs step (sa.xrows, kStructMmXRows per
// work item): each row from its move lists (struct_row) with X read per lane;
// sources of the row's own right-hand side; detector sums per wave in LDS,
// combined over the waves in a fixed order.  Partials go to chunk
// sa.chunk_base + item.
template <int MODE>
__global__ void __launch_bounds__(256) step_struct_mm_x(StructArgs sa, const StepInst *__restrict__ insts)
{
    constexpr int NT = 256, NW = NT / 64, XR = kStructMmXRows;
    extern __shared__ double s_det[];   // [NW][n_det][64]
    __shared__ double s_abs[kMatMax];
    __shared__ double s_w[4][NW][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const StepInst &I = insts[0];
    for (int q = tid; q < I.n_mat; q += NT) s_abs[q] = gp(I.absorb)[q];
    __syncthreads();
    const int64_t t = scalar_i64(I.t[0]);
    if (t >= scalar_i64(*I.t_end)) return;
    const int nrhs = I.n_rhs, nd = I.n_det;
    const bool active = lane < nrhs;
    const int xl = min(lane, nrhs - 1);
    Scale sc{0, 0};
    if (active) sc = step_scale(I, lane, t);
    const float scale = ldexpf(1.0f, -sc.k);
    const GLB float *X = gp((const float *)((t & 1) ? I.buf1 : I.buf0));
    GLB float *Y = gpw((float *)((t & 1) ? I.buf0 : I.buf1));
    const XColumn xa{X, nrhs, xl};
    const GLB int64_t *xrows = gp(sa.xrows);
    const GLB int64_t *xirr = gp(sa.xirr);
    const int64_t n_items = (sa.n_xrows + XR - 1) / XR;
    const int64_t nc = I.n_chunks;
    double *my_det = s_det + (int64_t)wave * nd * 64;
    // rows that take no move and no source: zero (a wave per row, the lanes
    // write its columns); they add nothing to the sums
    if (active)
        for (int64_t k = (int64_t)blockIdx.x * NW + wave; k < sa.n_zrows; k += (int64_t)gridDim.x * NW)
            Y[gp(sa.zrows)[k] * nrhs + lane] = 0.0f;
    // one set of partials per workgroup (chunk chunk_base + blockIdx.x), over a
    // fixed walk of the work items
    for (int d = 0; d < nd; ++d) my_det[d * 64 + lane] = 0.0;
    double sN = 0.0, sE = 0.0, sA = 0.0;
    float mx = 0.0f;
    for (int64_t j = blockIdx.x; j < n_items; j += gridDim.x) {
        const int64_t k0 = j * XR, k1 = min(k0 + XR, sa.n_xrows);
        for (int64_t k = k0 + wave; k < k1; k += NW) {
            const int64_t r = xrows[k];
            float v = struct_row_a<float, (MODE == 2) ? 2 : 0>(sa, r, xa, xirr[k], xirr[k + 1]) * scale;
            if (sa.n_src_entries > 0 && r < sa.n_states) {
                int e2 = gp(sa.xsrc)[k];
                double s = 0.0;
                bool any = false;
                for (; e2 < sa.n_src_entries && gp(I.src_row)[e2] == r; ++e2) {
                    if (gp(I.src_rhs)[e2] == lane) {
                        s += gp(I.src_w)[e2] * gp(I.amp)[t * I.n_src + gp(I.src_id)[e2]];
                        any = true;
                    }
                }
                if (any) v += (float)ldexp(s, -sc.En);
            }
            if (active) {
                Y[r * nrhs + lane] = v;
                if (r < sa.n_states) {
                    sN += (double)v;
                    sA += s_abs[gp(sa.mat)[r / kDirs]] * (double)v;
                    mx = fmaxf(mx, v);
                } else {
                    sE += (double)v;
                }
                if (sa.n_det_entries > 0) {
                    int e2 = gp(sa.xdet)[k];
                    for (; e2 < sa.n_det_entries && gp(I.det_row)[e2] == r; ++e2)
                        my_det[gp(I.det_id)[e2] * 64 + lane] += gp(I.det_F)[e2] * (double)v;
                }
            }
        }
    }
    s_w[0][wave][lane] = sN;
    s_w[1][wave][lane] = sE;
    s_w[2][wave][lane] = sA;
    s_w[3][wave][lane] = (double)mx;
    __syncthreads();
    const int64_t c = sa.chunk_base + blockIdx.x;
    if (wave == 0 && active) {
        const double N = ((s_w[0][0][lane] + s_w[0][1][lane]) + s_w[0][2][lane]) + s_w[0][3][lane];
        const double Es = ((s_w[1][0][lane] + s_w[1][1][lane]) + s_w[1][2][lane]) + s_w[1][3][lane];
        const double A = ((s_w[2][0][lane] + s_w[2][1][lane]) + s_w[2][2][lane]) + s_w[2][3][lane];
        const double M = fmax(fmax(s_w[3][0][lane], s_w[3][1][lane]), fmax(s_w[3][2][lane], s_w[3][3][lane]));
        GLB double *part = gpw(I.partials);
        part[((int64_t)kSlotN * nrhs + lane) * nc + c] = N;
        part[((int64_t)kSlotEsc * nrhs + lane) * nc + c] = Es;
        part[((int64_t)kSlotAbs * nrhs + lane) * nc + c] = A;
        part[((int64_t)kSlotMax * nrhs + lane) * nc + c] = M;
        for (int d = 0; d < nd; ++d) {
            const double D = ((s_det[(0 * nd + d) * 64 + lane] + s_det[(1 * nd + d) * 64 + lane]) +
                              s_det[(2 * nd + d) * 64 + lane]) +
                             s_det[(3 * nd + d) * 64 + lane];
            part[((int64_t)(kSlotDet + d) * nrhs + lane) * nc + c] = D;
        }
    }
}

}  // namespace

hipError_t launch_step(const StepInst *insts_dev, const WorkItem *work_dev, int64_t n_work, int n_inst,
                       int n_rhs_max, int value_f64, int rp64, int spmm, int grid, int xcd_remap,
                       const int64_t *xcd_bounds, int rows_per_tile, int n_det_max, int32_t *queue,
                       hipStream_t stream, int64_t n_slow, int64_t n_vox2, int vi)
{
    (void)n_inst;
    (void)n_rhs_max;
    (void)rows_per_tile;
    if (n_work <= 0) return hipSuccess;
    // workgroups past the work list would only start and exit; a multiple of
    // the XCD count keeps the per-XCD walk available
    grid = (int)std::min<int64_t>(grid, (n_work + kXcds - 1) / kXcds * kXcds);
    const dim3 g((unsigned)grid), b(kNT);
    if (spmm == 2 || spmm == 3) {
        // value-indexed fast groups (the dictionaries in dynamic LDS) for the
        // FP64 sums only: measured on the 96^3 slab with 64 rhs, they take
        // the FP64-sum step from 4.73 to 4.19 ms but the FP32 one from 4.05
        // to 4.70 ms
        const int ntab = vi & 0xff;
        const size_t dl = (size_t)ntab * kViDict * sizeof(float);
        const int x = xcd_remap & 1;
        if (ntab > 0 && spmm == 3) {
            if (rp64)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int64_t, true, true>), g, b, dl, stream,
                                   insts_dev, work_dev, n_work, x, xcd_bounds);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int32_t, true, true>), g, b, dl, stream,
                                   insts_dev, work_dev, n_work, x, xcd_bounds);
        } else if (rp64 && spmm == 3)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int64_t, true, false>), g, b, 0, stream, insts_dev,
                               work_dev, n_work, x, xcd_bounds);
        else if (rp64)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int64_t, false, false>), g, b, 0, stream, insts_dev,
                               work_dev, n_work, x, xcd_bounds);
        else if (spmm == 3)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int32_t, true, false>), g, b, 0, stream, insts_dev,
                               work_dev, n_work, x, xcd_bounds);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(step_spmm_grouped<int32_t, false, false>), g, b, 0, stream, insts_dev,
                               work_dev, n_work, x, xcd_bounds);
        if (n_det_max > 0) {
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(spmm_detectors, dim3(kDetParts, (unsigned)n_det_max), b, 0, stream, insts_dev);
        }
    } else if (spmm) {
        const size_t lds = (size_t)4 * n_det_max * 64 * sizeof(double);
        if (rp64)
            hipLaunchKernelGGL(step_spmm<int64_t>, g, b, lds, stream, insts_dev, work_dev, n_work, xcd_remap & 1,
                               xcd_bounds);
        else
            hipLaunchKernelGGL(step_spmm<int32_t>, g, b, lds, stream, insts_dev, work_dev, n_work, xcd_remap & 1,
                               xcd_bounds);
    } else {
        const dim3 g1((unsigned)grid);
        const int variant = (xcd_remap >> 1) & 15;
        const int remap = xcd_remap & 1;
        if (variant == DRTS_SPMV_GROUPED) {
            // the fast groups, then the listed rows, the two-voxel rows, the detectors
            // vi: dictionaries in bits 0-7, bit 8: a fast group holds a source row
            const size_t tab_lds = (size_t)(vi & 0xff) * kViDict * sizeof(float);
            if (vi & 0x100)
                hipLaunchKernelGGL((step_spmv_grouped_vi<kGroupPairsVi, true>), g1, dim3(kNT), tab_lds, stream,
                                   insts_dev, work_dev, n_work, remap, xcd_bounds);
            else if (vi)
                hipLaunchKernelGGL((step_spmv_grouped_vi<kGroupPairsVi, false>), g1, dim3(kNT), tab_lds, stream,
                                   insts_dev, work_dev, n_work, remap, xcd_bounds);
            else
                hipLaunchKernelGGL(step_spmv_grouped<kGroupPairs>, g1, dim3(kNT), 0, stream, insts_dev, work_dev,
                                   n_work, remap, xcd_bounds);
            const hipError_t e0 = hipGetLastError();
            if (e0 != hipSuccess) return e0;
            if (n_slow > 0) {
                const int64_t items = (n_slow + kRowListItem - 1) / kRowListItem;
                const dim3 gr((unsigned)std::min<int64_t>(items, 2048));
                if (rp64) hipLaunchKernelGGL(step_spmv_rowlist<int64_t>, gr, dim3(kNT), 0, stream, insts_dev);
                else hipLaunchKernelGGL(step_spmv_rowlist<int32_t>, gr, dim3(kNT), 0, stream, insts_dev);
            }
            if (n_vox2 > 0) {
                const int64_t items = (n_vox2 + kVox2Item - 1) / kVox2Item;
                hipLaunchKernelGGL(step_spmv_vox2, dim3((unsigned)std::min<int64_t>(items, 2048)), dim3(kNT), 0,
                                   stream, insts_dev);
            }
            if (n_det_max > 0) {
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(spmv_detectors, dim3(kDetParts, (unsigned)n_det_max), dim3(kNT), 0, stream,
                                   insts_dev);
            }
            return hipGetLastError();
        }
        if (variant == kVariantLongRows) {
            // rows of several hundred entries: a wave per row
            if (value_f64) {
                if (rp64) hipLaunchKernelGGL((step_spmv_long<double, int64_t>), g1, dim3(kNT), 0, stream, insts_dev, work_dev, n_work, remap, xcd_bounds);
                else hipLaunchKernelGGL((step_spmv_long<double, int32_t>), g1, dim3(kNT), 0, stream, insts_dev, work_dev, n_work, remap, xcd_bounds);
            } else {
                if (rp64) hipLaunchKernelGGL((step_spmv_long<float, int64_t>), g1, dim3(kNT), 0, stream, insts_dev, work_dev, n_work, remap, xcd_bounds);
                else hipLaunchKernelGGL((step_spmv_long<float, int32_t>), g1, dim3(kNT), 0, stream, insts_dev, work_dev, n_work, remap, xcd_bounds);
            }
            return hipGetLastError();
        }
        // the tiled step: quads through registers, or FP32 values straight into LDS
#define DRTS_SPMV1(VT, IT, RV, L) \
    hipLaunchKernelGGL((step_spmv<VT, IT, RV, L>), g1, dim3(RV), 0, stream, insts_dev, work_dev, n_work, remap, \
                       xcd_bounds, queue)
#define DRTS_SPMV(VT, IT, RV)                                           \
    do {                                                                \
        if (variant == DRTS_SPMV_LDS && sizeof(VT) == 4) DRTS_SPMV1(VT, IT, RV, 2); \
        else DRTS_SPMV1(VT, IT, RV, 0);                                 \
    } while (0)
        const int nt = rows_per_tile <= 64 ? 64 : (rows_per_tile <= 128 ? 128 : 256);
        if (value_f64) {
            if (rp64) {
                if (nt == 64) DRTS_SPMV(double, int64_t, 64);
                else if (nt == 128) DRTS_SPMV(double, int64_t, 128);
                else DRTS_SPMV(double, int64_t, 256);
            } else {
                if (nt == 64) DRTS_SPMV(double, int32_t, 64);
                else if (nt == 128) DRTS_SPMV(double, int32_t, 128);
                else DRTS_SPMV(double, int32_t, 256);
            }
        } else {
            if (rp64) {
                if (nt == 64) DRTS_SPMV(float, int64_t, 64);
                else if (nt == 128) DRTS_SPMV(float, int64_t, 128);
                else DRTS_SPMV(float, int64_t, 256);
            } else {
                if (nt == 64) DRTS_SPMV(float, int32_t, 64);
                else if (nt == 128) DRTS_SPMV(float, int32_t, 128);
                else DRTS_SPMV(float, int32_t, 256);
            }
        }
#undef DRTS_SPMV1
#undef DRTS_SPMV
    }
    return hipGetLastError();
}

hipError_t launch_structured(const StructArgs &sa, const StepInst *insts_dev, const WorkItem *work_dev,
                             int64_t n_work, int value_f64, int mode, int grid, int xcd_remap,
                             const int64_t *xcd_bounds, hipStream_t stream)
{
    if (n_work <= 0 && sa.n_xrows <= 0) return hipSuccess;
    // the tiles must be the ones the mode's kernel takes (the host chooses
    // both): modes 1 and 2 run the direction-major kernel (at most
    // kStructMatLds materials), modes 0 and 3 the gather kernel
    const bool dm_mode = !value_f64 && (mode == 1 || mode == 2);
    if (dm_mode ? (sa.seg_len != kStructDmSeg || sa.n_mat > kStructMatLds) : sa.seg_len != kStructSegLen)
        return hipErrorInvalidValue;
    const size_t dm = (size_t)(3 * (kStructDmSeg + 2) + kStructDmSeg) * kDirs * sizeof(float);
    // workgroups past the work list would only start and exit; a multiple of
    // the XCD count keeps the per-XCD walk available
    const dim3 g((unsigned)std::min<int64_t>(grid, std::max<int64_t>((n_work + kXcds - 1) / kXcds * kXcds, kXcds))),
        b(256);
    if (n_work > 0) {
        if (value_f64) {
            hipLaunchKernelGGL((step_struct<double, 0>), g, b, 0, stream, sa, insts_dev, work_dev, n_work,
                               xcd_remap & 1, xcd_bounds);
        } else if (mode == 0) {
            hipLaunchKernelGGL((step_struct<float, 0>), g, b, 0, stream, sa, insts_dev, work_dev, n_work,
                               xcd_remap & 1, xcd_bounds);
        } else if (mode == 1) {
            hipLaunchKernelGGL((step_struct_dm<1, false>), g, b, dm, stream, sa, nullptr, insts_dev, work_dev, n_work, xcd_remap & 1,
                               xcd_bounds);
        } else if (mode == 2) {
            hipLaunchKernelGGL((step_struct_dm<2, false>), g, b, dm, stream, sa, nullptr, insts_dev, work_dev, n_work, xcd_remap & 1,
                               xcd_bounds);
        } else {
            hipLaunchKernelGGL((step_struct<float, 3>), g, b, 0, stream, sa, insts_dev, work_dev, n_work,
                               xcd_remap & 1, xcd_bounds);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (sa.n_xrows > 0) {
        const int64_t items = (sa.n_xrows + kStructXRows - 1) / kStructXRows;
        const dim3 gx((unsigned)min(items, (int64_t)grid));
        if (value_f64)
            hipLaunchKernelGGL((step_struct_x<double, 0, false>), gx, b, 0, stream, sa, nullptr, insts_dev, nullptr, 0);
        else if (mode == 0 || mode == 1)
            hipLaunchKernelGGL((step_struct_x<float, 0, false>), gx, b, 0, stream, sa, nullptr, insts_dev, nullptr, 0);
        else
            hipLaunchKernelGGL((step_struct_x<float, 2, false>), gx, b, 0, stream, sa, nullptr, insts_dev, nullptr, 0);
    }
    return hipGetLastError();
}

hipError_t launch_structured_batch(const StructArgs *sas_dev, const StepInst *insts_dev, const WorkItem *work_dev,
                                   int64_t n_work, const WorkItem *xwork_dev, int64_t n_xwork, int mode, int grid,
                                   hipStream_t stream)
{
    if (mode != 1 && mode != 2) return hipErrorInvalidValue;
    const size_t dm = (size_t)(3 * (kStructDmSeg + 2) + kStructDmSeg) * kDirs * sizeof(float);
    const dim3 b(256);
    if (n_work > 0) {
        const dim3 g((unsigned)std::min<int64_t>(grid, std::max<int64_t>((n_work + kXcds - 1) / kXcds * kXcds, kXcds)));
        if (mode == 1)
            hipLaunchKernelGGL((step_struct_dm<1, true>), g, b, dm, stream, StructArgs{}, sas_dev, insts_dev, work_dev,
                               n_work, 0, nullptr);
        else
            hipLaunchKernelGGL((step_struct_dm<2, true>), g, b, dm, stream, StructArgs{}, sas_dev, insts_dev, work_dev,
                               n_work, 0, nullptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_xwork > 0) {
        const dim3 gx((unsigned)std::min<int64_t>(n_xwork, (int64_t)grid));
        if (mode == 1)
            hipLaunchKernelGGL((step_struct_x<float, 0, true>), gx, b, 0, stream, StructArgs{}, sas_dev, insts_dev,
                               xwork_dev, n_xwork);
        else
            hipLaunchKernelGGL((step_struct_x<float, 2, true>), gx, b, 0, stream, StructArgs{}, sas_dev, insts_dev,
                               xwork_dev, n_xwork);
    }
    return hipGetLastError();
}

hipError_t launch_structured_mm(const StructArgs &sa, const StepInst *insts_dev, const WorkItem *work_dev,
                                int64_t n_work, int mode, int grid, int n_det, hipStream_t stream)
{
    const dim3 b(256);
    (void)grid;
    if (n_work > 0) {
        const dim3 g((unsigned)sa.mm_push_grid);
        if (mode == 2)
            hipLaunchKernelGGL((step_struct_mm<2>), g, b, 0, stream, sa, insts_dev, work_dev, n_work);
        else
            hipLaunchKernelGGL((step_struct_mm<1>), g, b, 0, stream, sa, insts_dev, work_dev, n_work);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (sa.n_xrows > 0 || sa.n_zrows > 0) {
        const dim3 gx((unsigned)sa.mm_pull_grid);
        const size_t lds = (size_t)4 * n_det * 64 * sizeof(double);
        if (mode == 2)
            hipLaunchKernelGGL((step_struct_mm_x<2>), gx, b, lds, stream, sa, insts_dev);
        else
            hipLaunchKernelGGL((step_struct_mm_x<1>), gx, b, lds, stream, sa, insts_dev);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const StepInst *insts_dev, int n_inst, int n_rhs_max, int n_det_max, int32_t *queue,
                           hipStream_t stream)
{
    (void)n_det_max;
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_seg, dim3((unsigned)kFinSeg, (unsigned)n_inst, (unsigned)n_rhs_max), dim3(kNT), 0,
                       stream, insts_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_step, dim3((unsigned)n_inst, (unsigned)n_rhs_max), dim3(kNT), 0, stream, insts_dev,
                       queue);
    return hipGetLastError();
}

}  // namespace drts
