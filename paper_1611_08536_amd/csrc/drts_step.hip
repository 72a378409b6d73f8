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
#include "drts_internal.h"
#include "drts_step.h"

namespace drts {
namespace {

constexpr int kNT = 256;     // threads per workgroup
constexpr int kCap = 4096;   // matrix entries staged in LDS per pass
constexpr int kRowsMax = 256;
constexpr int kXcds = 8;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef int i4 __attribute__((ext_vector_type(4)));

template <typename VT> struct Quad;
template <> struct Quad<float> {
    f4 v;
    __device__ __forceinline__ void load(const float *p) { v = __builtin_nontemporal_load((const f4 *)p); }
    __device__ __forceinline__ float operator[](int j) const { return v[j]; }
};
template <> struct Quad<double> {
    d2 a, b;
    __device__ __forceinline__ void load(const double *p)
    {
        a = __builtin_nontemporal_load((const d2 *)p);
        b = __builtin_nontemporal_load((const d2 *)(p + 2));
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

__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
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
__device__ __forceinline__ Walk walk_of(int64_t n_work, int xcd_remap)
{
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (xcd_remap && G % kXcds == 0 && G >= kXcds) {
        const int64_t x = b % kXcds, local = b / kXcds, per = G / kXcds;
        const int64_t lo = x * n_work / kXcds, hi = (x + 1) * n_work / kXcds;
        return {lo + local, hi, per};
    }
    return {b, n_work, G};
}

// ---------------------------------------------------------------------------
// SpMV step (one right-hand side)
// ---------------------------------------------------------------------------
template <typename VT, typename IT>
__global__ void __launch_bounds__(kNT) step_spmv(const StepInst *__restrict__ insts,
                                                  const WorkItem *__restrict__ work, int64_t n_work,
                                                  int xcd_remap)
{
    constexpr int U = kCap / (4 * kNT);
    __shared__ VT s_prod[kCap];
    __shared__ IT s_rp[kRowsMax + 1];
    __shared__ VT s_y[kRowsMax];
    __shared__ double s_red[kNT];
    const int tid = threadIdx.x;
    const Walk wk = walk_of(n_work, xcd_remap);

    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        const int64_t t = I.t[0];
        if (t >= *I.t_end) continue;
        const Scale sc = step_scale(I, 0, t);
        const VT scale = (VT)ldexp(1.0, -sc.k);
        const IT *__restrict__ rp = (const IT *)I.row_ptr;
        const int32_t *__restrict__ col = I.col;
        const VT *__restrict__ val = (const VT *)I.val;
        const VT *__restrict__ x = (const VT *)((t & 1) ? I.buf1 : I.buf0);
        VT *__restrict__ y = (VT *)((t & 1) ? I.buf0 : I.buf1);
        const int R = I.rows_per_tile;

        double sN = 0.0, sE = 0.0, sA = 0.0, dsum = 0.0;
        VT mx = 0;
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int64_t tile1 = min(tile0 + (int64_t)I.tiles_per_chunk, I.n_tiles);
        for (int64_t tile = tile0; tile < tile1; ++tile) {
            const int64_t r0 = tile * R;
            const int nr = (int)min((int64_t)R, I.n_rows - r0);
            for (int i = tid; i <= nr; i += kNT) s_rp[i] = rp[r0 + i];
            __syncthreads();
            const IT b = s_rp[0], e = s_rp[nr];
            IT mylo = 0, myhi = 0;
            if (tid < nr) {
                mylo = s_rp[tid];
                myhi = s_rp[tid + 1];
            }
            VT acc = 0;
            for (IT a = b & ~(IT)3; a < e; a += kCap) {
                const IT cs = a < b ? b : a;
                const IT ce = (e - a < (IT)kCap) ? e : a + (IT)kCap;
                Quad<VT> qv[U];
                i4 qc[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const IT i = a + (IT)(4 * (tid + k * kNT));
                    if (i < ce) {
                        qc[k] = __builtin_nontemporal_load((const i4 *)(col + i));
                        qv[k].load(val + i);
                    }
                }
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const IT i = a + (IT)(4 * (tid + k * kNT));
                    if (i < ce) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const IT idx = i + j;
                            if (idx >= cs && idx < ce) s_prod[idx - a] = qv[k][j] * x[qc[k][j]];
                        }
                    }
                }
                __syncthreads();
                const IT lo = mylo > cs ? mylo : cs;
                const IT hi = myhi < ce ? myhi : ce;
                for (IT j = lo; j < hi; ++j) acc += s_prod[j - a];
                __syncthreads();
            }

            // epilogue: rescale, sources, store, FP64 totals
            if (tid < nr) {
                const int64_t r = r0 + tid;
                VT v = acc * scale;
                const int sb = I.src_tile[tile], se = I.src_tile[tile + 1];
                if (sb < se) {
                    int e2 = lower_bound_rows<IT>(I.src_row, sb, se, r);
                    double s = 0.0;
                    bool any = false;
                    for (; e2 < se && I.src_row[e2] == r; ++e2) {
                        s += I.src_w[e2] * I.amp[t * I.n_src + I.src_id[e2]];
                        any = true;
                    }
                    if (any) v += (VT)ldexp(s, -sc.En);
                }
                y[r] = v;
                s_y[tid] = v;
                if (r < I.n_states) {
                    sN += (double)v;
                    sA += I.absorb[I.mat[r / kDirs]] * (double)v;
                    mx = v > mx ? v : mx;
                } else {
                    sE += (double)v;
                }
            }
            const int db = I.det_tile[tile], de = I.det_tile[tile + 1];
            __syncthreads();
            if (db < de && tid < I.n_det) {
                for (int e2 = db; e2 < de; ++e2)
                    if (I.det_id[e2] == tid) dsum += I.det_F[e2] * (double)s_y[I.det_row[e2] - r0];
            }
        }
        // chunk partials, fixed-order tree reductions
        const int64_t nc = I.n_chunks, c = item.chunk;
        const double tN = block_sum(sN, s_red);
        const double tE = block_sum(sE, s_red);
        const double tA = block_sum(sA, s_red);
        const double tM = block_max((double)mx, s_red);
        if (tid == 0) {
            I.partials[kSlotN * nc + c] = tN;
            I.partials[kSlotEsc * nc + c] = tE;
            I.partials[kSlotAbs * nc + c] = tA;
            I.partials[kSlotMax * nc + c] = tM;
        }
        if (tid < I.n_det) I.partials[(int64_t)(kSlotDet + tid) * nc + c] = dsum;
    }
}

// ---------------------------------------------------------------------------
// SpMM step (n_rhs right-hand sides, FP32), lanes = right-hand sides
// ---------------------------------------------------------------------------
template <typename IT>
__global__ void __launch_bounds__(kNT) step_spmm(const StepInst *__restrict__ insts,
                                                  const WorkItem *__restrict__ work, int64_t n_work,
                                                  int xcd_remap)
{
    extern __shared__ double s_det[];   // [4 waves][n_det][64]
    __shared__ double s_w[4][4][64];     // per-wave totals for the fixed-order combine
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const Walk wk = walk_of(n_work, xcd_remap);

    for (int64_t wi = wk.begin; wi < wk.end; wi += wk.stride) {
        const WorkItem item = work[wi];
        const StepInst &I = insts[item.inst];
        const int64_t t = I.t[0];
        if (t >= *I.t_end) continue;
        const int nrhs = I.n_rhs, nd = I.n_det;
        const bool active = lane < nrhs;
        Scale sc{0, 0};
        if (active) sc = step_scale(I, lane, t);
        const float scale = ldexpf(1.0f, -sc.k);
        const IT *__restrict__ rp = (const IT *)I.row_ptr;
        const int32_t *__restrict__ col = I.col;
        const float *__restrict__ val = (const float *)I.val;
        const float *__restrict__ X = (const float *)((t & 1) ? I.buf1 : I.buf0);
        float *__restrict__ Y = (float *)((t & 1) ? I.buf0 : I.buf1);
        double *my_det = s_det + (int64_t)wave * nd * 64;
        for (int d = 0; d < nd; ++d) my_det[d * 64 + lane] = 0.0;

        double sN = 0.0, sE = 0.0, sA = 0.0;
        float mx = 0.0f;
        const int R = I.rows_per_tile;
        const int64_t tile0 = (int64_t)item.chunk * I.tiles_per_chunk;
        const int64_t tile1 = min(tile0 + (int64_t)I.tiles_per_chunk, I.n_tiles);
        for (int64_t tile = tile0; tile < tile1; ++tile) {
            const int64_t r0 = tile * R;
            const int nr = (int)min((int64_t)R, I.n_rows - r0);
            const int sb = I.src_tile[tile], se = I.src_tile[tile + 1];
            const int db = I.det_tile[tile], de = I.det_tile[tile + 1];
            for (int i = wave; i < nr; i += 4) {
                const int64_t r = r0 + i;
                const IT lo = rp[r], hi = rp[r + 1];
                float acc = 0.0f;
                IT j = lo;
                if (active) {
                    for (; j + 4 <= hi; j += 4) {
                        const int32_t c0 = col[j], c1 = col[j + 1], c2 = col[j + 2], c3 = col[j + 3];
                        const float v0 = val[j], v1 = val[j + 1], v2 = val[j + 2], v3 = val[j + 3];
                        const float x0 = X[(int64_t)c0 * nrhs + lane];
                        const float x1 = X[(int64_t)c1 * nrhs + lane];
                        const float x2 = X[(int64_t)c2 * nrhs + lane];
                        const float x3 = X[(int64_t)c3 * nrhs + lane];
                        acc += v0 * x0;
                        acc += v1 * x1;
                        acc += v2 * x2;
                        acc += v3 * x3;
                    }
                    for (; j < hi; ++j) acc += val[j] * X[(int64_t)col[j] * nrhs + lane];
                }
                float v = acc * scale;
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
                if (active) {
                    Y[r * nrhs + lane] = v;
                    if (r < I.n_states) {
                        sN += (double)v;
                        sA += I.absorb[I.mat[r / kDirs]] * (double)v;
                        mx = fmaxf(mx, v);
                    } else {
                        sE += (double)v;
                    }
                    if (db < de) {
                        int e2 = lower_bound_rows<IT>(I.det_row, db, de, r);
                        for (; e2 < de && I.det_row[e2] == r; ++e2)
                            my_det[I.det_id[e2] * 64 + lane] += I.det_F[e2] * (double)v;
                    }
                }
            }
        }
        s_w[0][wave][lane] = sN;
        s_w[1][wave][lane] = sE;
        s_w[2][wave][lane] = sA;
        s_w[3][wave][lane] = (double)mx;
        __syncthreads();
        const int64_t nc = I.n_chunks, c = item.chunk;
        if (wave == 0 && active) {
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
}

// ---------------------------------------------------------------------------
// finalize: fixed-order reduction of the chunk partials, series and control
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kNT) finalize_step(const StepInst *__restrict__ insts)
{
    __shared__ double red[kNT];
    const StepInst &I = insts[blockIdx.x];
    const int rhs = blockIdx.y;
    if (rhs >= I.n_rhs) return;
    const int64_t t = I.t[rhs];
    if (t >= *I.t_end) return;
    const int tid = threadIdx.x;
    const int64_t nc = I.n_chunks;
    const int nr = I.n_rhs;
    const Scale sc = step_scale(I, rhs, t);
    auto slot = [&](int kind) { return I.partials + ((int64_t)kind * nr + rhs) * nc; };
    double a = 0.0;
    const double *p = slot(kSlotN);
    for (int64_t c = tid; c < nc; c += kNT) a += p[c];
    const double N = block_sum(a, red);
    a = 0.0;
    p = slot(kSlotEsc);
    for (int64_t c = tid; c < nc; c += kNT) a += p[c];
    const double Esc = block_sum(a, red);
    a = 0.0;
    p = slot(kSlotAbs);
    for (int64_t c = tid; c < nc; c += kNT) a += p[c];
    const double Abs = block_sum(a, red);
    a = 0.0;
    p = slot(kSlotMax);
    for (int64_t c = tid; c < nc; c += kNT) a = fmax(a, p[c]);
    const double Mx = block_max(a, red);
    for (int d = 0; d < I.n_det; ++d) {
        a = 0.0;
        p = slot(kSlotDet + d);
        for (int64_t c = tid; c < nc; c += kNT) a += p[c];
        const double Dd = block_sum(a, red);
        if (tid == 0) I.ser_det[(t * I.n_det + d) * nr + rhs] = Dd;
    }
    if (tid == 0) {
        I.ser_tot[(t * 3 + 0) * nr + rhs] = N;
        I.ser_tot[(t * 3 + 1) * nr + rhs] = Esc;
        I.ser_tot[(t * 3 + 2) * nr + rhs] = I.abs_cur[rhs];
        I.ser_abs_exp[t * nr + rhs] = I.E[rhs];
        I.ser_exp[t * nr + rhs] = sc.En;
        I.abs_cur[rhs] = Abs;
        I.M[rhs] = Mx;
        I.E[rhs] = sc.En;
        I.t[rhs] = t + 1;
    }
}

}  // namespace

hipError_t launch_step(const StepInst *insts_dev, const WorkItem *work_dev, int64_t n_work, int n_inst,
                       int n_rhs_max, int value_f64, int rp64, int spmm, int grid, int xcd_remap,
                       int rows_per_tile, int n_det_max, hipStream_t stream)
{
    (void)n_inst;
    (void)n_rhs_max;
    (void)rows_per_tile;
    if (n_work <= 0) return hipSuccess;
    const dim3 g((unsigned)grid), b(kNT);
    if (spmm) {
        const size_t lds = (size_t)4 * n_det_max * 64 * sizeof(double);
        if (rp64)
            hipLaunchKernelGGL(step_spmm<int64_t>, g, b, lds, stream, insts_dev, work_dev, n_work, xcd_remap);
        else
            hipLaunchKernelGGL(step_spmm<int32_t>, g, b, lds, stream, insts_dev, work_dev, n_work, xcd_remap);
    } else if (value_f64) {
        if (rp64)
            hipLaunchKernelGGL((step_spmv<double, int64_t>), g, b, 0, stream, insts_dev, work_dev, n_work, xcd_remap);
        else
            hipLaunchKernelGGL((step_spmv<double, int32_t>), g, b, 0, stream, insts_dev, work_dev, n_work, xcd_remap);
    } else {
        if (rp64)
            hipLaunchKernelGGL((step_spmv<float, int64_t>), g, b, 0, stream, insts_dev, work_dev, n_work, xcd_remap);
        else
            hipLaunchKernelGGL((step_spmv<float, int32_t>), g, b, 0, stream, insts_dev, work_dev, n_work, xcd_remap);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const StepInst *insts_dev, int n_inst, int n_rhs_max, int n_det_max, hipStream_t stream)
{
    (void)n_det_max;
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_step, dim3((unsigned)n_inst, (unsigned)n_rhs_max), dim3(kNT), 0, stream, insts_dev);
    return hipGetLastError();
}

}  // namespace drts
