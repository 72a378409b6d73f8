// Device assembly of [A; L] in CSR form (Eq. (21)/(23) plus escape rows).
//
// Pull formulation, one thread per row.  Row (w, m') of a state receives
//   - the plain move of its upstream voxel u = w - e_m' (direction m' kept),
//     when u is inside the grid and has the same refractive index as w;
//   - every irregular move listed for it on the host (wall reflection,
//     Fresnel reflected or transmitted part), sorted by (voxel, direction).
// An escape row receives the one move (v, m) that leaves the grid.
// Each move (u, m, f) contributes f * C_q(u)[m][n] to column 26 u + n; moves
// of one voxel are summed per column in ascending m.  Exact zeros are not
// stored.  A count pass, an exclusive scan and a fill pass produce the CSR.
#include <hipcub/hipcub.hpp>

#include "drts_internal.h"

namespace drts {
namespace {

struct AsmArgs {
    int nx, ny, nz;
    int rounding;  // DRTS_ROUND_* (FP32 values only)
    int64_t n_states, n_rows, n_irr;
    const uint8_t *mat;
    const double *index;
    const double *blocks;  // [q][m][n]
    const int64_t *irr_row, *irr_vox;
    const int32_t *irr_dir;
    const double *irr_f;
    const uint32_t *irr_bits;
    const int64_t *escape_state;
};

__device__ inline uint64_t mix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// FP64 -> FP32 of a positive value: nearest, or the unbiased choice between
// the two float neighbours keyed on (row, col).
__device__ inline float to_f32(double a, int rounding, int64_t row, int64_t col)
{
    float f = (float)a;
    if (rounding == DRTS_ROUND_DITHER && (double)f != a) {
        const uint32_t bits = __float_as_uint(f);
        const float g = __uint_as_float((double)f < a ? bits + 1u : bits - 1u);
        const double p = fabs((double)f - a) / fabs((double)g - (double)f);
        const uint64_t key = ((uint64_t)row << 32) ^ (uint64_t)(uint32_t)col;
        const double u = (double)(mix64(key) >> 11) * 0x1p-53;
        if (u < p) f = g;
    }
    return f;
}

__device__ inline int64_t lower_bound64(const int64_t *a, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename VT> struct Store;
template <> struct Store<double> {
    __device__ static double cvt(double a, int, int64_t, int64_t) { return a; }
};
template <> struct Store<float> {
    __device__ static float cvt(double a, int rnd, int64_t r, int64_t c) { return to_f32(a, rnd, r, c); }
};

// Emits the merged entries of one voxel group: moves [k0, k1) of the irregular
// list (all with source voxel u) or, when single_dir >= 0, the one move
// (u, single_dir, 1.0).  Returns the number of nonzero entries.
template <bool FILL, typename VT>
__device__ int emit_group(const AsmArgs &a, int64_t row, int64_t u, int single_dir, int64_t k0, int64_t k1,
                          int32_t *col, VT *val, int64_t pos)
{
    const double *C = a.blocks + (int64_t)a.mat[u] * kDirs * kDirs;
    int cnt = 0;
    for (int n = 0; n < kDirs; ++n) {
        double v = 0.0;
        if (single_dir >= 0) {
            v = C[single_dir * kDirs + n];
        } else {
            for (int64_t k = k0; k < k1; ++k) {
                const double c = C[a.irr_dir[k] * kDirs + n];
                if (c != 0.0) v = v + a.irr_f[k] * c;
            }
        }
        if (v != 0.0) {
            if (FILL) {
                const int64_t cc = kDirs * u + n;
                col[pos + cnt] = (int32_t)cc;
                val[pos + cnt] = Store<VT>::cvt(v, a.rounding, row, cc);
            }
            ++cnt;
        }
    }
    return cnt;
}

template <bool FILL, typename VT, typename IT>
__global__ void __launch_bounds__(256) assemble_rows(AsmArgs a, int64_t *counts, const IT *row_ptr,
                                                      int32_t *col, VT *val)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_rows) return;
    int64_t pos = FILL ? (int64_t)row_ptr[r] : 0;
    int64_t total = 0;
    if (r >= a.n_states) {
        const int64_t s = a.escape_state[r - a.n_states];
        total = emit_group<FILL, VT>(a, r, s / kDirs, (int)(s % kDirs), 0, 0, col, val, pos);
    } else {
        const int64_t w = r / kDirs;
        const int mp = (int)(r % kDirs);
        const int x = (int)(w % a.nx), y = (int)((w / a.nx) % a.ny), z = (int)(w / ((int64_t)a.nx * a.ny));
        const int ux = x - dir_dx(mp), uy = y - dir_dy(mp), uz = z - dir_dz(mp);
        int64_t ureg = -1;
        if (ux >= 0 && ux < a.nx && uy >= 0 && uy < a.ny && uz >= 0 && uz < a.nz) {
            const int64_t u = ux + (int64_t)a.nx * (uy + (int64_t)a.ny * uz);
            if (a.index[a.mat[u]] == a.index[a.mat[w]]) ureg = u;
        }
        int64_t k = 0, kend = 0;
        if (a.n_irr > 0 && ((a.irr_bits[r >> 5] >> (r & 31)) & 1u)) {
            k = lower_bound64(a.irr_row, a.n_irr, r);
            kend = k;
            while (kend < a.n_irr && a.irr_row[kend] == r) ++kend;
        }
        // walk the irregular groups in voxel order, placing the plain move
        while (k < kend || ureg >= 0) {
            const int64_t ug = k < kend ? a.irr_vox[k] : INT64_MAX;
            if (ureg >= 0 && ureg < ug) {
                total += emit_group<FILL, VT>(a, r, ureg, mp, 0, 0, col, val, pos + total);
                ureg = -1;
                continue;
            }
            int64_t k1 = k;
            while (k1 < kend && a.irr_vox[k1] == ug) ++k1;
            total += emit_group<FILL, VT>(a, r, ug, -1, k, k1, col, val, pos + total);
            k = k1;
        }
    }
    if (!FILL) counts[r] = total;
}

// ---- Lebedev-86 media (Sec. 3, Eq. (18)-(21)) -------------------------------------
//
// Pull formulation, one thread per row.  State row (j, m) walks direction m's
// list of (offset, n, weight) -- descending offsets, ascending n, so that the
// source voxels i = j - offset and the columns 86 i + n come out ascending --
// and takes w C_q(i)[m][n] from every source voxel inside the grid.  Escape row
// (v, m) takes, per direction n, the scan-order sum of the weights of the
// pair's offsets that leave the grid, times C_q(v)[m][n].  Each entry is one
// product (or one weight sum times one coefficient): the same values the push
// assembly of the method gives.
struct LebArgs {
    int nx, ny, nz;
    int rounding;
    int64_t n_states, n_rows;
    const uint8_t *mat;
    const double *blocks;          // [q][86][86]
    const int64_t *pair_ptr;       // [86*86 + 1]
    const uint32_t *pair_key;
    const double *pair_w;
    const int64_t *arr_ptr;        // [86 + 1]
    const uint32_t *arr_key;
    const double *arr_w;
    const int64_t *escape_state;
};

constexpr int kLebDirs = 86;

template <bool FILL, typename VT, typename IT>
__global__ void __launch_bounds__(256) assemble_leb_rows(LebArgs a, int64_t *counts, const IT *row_ptr,
                                                          int32_t *col, VT *val)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_rows) return;
    int64_t pos = FILL ? (int64_t)row_ptr[r] : 0;
    int64_t cnt = 0;
    if (r < a.n_states) {
        const int m = (int)(r % kLebDirs);
        const int64_t j = r / kLebDirs;
        const int x = (int)(j % a.nx), y = (int)((j / a.nx) % a.ny), z = (int)(j / ((int64_t)a.nx * a.ny));
        for (int64_t e = a.arr_ptr[m]; e < a.arr_ptr[m + 1]; ++e) {
            const uint32_t k = a.arr_key[e];
            const int ix = x - off_dx(k), iy = y - off_dy(k), iz = z - off_dz(k);
            if (ix < 0 || ix >= a.nx || iy < 0 || iy >= a.ny || iz < 0 || iz >= a.nz) continue;
            const int64_t i = ix + (int64_t)a.nx * (iy + (int64_t)a.ny * iz);
            const int n = off_n(k);
            const double c = a.blocks[((int64_t)a.mat[i] * kLebDirs + m) * kLebDirs + n];
            if (c == 0.0) continue;
            const double v = a.arr_w[e] * c;
            if (v == 0.0) continue;
            if (FILL) {
                const int64_t cc = kLebDirs * i + n;
                col[pos + cnt] = (int32_t)cc;
                val[pos + cnt] = Store<VT>::cvt(v, a.rounding, r, cc);
            }
            ++cnt;
        }
    } else {
        const int64_t s = a.escape_state[r - a.n_states];
        const int m = (int)(s % kLebDirs);
        const int64_t v = s / kLebDirs;
        const int x = (int)(v % a.nx), y = (int)((v / a.nx) % a.ny), z = (int)(v / ((int64_t)a.nx * a.ny));
        const double *C = a.blocks + ((int64_t)a.mat[v] * kLebDirs + m) * kLebDirs;
        for (int n = 0; n < kLebDirs; ++n) {
            const double c = C[n];
            if (c == 0.0) continue;
            double esc = 0.0;
            bool any = false;
            for (int64_t e = a.pair_ptr[m * kLebDirs + n]; e < a.pair_ptr[m * kLebDirs + n + 1]; ++e) {
                const uint32_t k = a.pair_key[e];
                const int ux = x + off_dx(k), uy = y + off_dy(k), uz = z + off_dz(k);
                if (ux < 0 || ux >= a.nx || uy < 0 || uy >= a.ny || uz < 0 || uz >= a.nz) {
                    esc += a.pair_w[e];
                    any = true;
                }
            }
            const double vv = esc * c;
            if (!any || vv == 0.0) continue;
            if (FILL) {
                const int64_t cc = kLebDirs * v + n;
                col[pos + cnt] = (int32_t)cc;
                val[pos + cnt] = Store<VT>::cvt(vv, a.rounding, r, cc);
            }
            ++cnt;
        }
    }
    if (!FILL) counts[r] = cnt;
}

template <typename IT>
__global__ void narrow_row_ptr(const int64_t *in, IT *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (IT)in[i];
}

template <typename T> int upload(Device &dev, Buffer &b, const std::vector<T> &h)
{
    const size_t bytes = std::max<size_t>(h.size() * sizeof(T), 16);
    int rc = b.allocate(&dev, bytes);
    if (rc) return rc;
    if (!h.empty()) DRTS_HIP(hipMemcpyAsync(b.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, dev.stream));
    return DRTS_OK;
}

template <typename VT>
int fill_values(Matrix *A, const AsmArgs &args, const LebArgs *leb, Buffer &rp64)
{
    Device &dev = A->dev;
    const int64_t R = args.n_rows;
    const unsigned blocks = (unsigned)((R + 255) / 256);
    const size_t pad = 4;
    int rc = A->col.allocate(&dev, (A->nnz + pad) * sizeof(int32_t));
    if (!rc) rc = A->val.allocate(&dev, (A->nnz + pad) * sizeof(VT));
    if (rc) return rc;
    DRTS_HIP(hipMemsetAsync(A->col.as<int32_t>() + A->nnz, 0, pad * sizeof(int32_t), dev.stream));
    DRTS_HIP(hipMemsetAsync(A->val.as<VT>() + A->nnz, 0, pad * sizeof(VT), dev.stream));
    if (leb && A->rp64) {
        hipLaunchKernelGGL((assemble_leb_rows<true, VT, int64_t>), dim3(blocks), dim3(256), 0, dev.stream, *leb,
                           (int64_t *)nullptr, A->row_ptr.as<int64_t>(), A->col.as<int32_t>(), A->val.as<VT>());
    } else if (leb) {
        hipLaunchKernelGGL((assemble_leb_rows<true, VT, int32_t>), dim3(blocks), dim3(256), 0, dev.stream, *leb,
                           (int64_t *)nullptr, A->row_ptr.as<int32_t>(), A->col.as<int32_t>(), A->val.as<VT>());
    } else if (A->rp64) {
        hipLaunchKernelGGL((assemble_rows<true, VT, int64_t>), dim3(blocks), dim3(256), 0, dev.stream, args,
                           (int64_t *)nullptr, A->row_ptr.as<int64_t>(), A->col.as<int32_t>(), A->val.as<VT>());
    } else {
        hipLaunchKernelGGL((assemble_rows<true, VT, int32_t>), dim3(blocks), dim3(256), 0, dev.stream, args,
                           (int64_t *)nullptr, A->row_ptr.as<int32_t>(), A->col.as<int32_t>(), A->val.as<VT>());
    }
    DRTS_HIP(hipGetLastError());
    (void)rp64;
    return DRTS_OK;
}

}  // namespace

int assemble_on_device(Matrix *A, bool with_csr)
{
    Device &dev = A->dev;
    Model &M = A->model;
    int rc;
    if ((rc = upload(dev, A->mat_of_voxel, M.mat_of_voxel))) return rc;
    if ((rc = upload(dev, A->index, M.index))) return rc;
    if ((rc = upload(dev, A->absorb, M.absorb))) return rc;
    if ((rc = upload(dev, A->blocks64, M.blocks))) return rc;
    {
        // nearest FP32 value of every block entry
        std::vector<float> hi(M.blocks.size());
        for (size_t i = 0; i < M.blocks.size(); ++i) hi[i] = (float)M.blocks[i];
        if ((rc = upload(dev, A->blocks32, hi))) return rc;
    }
    if ((rc = upload(dev, A->irr_row, M.irr_row))) return rc;
    if ((rc = upload(dev, A->irr_vox, M.irr_vox))) return rc;
    if ((rc = upload(dev, A->irr_dir, M.irr_dir))) return rc;
    if ((rc = upload(dev, A->irr_f, M.irr_f))) return rc;
    if ((rc = upload(dev, A->escape_state, M.escape_state))) return rc;
    {
        std::vector<uint32_t> bits((size_t)((M.n_states + 31) / 32), 0u);
        for (int64_t r : M.irr_row) bits[(size_t)(r >> 5)] |= 1u << (r & 31);
        if ((rc = upload(dev, A->irr_bits, bits))) return rc;
    }

    AsmArgs args;
    args.nx = M.nx;
    args.ny = M.ny;
    args.nz = M.nz;
    args.rounding = M.rounding;
    args.n_states = M.n_states;
    args.n_rows = M.n_rows;
    args.n_irr = (int64_t)M.irr_row.size();
    args.mat = A->mat_of_voxel.as<uint8_t>();
    args.index = A->index.as<double>();
    args.blocks = A->blocks64.as<double>();
    args.irr_row = A->irr_row.as<int64_t>();
    args.irr_vox = A->irr_vox.as<int64_t>();
    args.irr_dir = A->irr_dir.as<int32_t>();
    args.irr_f = A->irr_f.as<double>();
    args.irr_bits = A->irr_bits.as<uint32_t>();
    args.escape_state = A->escape_state.as<int64_t>();

    LebArgs leb{};
    const bool is_leb = M.n_dir != kDirs;
    if (is_leb) {
        if ((rc = upload(dev, A->pair_ptr, M.pair_ptr))) return rc;
        if ((rc = upload(dev, A->pair_key, M.pair_key))) return rc;
        if ((rc = upload(dev, A->pair_w, M.pair_w))) return rc;
        if ((rc = upload(dev, A->arr_ptr, M.arr_ptr))) return rc;
        if ((rc = upload(dev, A->arr_key, M.arr_key))) return rc;
        if ((rc = upload(dev, A->arr_w, M.arr_w))) return rc;
        leb.nx = M.nx;
        leb.ny = M.ny;
        leb.nz = M.nz;
        leb.rounding = M.rounding;
        leb.n_states = M.n_states;
        leb.n_rows = M.n_rows;
        leb.mat = A->mat_of_voxel.as<uint8_t>();
        leb.blocks = A->blocks64.as<double>();
        leb.pair_ptr = A->pair_ptr.as<int64_t>();
        leb.pair_key = A->pair_key.as<uint32_t>();
        leb.pair_w = A->pair_w.as<double>();
        leb.arr_ptr = A->arr_ptr.as<int64_t>();
        leb.arr_key = A->arr_key.as<uint32_t>();
        leb.arr_w = A->arr_w.as<double>();
        leb.escape_state = A->escape_state.as<int64_t>();
    }

    const int64_t R = M.n_rows;
    Buffer counts, rp64, tmp;
    if ((rc = counts.allocate(&dev, (R + 1) * sizeof(int64_t)))) return rc;
    if ((rc = rp64.allocate(&dev, (R + 1) * sizeof(int64_t)))) return rc;
    DRTS_HIP(hipMemsetAsync(counts.as<int64_t>() + R, 0, sizeof(int64_t), dev.stream));
    const unsigned blocks = (unsigned)((R + 255) / 256);
    if (is_leb)
        hipLaunchKernelGGL((assemble_leb_rows<false, double, int64_t>), dim3(blocks), dim3(256), 0, dev.stream, leb,
                           counts.as<int64_t>(), (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr);
    else
        hipLaunchKernelGGL((assemble_rows<false, double, int64_t>), dim3(blocks), dim3(256), 0, dev.stream, args,
                           counts.as<int64_t>(), (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr);
    DRTS_HIP(hipGetLastError());

    size_t tmp_bytes = 0;
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, counts.as<int64_t>(), rp64.as<int64_t>(),
                                             (size_t)(R + 1), dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tmp_bytes, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.ptr, tmp_bytes, counts.as<int64_t>(), rp64.as<int64_t>(),
                                             (size_t)(R + 1), dev.stream));
    int64_t nnz = 0;
    DRTS_HIP(hipMemcpyAsync(&nnz, rp64.as<int64_t>() + R, sizeof(int64_t), hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    tmp.reset();
    counts.reset();
    A->nnz = nnz;
    A->rp64 = nnz > (int64_t)INT32_MAX - 8;
    if (!with_csr) {
        A->has_csr = false;
        return DRTS_OK;
    }
    if (A->rp64) {
        A->row_ptr.dev = rp64.dev;
        A->row_ptr.ptr = rp64.ptr;
        A->row_ptr.bytes = rp64.bytes;
        rp64.ptr = nullptr;
        rp64.bytes = 0;
    } else {
        if ((rc = A->row_ptr.allocate(&dev, (R + 1) * sizeof(int32_t)))) return rc;
        hipLaunchKernelGGL(narrow_row_ptr<int32_t>, dim3((unsigned)((R + 1 + 255) / 256)), dim3(256), 0,
                           dev.stream, rp64.as<int64_t>(), A->row_ptr.as<int32_t>(), R + 1);
        DRTS_HIP(hipGetLastError());
    }
    rc = (M.value_type == DRTS_F64) ? fill_values<double>(A, args, is_leb ? &leb : nullptr, rp64)
                                    : fill_values<float>(A, args, is_leb ? &leb : nullptr, rp64);
    if (rc) return rc;
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    return DRTS_OK;
}

}  // namespace drts
