// Row groups of an assembled [A; L]: rows whose column lists are equal.  In a
// lattice matrix the rows that pull from one source voxel (one per direction,
// state or escape row) all hold that voxel's whole state as their columns;
// the many-rhs step gathers such a group's right-hand-side rows once and
// forms every member from them.
//
// Built on the device on first use by a many-rhs solver: each row gets the
// key (first column, length) (empty rows sort last), a stable radix sort of
// (key, row) puts candidate rows next to each other in ascending row order,
// a row starts a new group unless its key and whole column list equal its
// predecessor's, and a scan numbers the groups.  Groups of more than
// kGroupMax rows are split on the host.  When the rows group (at least two a
// group on average) the values are copied in group order -- every member's
// entries in turn, so a group's values are one contiguous block -- with each
// member's row and material beside them: the step then reads every array it
// needs of a group contiguously.
#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "drts_internal.h"
#include "drts_step.h"

namespace drts {
namespace {

template <typename IT>
__global__ void __launch_bounds__(256) group_keys(const IT *rp, const int32_t *col, int64_t n_rows, uint64_t *key,
                                                  int32_t *row)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t lo = (int64_t)rp[r], hi = (int64_t)rp[r + 1];
    key[r] = hi > lo ? ((uint64_t)(uint32_t)col[lo] << 32) | (uint64_t)(hi - lo) : ~0ull;
    row[r] = (int32_t)r;
}

template <typename IT>
__global__ void __launch_bounds__(256) group_starts(const uint64_t *key, const int32_t *row, const IT *rp,
                                                    const int32_t *col, int64_t n, int32_t *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t f = 1;
    if (i > 0 && key[i] == key[i - 1]) {
        const int64_t a = (int64_t)rp[row[i]], b = (int64_t)rp[row[i - 1]];
        const int64_t len = (int64_t)rp[row[i] + 1] - a;
        f = 0;
        for (int64_t k = 0; k < len; ++k) {
            if (col[a + k] != col[b + k]) {
                f = 1;
                break;
            }
        }
    }
    flag[i] = f;
}

// member i (sorted order): its entry count and the material of its voxel
template <typename IT>
__global__ void __launch_bounds__(256) member_info(const int32_t *grp_row, const IT *rp, const uint8_t *mat,
                                                   int64_t n, int64_t n_states, uint64_t vox_mul, int64_t *len,
                                                   uint8_t *gmat)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = grp_row[i];
    len[i] = (int64_t)rp[r + 1] - (int64_t)rp[r];
    gmat[i] = r < n_states ? mat[(int64_t)__umul64hi((uint64_t)r, vox_mul)] : (uint8_t)0;
}

// values in group order: member i's entries at moff[i] onwards
template <typename IT>
__global__ void __launch_bounds__(256) member_values(const int32_t *grp_row, const IT *rp, const float *val,
                                                     const int64_t *moff, int64_t n, float *gval)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = grp_row[i], lo = (int64_t)rp[r], hi = (int64_t)rp[r + 1], o = moff[i];
    for (int64_t k = lo; k < hi; ++k) gval[o + (k - lo)] = val[k];
}

// per group: offset of its values, of its leader's columns, entries a row
template <typename IT>
__global__ void __launch_bounds__(256) group_offsets(const int32_t *grp_ptr, const int32_t *grp_row, const IT *rp,
                                                     const int64_t *moff, int64_t n_groups, int64_t *voff,
                                                     int64_t *coff, int32_t *len)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const int64_t r = grp_row[grp_ptr[g]];
    voff[g] = moff[grp_ptr[g]];
    coff[g] = (int64_t)rp[r];
    len[g] = (int32_t)((int64_t)rp[r + 1] - (int64_t)rp[r]);
}

__global__ void __launch_bounds__(256) group_scatter(const int32_t *flag, const int32_t *pos, int64_t n,
                                                     int32_t *grp_ptr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) grp_ptr[pos[i]] = (int32_t)i;
}

template <typename IT>
int build_groups(Matrix &A)
{
    Device &dev = A.dev;
    const int64_t R = A.model.n_rows;
    const IT *rp = A.row_ptr.as<IT>();
    const int32_t *col = A.col.as<int32_t>();
    Buffer key, key_s, row, flag, pos, tmp, gp;
    int rc;
    if ((rc = key.allocate(&dev, R * sizeof(uint64_t)))) return rc;
    if ((rc = key_s.allocate(&dev, R * sizeof(uint64_t)))) return rc;
    if ((rc = row.allocate(&dev, R * sizeof(int32_t)))) return rc;
    if ((rc = A.grp_row.allocate(&dev, R * sizeof(int32_t)))) return rc;
    const unsigned blocks = (unsigned)((R + 255) / 256);
    hipLaunchKernelGGL(group_keys<IT>, dim3(blocks), dim3(256), 0, dev.stream, rp, col, R, key.as<uint64_t>(),
                       row.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    size_t tb = 0, tb2 = 0;
    DRTS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key.as<uint64_t>(), key_s.as<uint64_t>(),
                                                row.as<int32_t>(), A.grp_row.as<int32_t>(), (int)R, 0, 64,
                                                dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tb, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.ptr, tb, key.as<uint64_t>(), key_s.as<uint64_t>(),
                                                row.as<int32_t>(), A.grp_row.as<int32_t>(), (int)R, 0, 64,
                                                dev.stream));
    tmp.reset();
    key.reset();
    row.reset();
    if ((rc = flag.allocate(&dev, R * sizeof(int32_t)))) return rc;
    if ((rc = pos.allocate(&dev, R * sizeof(int32_t)))) return rc;
    hipLaunchKernelGGL(group_starts<IT>, dim3(blocks), dim3(256), 0, dev.stream, key_s.as<uint64_t>(),
                       A.grp_row.as<int32_t>(), rp, col, R, flag.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, flag.as<int32_t>(), pos.as<int32_t>(), (int)R,
                                             dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tb2, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.ptr, tb2, flag.as<int32_t>(), pos.as<int32_t>(), (int)R,
                                             dev.stream));
    int32_t last[2] = {0, 0};
    DRTS_HIP(hipMemcpyAsync(&last[0], pos.as<int32_t>() + R - 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                            dev.stream));
    DRTS_HIP(hipMemcpyAsync(&last[1], flag.as<int32_t>() + R - 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                            dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    const int64_t n_groups = (int64_t)last[0] + last[1];
    if ((rc = gp.allocate(&dev, (n_groups + 1) * sizeof(int32_t)))) return rc;
    hipLaunchKernelGGL(group_scatter, dim3(blocks), dim3(256), 0, dev.stream, flag.as<int32_t>(),
                       pos.as<int32_t>(), R, gp.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    // group starts on the host: split groups of more than kGroupMax rows
    std::vector<int32_t> h((size_t)n_groups + 1);
    DRTS_HIP(hipMemcpyAsync(h.data(), gp.ptr, (size_t)n_groups * sizeof(int32_t), hipMemcpyDeviceToHost,
                            dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    h[(size_t)n_groups] = (int32_t)R;
    std::vector<int32_t> out;
    out.reserve(h.size());
    for (int64_t g = 0; g < n_groups; ++g)
        for (int64_t s = h[(size_t)g]; s < h[(size_t)g + 1]; s += kGroupMax) out.push_back((int32_t)s);
    out.push_back((int32_t)R);
    const int64_t G = (int64_t)out.size() - 1;
    flag.reset();
    pos.reset();
    gp.reset();
    key_s.reset();
    tmp.reset();
    if (R < 2 * G) {
        // the rows do not group: the row-by-row step serves this matrix
        A.grp_row.reset();
        A.n_groups = 0;
        return DRTS_OK;
    }
    if ((rc = A.grp_ptr.allocate(&dev, out.size() * sizeof(int32_t)))) return rc;
    DRTS_HIP(hipMemcpyAsync(A.grp_ptr.ptr, out.data(), out.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                            dev.stream));
    // members' entry counts and materials, their value offsets (a scan), the
    // values in group order and the per-group offsets
    Buffer len, moff;
    if ((rc = len.allocate(&dev, R * sizeof(int64_t)))) return rc;
    if ((rc = moff.allocate(&dev, R * sizeof(int64_t)))) return rc;
    if ((rc = A.grp_mat.allocate(&dev, R))) return rc;
    hipLaunchKernelGGL(member_info<IT>, dim3(blocks), dim3(256), 0, dev.stream, A.grp_row.as<int32_t>(), rp,
                       A.mat_of_voxel.as<uint8_t>(), R, A.model.n_states, vox_mul_of(A.model.n_dir),
                       len.as<int64_t>(), A.grp_mat.as<uint8_t>());
    DRTS_HIP(hipGetLastError());
    size_t tb3 = 0;
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb3, len.as<int64_t>(), moff.as<int64_t>(), (int)R,
                                             dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tb3, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.ptr, tb3, len.as<int64_t>(), moff.as<int64_t>(), (int)R,
                                             dev.stream));
    tmp.reset();
    len.reset();
    // (the same padding after the last entry as the CSR values)
    if ((rc = A.grp_val.allocate(&dev, A.val.bytes))) return rc;
    DRTS_HIP(hipMemsetAsync(A.grp_val.ptr, 0, A.val.bytes, dev.stream));
    hipLaunchKernelGGL(member_values<IT>, dim3(blocks), dim3(256), 0, dev.stream, A.grp_row.as<int32_t>(), rp,
                       A.val.as<float>(), moff.as<int64_t>(), R, A.grp_val.as<float>());
    DRTS_HIP(hipGetLastError());
    if ((rc = A.grp_voff.allocate(&dev, G * sizeof(int64_t)))) return rc;
    if ((rc = A.grp_coff.allocate(&dev, G * sizeof(int64_t)))) return rc;
    if ((rc = A.grp_len.allocate(&dev, G * sizeof(int32_t)))) return rc;
    hipLaunchKernelGGL(group_offsets<IT>, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, dev.stream,
                       A.grp_ptr.as<int32_t>(), A.grp_row.as<int32_t>(), rp, moff.as<int64_t>(), G,
                       A.grp_voff.as<int64_t>(), A.grp_coff.as<int64_t>(), A.grp_len.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    A.n_groups = G;
    return DRTS_OK;
}

}  // namespace

int row_groups(const Matrix &Ac)
{
    // the groups are a property of the matrix, computed once and kept with it
    Matrix &A = const_cast<Matrix &>(Ac);
    if (A.n_groups >= 0) return DRTS_OK;
    const int64_t R = A.model.n_rows;
    if (!A.has_csr || R <= 0 || R >= INT32_MAX || A.model.value_type != DRTS_F32) {
        A.n_groups = 0;
        return DRTS_OK;
    }
    const int rc = A.rp64 ? build_groups<int64_t>(A) : build_groups<int32_t>(A);
    if (rc) {
        Buffer *b[] = {&A.grp_ptr, &A.grp_row, &A.grp_mat, &A.grp_val, &A.grp_voff, &A.grp_coff, &A.grp_len};
        for (Buffer *x : b) x->reset();
        A.n_groups = -1;
    }
    return rc;
}

}  // namespace drts
