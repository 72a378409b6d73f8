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
// group on average) the values are copied in group order -- a group's values
// one contiguous block, column-major (entry k of every member, then entry
// k+1) -- with each member's row and material beside them: the steps then
// read every array they need of a group contiguously, and the members' k-th
// entries with one coalesced load.
#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

#include <cstring>

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

// per group its descriptor: members, offset of its values (the first
// member's offset in the scan of entry counts), its leader's columns and
// whether they are one run
template <typename IT>
__global__ void __launch_bounds__(256) group_descs(const int32_t *grp_ptr, const int32_t *grp_row, const IT *rp,
                                                   const int32_t *col, const int64_t *moff, int64_t n_groups,
                                                   GroupDesc *desc)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const int64_t r = grp_row[grp_ptr[g]];
    const int64_t lo = (int64_t)rp[r], n = (int64_t)rp[r + 1] - lo;
    GroupDesc D;
    D.voff = moff[grp_ptr[g]];
    D.coff = lo;
    D.m0 = grp_ptr[g];
    D.nm = grp_ptr[g + 1] - grp_ptr[g];
    D.n = (int32_t)n;
    D.cstart = n > 0 ? col[lo] : -1;
    for (int64_t k = 1; k < n && D.cstart >= 0; ++k)
        if (col[lo + k] != col[lo] + k) D.cstart = -1;
    desc[g] = D;
}

// values in group order, column-major within a group: entry k of member j of
// group g at voff + k * nm + j
template <typename IT>
__global__ void __launch_bounds__(256) group_values(const GroupDesc *desc, const int32_t *grp_row, const IT *rp,
                                                    const float *val, int64_t n_groups, float *gval)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const GroupDesc D = desc[g];
    for (int j = 0; j < D.nm; ++j) {
        const int64_t lo = (int64_t)rp[grp_row[D.m0 + j]];
        for (int k = 0; k < D.n; ++k) gval[D.voff + (int64_t)k * D.nm + j] = val[lo + k];
    }
}

// bit g: a member of group g is in the ascending row list rows[0 .. n)
__global__ void __launch_bounds__(256) group_flag_bits(const GroupDesc *desc, const int32_t *grp_row,
                                                       int64_t n_groups, const int64_t *rows, int64_t n,
                                                       uint32_t *bits)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one word of 32 groups
    if (w * 32 >= n_groups) return;
    uint32_t word = 0;
    for (int b = 0; b < 32 && w * 32 + b < n_groups; ++b) {
        const GroupDesc D = desc[w * 32 + b];
        for (int j = 0; j < D.nm; ++j) {
            const int64_t r = grp_row[D.m0 + j];
            int64_t lo = 0, hi = n;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (rows[mid] < r) lo = mid + 1;
                else hi = mid;
            }
            if (lo < n && rows[lo] == r) word |= 1u << b;
        }
    }
    bits[w] = word;
}

// Per group its kind -- fast (a full lattice row: kSpmmUnroll columns that
// are one run), two-voxel (kVox2Len columns in two runs of kVox2Run: a
// voxel's states and another voxel's) or other -- and per member whether it
// is a two-voxel row or another group's row; the entries of the other groups'
// members (an integer count: the order of the additions does not matter).
__global__ void __launch_bounds__(256) group_kinds(const GroupDesc *desc, const int32_t *col, int64_t n_groups,
                                                   uint8_t *fast, uint8_t *member_vox2, uint8_t *member_slow,
                                                   unsigned long long *slow_entries)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const GroupDesc D = desc[g];
    const bool f = D.n == kSpmmUnrollHost && D.cstart >= 0;
    bool v2 = false;
    if (!f && D.n == kVox2Len) {
        const int32_t a = col[D.coff], b = col[D.coff + kVox2Run];
        v2 = true;
        for (int k = 1; k < kVox2Run && v2; ++k)
            v2 = col[D.coff + k] == a + k && col[D.coff + kVox2Run + k] == b + k;
    }
    fast[g] = f ? 1 : 0;
    for (int j = 0; j < D.nm; ++j) {
        member_vox2[D.m0 + j] = v2 ? 1 : 0;
        member_slow[D.m0 + j] = (f || v2) ? 0 : 1;
    }
    if (!f && !v2) atomicAdd(slow_entries, (unsigned long long)D.n * (unsigned long long)D.nm);
}

// Two-voxel row i of the list (member position pos[i]): its info (row, the
// two runs' first columns, material) and its values, copied in list order.
template <typename IT>
__global__ void __launch_bounds__(256) vox2_build(const int32_t *pos, int64_t n, const int32_t *grp_row,
                                                  const uint8_t *grp_mat, const IT *rp, const int32_t *col,
                                                  const float *val, int32_t *info, float *v2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = grp_row[pos[i]];
    const int64_t lo = (int64_t)rp[r];
    info[4 * i] = r;
    info[4 * i + 1] = col[lo];
    info[4 * i + 2] = col[lo + kVox2Run];
    info[4 * i + 3] = grp_mat[pos[i]];
    for (int k = 0; k < kVox2Len; ++k) v2[i * kVox2Len + k] = val[lo + k];
}

__global__ void __launch_bounds__(256) group_scatter(const int32_t *flag, const int32_t *pos, int64_t n,
                                                     int32_t *grp_ptr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) grp_ptr[pos[i]] = (int32_t)i;
}

// ---- brick order of the fast groups ---------------------------------------------
// The fast list is put in the order of bricks of kBrick^3 source voxels
// (bricks in z, y, x order; voxels within a brick in z, y, x order, x
// fastest), so that the value-indexed step can form a brick's groups in one
// workgroup and stage the rows they write.  brick_key: the brick and the
// position within it of fast group f's source voxel.
__global__ void __launch_bounds__(256) brick_keys(const GroupDesc *desc, const int32_t *fast, int64_t n_fast,
                                                  int n_dir, int nx, int ny, uint64_t *key)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_fast) return;
    const int64_t u = desc[fast[f]].cstart / n_dir;
    const int64_t x = u % nx, y = (u / nx) % ny, z = u / ((int64_t)nx * ny);
    const int64_t nbx = (nx + kBrick - 1) / kBrick, nby = (ny + kBrick - 1) / kBrick;
    const uint64_t brick = ((uint64_t)(z / kBrick) * nby + (uint64_t)(y / kBrick)) * nbx + (uint64_t)(x / kBrick);
    const uint64_t local = ((uint64_t)(z % kBrick) * kBrick + (uint64_t)(y % kBrick)) * kBrick + (uint64_t)(x % kBrick);
    key[f] = brick * (uint64_t)(kBrick * kBrick * kBrick) + local;
}

// first[f] = 1 where fast index f starts a brick
__global__ void __launch_bounds__(256) brick_starts(const uint64_t *key, int64_t n, uint8_t *first)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    const uint64_t b = key[f] / (uint64_t)(kBrick * kBrick * kBrick);
    first[f] = (f == 0 || key[f - 1] / (uint64_t)(kBrick * kBrick * kBrick) != b) ? 1 : 0;
}

// brick i: its origin voxel (from the brick number of its first group's key)
__global__ void __launch_bounds__(256) brick_origins(const int32_t *ptr, const uint64_t *key, int64_t n_brick, int nx,
                                                     int ny, int32_t *org)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_brick) return;
    const uint64_t b = key[ptr[i]] / (uint64_t)(kBrick * kBrick * kBrick);
    const int64_t nbx = (nx + kBrick - 1) / kBrick, nby = (ny + kBrick - 1) / kBrick;
    const int64_t bx = (int64_t)(b % (uint64_t)nbx), by = (int64_t)((b / (uint64_t)nbx) % (uint64_t)nby);
    const int64_t bz = (int64_t)(b / ((uint64_t)nbx * nby));
    org[i] = (int32_t)((bz * kBrick * ny + by * kBrick) * nx + bx * kBrick);
}

int order_fast_in_bricks(Matrix &A)
{
    Device &dev = A.dev;
    const int64_t G = A.n_fast;
    A.n_brick = 0;
    const Model &M = A.model;
    // consecutive fast groups of the brick order lie up to kBrick planes of
    // source voxels apart; the FP32 step takes a pair's values at 32-bit
    // offsets from the lower of the two, so larger planes keep the group order
    if (G <= 0 || M.nx <= 0 || M.n_vox >= INT32_MAX ||
        (int64_t)(kBrick + 1) * M.nx * M.ny * 26 * 26 * 4 >= (int64_t)INT32_MAX)
        return DRTS_OK;
    int rc;
    Buffer key, key_s, ids, tmp, first, cnt;
    if ((rc = key.allocate(&dev, G * sizeof(uint64_t)))) return rc;
    if ((rc = key_s.allocate(&dev, G * sizeof(uint64_t)))) return rc;
    if ((rc = ids.allocate(&dev, G * sizeof(int32_t)))) return rc;
    const unsigned gb = (unsigned)((G + 255) / 256);
    hipLaunchKernelGGL(brick_keys, dim3(gb), dim3(256), 0, dev.stream, A.grp_desc.as<GroupDesc>(),
                       A.grp_fast.as<int32_t>(), G, M.n_dir, M.nx, M.ny, key.as<uint64_t>());
    DRTS_HIP(hipGetLastError());
    size_t tb = 0, tb2 = 0;
    DRTS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key.as<uint64_t>(), key_s.as<uint64_t>(),
                                                A.grp_fast.as<int32_t>(), ids.as<int32_t>(), (int)G, 0, 64,
                                                dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tb, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.ptr, tb, key.as<uint64_t>(), key_s.as<uint64_t>(),
                                                A.grp_fast.as<int32_t>(), ids.as<int32_t>(), (int)G, 0, 64,
                                                dev.stream));
    DRTS_HIP(hipMemcpyAsync(A.grp_fast.ptr, ids.ptr, G * sizeof(int32_t), hipMemcpyDeviceToDevice, dev.stream));
    // brick starts and origins
    if ((rc = first.allocate(&dev, G))) return rc;
    if ((rc = cnt.allocate(&dev, sizeof(int64_t)))) return rc;
    hipLaunchKernelGGL(brick_starts, dim3(gb), dim3(256), 0, dev.stream, key_s.as<uint64_t>(), G, first.as<uint8_t>());
    DRTS_HIP(hipGetLastError());
    if ((rc = A.brick_ptr.allocate(&dev, (G + 1) * sizeof(int32_t)))) return rc;
    hipcub::CountingInputIterator<int32_t> fidx(0);
    DRTS_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb2, fidx, first.as<uint8_t>(), A.brick_ptr.as<int32_t>(),
                                           cnt.as<int64_t>(), (int)G, dev.stream));
    tmp.reset();
    if ((rc = tmp.allocate(&dev, std::max<size_t>(tb2, 16)))) return rc;
    DRTS_HIP(hipcub::DeviceSelect::Flagged(tmp.ptr, tb2, fidx, first.as<uint8_t>(), A.brick_ptr.as<int32_t>(),
                                           cnt.as<int64_t>(), (int)G, dev.stream));
    int64_t nb = 0;
    DRTS_HIP(hipMemcpyAsync(&nb, cnt.ptr, sizeof nb, hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    const int32_t end = (int32_t)G;
    DRTS_HIP(hipMemcpyAsync(A.brick_ptr.as<int32_t>() + nb, &end, sizeof end, hipMemcpyHostToDevice, dev.stream));
    if ((rc = A.brick_org.allocate(&dev, std::max<int64_t>(nb, 1) * sizeof(int32_t)))) return rc;
    hipLaunchKernelGGL(brick_origins, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, dev.stream,
                       A.brick_ptr.as<int32_t>(), key_s.as<uint64_t>(), nb, M.nx, M.ny, A.brick_org.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    A.n_brick = nb;
    return DRTS_OK;
}

// ---- value-indexed fast groups ------------------------------------------------
// A fast group's dictionary is the one of its source voxel's material (the
// voxel whose states are its columns).  Any assignment would be exact; this
// one keeps each dictionary to the few distinct values of one material's rows.
constexpr uint32_t kViEmpty = 0xffffffffu;

__device__ __forceinline__ int vi_table_of(const GroupDesc &D, const uint8_t *mat_of_voxel, int n_dir)
{
    return mat_of_voxel[D.cstart / n_dir];
}

// Inserts the bit pattern of every value of fast group f into its
// dictionary's hash set (linear probing; a full set raises *overflow).
__global__ void __launch_bounds__(256) vi_insert(const GroupDesc *desc, const int32_t *fast, int64_t n_fast,
                                                 const float *gval, const uint8_t *mat_of_voxel, int n_dir,
                                                 uint32_t *hs, int32_t *overflow)
{
    for (int64_t f = blockIdx.x; f < n_fast; f += gridDim.x) {
        const GroupDesc D = desc[fast[f]];
        uint32_t *set = hs + (size_t)vi_table_of(D, mat_of_voxel, n_dir) * kViHash;
        for (int e = threadIdx.x; e < D.n * D.nm; e += blockDim.x) {
            const uint32_t bits = __float_as_uint(gval[D.voff + e]);
            if (bits == kViEmpty) {
                atomicExch(overflow, 1);
                continue;
            }
            uint32_t h = (bits * 2654435761u) >> 20;
            bool done = false;
            for (int p = 0; p < kViHash && !done; ++p, h = (h + 1) & (kViHash - 1)) {
                const uint32_t cur = __hip_atomic_load(set + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (cur == bits) done = true;
                else if (cur == kViEmpty) {
                    const uint32_t old = atomicCAS(set + h, kViEmpty, bits);
                    done = old == kViEmpty || old == bits;
                }
            }
            if (!done) atomicExch(overflow, 1);
        }
    }
}

// Slot j of fast group f: member j's values as indices into its dictionary
// (sorted bit patterns: an exact match by binary search), the dictionary at
// byte kViTabByte, the group's position in its brick at byte kViPosByte and
// the member's row in word kViRowWord (for j >= the member count: no
// indices, the last member's row).
__global__ void __launch_bounds__(256) vi_encode(const GroupDesc *desc, const int32_t *fast, int64_t n_fast,
                                                 const float *gval, const int32_t *grp_row,
                                                 const uint8_t *mat_of_voxel, int n_dir, int nx, int ny,
                                                 const uint32_t *dict_bits, const int32_t *dict_n, uint8_t *idx,
                                                 int32_t *missing)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n_fast * 26) return;
    const int64_t f = gid / 26;
    const int j = (int)(gid % 26);
    const GroupDesc D = desc[fast[f]];
    const int tab = vi_table_of(D, mat_of_voxel, n_dir);
    const uint32_t *dk = dict_bits + (size_t)tab * kViDict;
    const int nd = dict_n[tab];
    uint32_t w[kViSlot / 4] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (j < D.nm) {
        for (int k = 0; k < D.n; ++k) {
            const uint32_t bits = __float_as_uint(gval[D.voff + (int64_t)k * D.nm + j]);
            int lo = 0, hi = nd;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (dk[mid] < bits) lo = mid + 1;
                else hi = mid;
            }
            if (lo >= nd || dk[lo] != bits) atomicExch(missing, 1);
            w[k >> 2] |= (uint32_t)(lo & 0xff) << (8 * (k & 3));
        }
    }
    w[kViTabByte >> 2] |= (uint32_t)tab << (8 * (kViTabByte & 3));
    // the source voxel's position in its brick
    const int64_t u = D.cstart / n_dir;
    const int64_t x = u % nx, y = (u / nx) % ny, z = u / ((int64_t)nx * ny);
    const uint32_t pos = (uint32_t)(((z % kBrick) * kBrick + (y % kBrick)) * kBrick + (x % kBrick));
    w[kViPosByte >> 2] |= pos << (8 * (kViPosByte & 3));
    w[kViRowWord] = (uint32_t)grp_row[D.m0 + min(j, D.nm - 1)];
    uint4 *out = (uint4 *)(idx + f * kViBlock + (int64_t)j * kViSlot);
    out[0] = make_uint4(w[0], w[1], w[2], w[3]);
    out[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

template <typename T> int upload_host(Device &dev, Buffer &b, const std::vector<T> &v)
{
    int rc = b.allocate(&dev, std::max<size_t>(v.size(), 1) * sizeof(T));
    if (rc) return rc;
    if (!v.empty()) DRTS_HIP(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, dev.stream));
    return DRTS_OK;
}

__global__ void __launch_bounds__(256) fdesc_build(const GroupDesc *desc, const int32_t *fast, int64_t n_fast,
                                                   int32_t *fd)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_fast) return;
    const int32_t g = fast[f];
    const GroupDesc D = desc[g];
    fd[4 * f] = D.m0;
    fd[4 * f + 1] = D.nm;
    fd[4 * f + 2] = D.cstart;
    fd[4 * f + 3] = g;
}

// fast_of[g] = f for fast group g = fast[f] (the other entries stay -1)
__global__ void __launch_bounds__(256) fast_index_of(const int32_t *fast, int64_t n_fast, int32_t *fast_of)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n_fast) fast_of[fast[f]] = (int32_t)f;
}

__global__ void __launch_bounds__(256) fast_flag_bits(const int32_t *fast, int64_t n_fast, const uint32_t *gbits,
                                                      uint32_t *fbits)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w * 32 >= n_fast) return;
    uint32_t word = 0;
    for (int b = 0; b < 32 && w * 32 + b < n_fast; ++b) {
        const int32_t g = fast[w * 32 + b];
        word |= ((gbits[g >> 5] >> (g & 31)) & 1u) << b;
    }
    fbits[w] = word;
}

// Builds A.vi_idx / A.vi_dict (and the map of A's n_groups groups to fast
// indices), or leaves A.vi_ntab = 0 when a material has
// more than kViDict distinct values among its fast groups' entries (or there
// are more than kViTabs materials).
int build_value_index(Matrix &A, int64_t n_groups)
{
    Device &dev = A.dev;
    A.vi_ntab = 0;
    const int n_mat = (int)A.model.absorb.size();
    if (A.n_fast <= 0 || n_mat <= 0 || n_mat > kViTabs || A.n_brick <= 0) return DRTS_OK;
    int rc;
    Buffer hs, flags;
    if ((rc = hs.allocate(&dev, (size_t)n_mat * kViHash * sizeof(uint32_t)))) return rc;
    if ((rc = flags.allocate(&dev, 2 * sizeof(int32_t)))) return rc;
    DRTS_HIP(hipMemsetAsync(hs.ptr, 0xff, (size_t)n_mat * kViHash * sizeof(uint32_t), dev.stream));
    DRTS_HIP(hipMemsetAsync(flags.ptr, 0, 2 * sizeof(int32_t), dev.stream));
    const unsigned ib = (unsigned)std::min<int64_t>(A.n_fast, 65536);
    hipLaunchKernelGGL(vi_insert, dim3(ib), dim3(256), 0, dev.stream, A.grp_desc.as<GroupDesc>(),
                       A.grp_fast.as<int32_t>(), A.n_fast, A.grp_val.as<float>(), A.mat_of_voxel.as<uint8_t>(),
                       A.model.n_dir, hs.as<uint32_t>(), flags.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    std::vector<uint32_t> h((size_t)n_mat * kViHash);
    int32_t fl[2] = {0, 0};
    DRTS_HIP(hipMemcpyAsync(h.data(), hs.ptr, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipMemcpyAsync(fl, flags.ptr, sizeof fl, hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    if (fl[0]) return DRTS_OK;
    // per material: its distinct bit patterns, sorted
    std::vector<uint32_t> dict((size_t)n_mat * kViDict, 0u);
    std::vector<int32_t> dn((size_t)n_mat, 0);
    std::vector<float> dval((size_t)n_mat * kViDict, 0.0f);
    for (int q = 0; q < n_mat; ++q) {
        std::vector<uint32_t> u;
        for (int i = 0; i < kViHash; ++i)
            if (h[(size_t)q * kViHash + i] != kViEmpty) u.push_back(h[(size_t)q * kViHash + i]);
        if (u.size() > (size_t)kViDict) return DRTS_OK;
        std::sort(u.begin(), u.end());
        dn[(size_t)q] = (int32_t)u.size();
        for (size_t i = 0; i < u.size(); ++i) {
            dict[(size_t)q * kViDict + i] = u[i];
            std::memcpy(&dval[(size_t)q * kViDict + i], &u[i], sizeof(float));
        }
    }
    Buffer dbits, dcount;
    if ((rc = upload_host(dev, dbits, dict))) return rc;
    if ((rc = upload_host(dev, dcount, dn))) return rc;
    if ((rc = A.vi_idx.allocate(&dev, (size_t)A.n_fast * kViBlock))) return rc;
    if ((rc = upload_host(dev, A.vi_dict, dval))) return rc;
    const int64_t nt = A.n_fast * 26;
    hipLaunchKernelGGL(vi_encode, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, dev.stream,
                       A.grp_desc.as<GroupDesc>(), A.grp_fast.as<int32_t>(), A.n_fast, A.grp_val.as<float>(),
                       A.grp_row.as<int32_t>(), A.mat_of_voxel.as<uint8_t>(), A.model.n_dir, A.model.nx, A.model.ny,
                       dbits.as<uint32_t>(),
                       dcount.as<int32_t>(), A.vi_idx.as<uint8_t>(), flags.as<int32_t>() + 1);
    DRTS_HIP(hipGetLastError());
    DRTS_HIP(hipMemcpyAsync(fl, flags.ptr, sizeof fl, hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    if (fl[1]) {
        A.vi_idx.reset();
        A.vi_dict.reset();
        return DRTS_OK;
    }
    if ((rc = A.vi_fdesc.allocate(&dev, (size_t)A.n_fast * 4 * sizeof(int32_t)))) return rc;
    hipLaunchKernelGGL(fdesc_build, dim3((unsigned)((A.n_fast + 255) / 256)), dim3(256), 0, dev.stream,
                       A.grp_desc.as<GroupDesc>(), A.grp_fast.as<int32_t>(), A.n_fast, A.vi_fdesc.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    // each group's fast index (the many-rhs step walks the groups in group order)
    if ((rc = A.vi_fast_of.allocate(&dev, (size_t)n_groups * sizeof(int32_t)))) return rc;
    DRTS_HIP(hipMemsetAsync(A.vi_fast_of.ptr, 0xff, (size_t)n_groups * sizeof(int32_t), dev.stream));
    hipLaunchKernelGGL(fast_index_of, dim3((unsigned)((A.n_fast + 255) / 256)), dim3(256), 0, dev.stream,
                       A.grp_fast.as<int32_t>(), A.n_fast, A.vi_fast_of.as<int32_t>());
    DRTS_HIP(hipGetLastError());
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    A.vi_ntab = n_mat;
    return DRTS_OK;
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
    Buffer gptr;
    if ((rc = gptr.allocate(&dev, out.size() * sizeof(int32_t)))) return rc;
    DRTS_HIP(hipMemcpyAsync(gptr.ptr, out.data(), out.size() * sizeof(int32_t), hipMemcpyHostToDevice,
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
    if ((rc = A.grp_desc.allocate(&dev, G * sizeof(GroupDesc)))) return rc;
    const unsigned gblocks = (unsigned)((G + 255) / 256);
    hipLaunchKernelGGL(group_descs<IT>, dim3(gblocks), dim3(256), 0, dev.stream, gptr.as<int32_t>(),
                       A.grp_row.as<int32_t>(), rp, col, moff.as<int64_t>(), G, A.grp_desc.as<GroupDesc>());
    DRTS_HIP(hipGetLastError());
    // (the same padding after the last entry as the CSR values)
    if ((rc = A.grp_val.allocate(&dev, A.val.bytes))) return rc;
    DRTS_HIP(hipMemsetAsync(A.grp_val.ptr, 0, A.val.bytes, dev.stream));
    hipLaunchKernelGGL(group_values<IT>, dim3(gblocks), dim3(256), 0, dev.stream, A.grp_desc.as<GroupDesc>(),
                       A.grp_row.as<int32_t>(), rp, A.val.as<float>(), G, A.grp_val.as<float>());
    DRTS_HIP(hipGetLastError());
    // the single-rhs step takes the fast groups by row groups and the rows of
    // the others one by one: the list of fast groups and the list of those rows
    Buffer fast, mvox2, mslow, v2pos, cnt;
    if ((rc = fast.allocate(&dev, G))) return rc;
    if ((rc = mvox2.allocate(&dev, R))) return rc;
    if ((rc = mslow.allocate(&dev, R))) return rc;
    if ((rc = cnt.allocate(&dev, 4 * sizeof(int64_t)))) return rc;
    DRTS_HIP(hipMemsetAsync(cnt.ptr, 0, 4 * sizeof(int64_t), dev.stream));
    hipLaunchKernelGGL(group_kinds, dim3(gblocks), dim3(256), 0, dev.stream, A.grp_desc.as<GroupDesc>(), col, G,
                       fast.as<uint8_t>(), mvox2.as<uint8_t>(), mslow.as<uint8_t>(),
                       (unsigned long long *)(cnt.as<int64_t>() + 2));
    DRTS_HIP(hipGetLastError());
    if ((rc = A.grp_fast.allocate(&dev, G * sizeof(int32_t)))) return rc;
    if ((rc = A.slow_rows.allocate(&dev, R * sizeof(int32_t)))) return rc;
    if ((rc = v2pos.allocate(&dev, R * sizeof(int32_t)))) return rc;
    hipcub::CountingInputIterator<int32_t> gidx(0);
    size_t tb4 = 0, tb5 = 0, tb6 = 0;
    DRTS_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb4, gidx, fast.as<uint8_t>(), A.grp_fast.as<int32_t>(),
                                           cnt.as<int64_t>(), (int)G, dev.stream));
    DRTS_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb5, A.grp_row.as<int32_t>(), mslow.as<uint8_t>(),
                                           A.slow_rows.as<int32_t>(), cnt.as<int64_t>() + 1, (int)R, dev.stream));
    DRTS_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb6, gidx, mvox2.as<uint8_t>(), v2pos.as<int32_t>(),
                                           cnt.as<int64_t>() + 3, (int)R, dev.stream));
    if ((rc = tmp.allocate(&dev, std::max<size_t>(std::max(std::max(tb4, tb5), tb6), 16)))) return rc;
    DRTS_HIP(hipcub::DeviceSelect::Flagged(tmp.ptr, tb4, gidx, fast.as<uint8_t>(), A.grp_fast.as<int32_t>(),
                                           cnt.as<int64_t>(), (int)G, dev.stream));
    DRTS_HIP(hipcub::DeviceSelect::Flagged(tmp.ptr, tb5, A.grp_row.as<int32_t>(), mslow.as<uint8_t>(),
                                           A.slow_rows.as<int32_t>(), cnt.as<int64_t>() + 1, (int)R, dev.stream));
    DRTS_HIP(hipcub::DeviceSelect::Flagged(tmp.ptr, tb6, gidx, mvox2.as<uint8_t>(), v2pos.as<int32_t>(),
                                           cnt.as<int64_t>() + 3, (int)R, dev.stream));
    int64_t counts[4] = {0, 0, 0, 0};
    DRTS_HIP(hipMemcpyAsync(counts, cnt.ptr, sizeof counts, hipMemcpyDeviceToHost, dev.stream));
    DRTS_HIP(hipStreamSynchronize(dev.stream));
    A.n_fast = counts[0];
    A.n_slow = counts[1];
    A.n_slow_nnz = counts[2];
    A.n_vox2 = counts[3];
    if ((rc = order_fast_in_bricks(A))) return rc;
    // the two-voxel rows' info and values in list order
    if ((rc = A.vox2_info.allocate(&dev, (size_t)std::max<int64_t>(A.n_vox2, 1) * 4 * sizeof(int32_t)))) return rc;
    if ((rc = A.vox2_val.allocate(&dev, (size_t)std::max<int64_t>(A.n_vox2, 1) * kVox2Len * sizeof(float))))
        return rc;
    if (A.n_vox2 > 0) {
        hipLaunchKernelGGL(vox2_build<IT>, dim3((unsigned)((A.n_vox2 + 255) / 256)), dim3(256), 0, dev.stream,
                           v2pos.as<int32_t>(), A.n_vox2, A.grp_row.as<int32_t>(), A.grp_mat.as<uint8_t>(), rp, col,
                           A.val.as<float>(), A.vox2_info.as<int32_t>(), A.vox2_val.as<float>());
        DRTS_HIP(hipGetLastError());
        DRTS_HIP(hipStreamSynchronize(dev.stream));
    }
    if ((rc = build_value_index(A, G))) return rc;
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
        Buffer *b[] = {&A.grp_desc, &A.grp_row,   &A.grp_mat,   &A.grp_val,   &A.grp_fast,
                       &A.slow_rows, &A.vox2_info, &A.vox2_val,  &A.vi_idx,    &A.vi_dict,
                       &A.brick_ptr, &A.brick_org, &A.vi_fdesc,  &A.vi_fast_of};
        for (Buffer *x : b) x->reset();
        A.n_groups = -1;
    }
    return rc;
}

int group_flags(const Matrix &A, const int64_t *rows, int64_t n, uint32_t *bits, hipStream_t stream)
{
    const int64_t words = (A.n_groups + 31) / 32;
    if (words <= 0) return DRTS_OK;
    hipLaunchKernelGGL(group_flag_bits, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream,
                       A.grp_desc.as<GroupDesc>(), A.grp_row.as<int32_t>(), A.n_groups, rows, n, bits);
    DRTS_HIP(hipGetLastError());
    return DRTS_OK;
}

int fast_flags(const Matrix &A, const uint32_t *gbits, uint32_t *fbits, hipStream_t stream)
{
    const int64_t words = (A.n_fast + 31) / 32;
    if (words <= 0) return DRTS_OK;
    hipLaunchKernelGGL(fast_flag_bits, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream,
                       A.grp_fast.as<int32_t>(), A.n_fast, gbits, fbits);
    DRTS_HIP(hipGetLastError());
    return DRTS_OK;
}

}  // namespace drts
