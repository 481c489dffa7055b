// build.hip -- vor_build_grid: the setup phase of the straight-path method
// (Sect. 2.2, setup items 1-3) on the GPU.
//
//  1. validate the sites and give each a 30-bit Hilbert key;
//  2. radix-sort the sites into Hilbert order (internal order);
//  3. bucket the sites into a uniform grid (stable radix sort by bucket);
//  4. per site, clip the box by the bisector half-spaces of nearby sites,
//     taken nearest-first from rings of buckets, until no farther site can
//     cut the cell (its distance exceeds twice the largest vertex radius);
//     the planes left bounding the cell are its neighbours (Sect. 2.1);
//  5. make the lists symmetric, sort each row, and lay out the trace
//     records (FP64 sites and FP32 offsets per neighbour, CSR by cell).
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/voronoi_rt_diag.h"
#include "clip_wave.h"

using namespace vrt;

namespace {

__global__ void k_validate_keys(const double *__restrict__ sites, int64_t M, BoxArg box, double scale,
                                uint32_t *__restrict__ keys, int32_t *__restrict__ vals, int *__restrict__ err)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    uint32_t c[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        double x = sites[3 * i + a];
        if (!(x >= box.lo[a] && x <= box.hi[a])) ok = false;   // also rejects NaN
        double f = ok ? (x - box.lo[a]) * scale : 0.0;
        int q = (int)f;
        q = q < 0 ? 0 : (q > (1 << kHilbertBits) - 1 ? (1 << kHilbertBits) - 1 : q);
        c[a] = (uint32_t)q;
    }
    if (!ok) atomicOr(err, ERR_OUTSIDE);
    keys[i] = hilbert_key(c[0], c[1], c[2]);
    vals[i] = (int32_t)i;
}

__global__ void k_gather_sites(const double *__restrict__ sites, const int32_t *__restrict__ order, int64_t M,
                               Site *__restrict__ out, int32_t *__restrict__ perm, int32_t *__restrict__ inv_perm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int32_t u = order[i];
    Site s;
    s.x = sites[3 * (int64_t)u];
    s.y = sites[3 * (int64_t)u + 1];
    s.z = sites[3 * (int64_t)u + 2];
    s.uid = u;
    out[i] = s;
    perm[i] = u;
    inv_perm[u] = (int32_t)i;
}

struct GridArg {
    double lo[3];
    double inv_h[3];
    int32_t dims[3];
};

__global__ void k_bucket_keys(const Site *__restrict__ sites, int64_t M, GridArg g, uint32_t *__restrict__ keys,
                              int32_t *__restrict__ vals, int32_t *__restrict__ counts)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    Site s = sites[i];
    int bx = bucket_coord(s.x, g.lo[0], g.inv_h[0], g.dims[0]);
    int by = bucket_coord(s.y, g.lo[1], g.inv_h[1], g.dims[1]);
    int bz = bucket_coord(s.z, g.lo[2], g.inv_h[2], g.dims[2]);
    uint32_t b = (uint32_t)((bz * g.dims[1] + by) * g.dims[0] + bx);
    keys[i] = b;
    vals[i] = (int32_t)i;
    atomicAdd(&counts[b], 1);
}

__global__ void k_bucket_fill(const Site *__restrict__ sites, const int32_t *__restrict__ order, int64_t M,
                              Site *__restrict__ out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    int32_t i = order[k];
    Site s = sites[i];
    s.uid = (s.uid << 32) | (int64_t)(uint32_t)i;
    out[k] = s;
}

struct ClipArgs {
    const Site *sites;        // internal order
    BucketGridView grid;
    BoxArg box;
    int64_t M;
    int32_t *nbr;             // [M * kMaxNbr] first-pass lists
    int32_t *cnt;             // [M]
    uint8_t *walls;           // [M]
    int32_t *retry;           // [M] sites whose cell needs the large capacity
    int32_t *n_retry;
    int *err;
    double *volume;           // [M] cell volumes
    double *bbox;             // [6 M] cell bounding boxes, or null
};

// First pass: one wave per site with a small cell in LDS; cells that run
// out of faces are queued for the second pass.
__global__ void __launch_bounds__(64) k_clip(ClipArgs A)
{
    __shared__ WaveCellSmall cell;
    const int64_t i = blockIdx.x;
    uint8_t wm = 0;
    double vol = 0.0, bb[6];
    int n = wclip_site(cell, A.sites, A.grid, A.box, i, A.nbr + i * kMaxNbr, kMaxNbr, &wm, &vol,
                       A.bbox ? bb : nullptr);
    if (threadIdx.x == 0) {
        A.volume[i] = vol;
        if (A.bbox && n >= 0)
            for (int a = 0; a < 6; ++a) A.bbox[6 * i + a] = bb[a];
        if (n == -ERR_CAPACITY) {
            A.retry[atomicAdd(A.n_retry, 1)] = (int32_t)i;
            n = 0;
        } else if (n < 0) {
            atomicOr(A.err, -n);
            n = 0;
        }
        A.cnt[i] = n;
        A.walls[i] = wm;
    }
}

// Second pass over the queued sites, with large cells (up to 255 faces).
__global__ void __launch_bounds__(64) k_clip_big(ClipArgs A, int32_t *__restrict__ big_nbr, int32_t *__restrict__ slot)
{
    __shared__ WaveCellBig cell;
    const int k = blockIdx.x;
    const int64_t i = A.retry[k];
    uint8_t wm = 0;
    double vol = 0.0, bb[6];
    int n = wclip_site(cell, A.sites, A.grid, A.box, i, big_nbr + (int64_t)k * kMaxNbrBig, kMaxNbrBig, &wm, &vol,
                       A.bbox ? bb : nullptr);
    if (threadIdx.x == 0) {
        A.volume[i] = vol;
        if (A.bbox && n >= 0)
            for (int a = 0; a < 6; ++a) A.bbox[6 * i + a] = bb[a];
        slot[i] = k;
        if (n < 0) {
            atomicOr(A.err, -n);
            n = 0;
        }
        A.cnt[i] = n;
        A.walls[i] = wm;
    }
}

// The paper's locate structure (Sect. 2.3): a regular grid of blocks over
// the box; block k lists every cell whose bounding box overlaps it. The box
// of cell i is widened by 1e-9 of its extent (plus 1e-12 of the domain's)
// on each side, so that rounding in its vertices cannot drop a block the
// cell reaches. Blocks are numbered (x * ny + y) * nz + z.
struct LocArgs {
    const double *bbox;   // [6 M] internal order
    int64_t M;
    double lo[3], inv_h[3], ext[3];
    int32_t dims[3];
};

__device__ __forceinline__ void loc_range(const LocArgs &A, int64_t i, int b0[3], int b1[3])
{
    for (int a = 0; a < 3; ++a) {
        const double lo = A.bbox[6 * i + a], hi = A.bbox[6 * i + a + 3];
        const double m = 1e-9 * (hi - lo) + 1e-12 * A.ext[a];
        b0[a] = bucket_coord(lo - m, A.lo[a], A.inv_h[a], A.dims[a]);
        b1[a] = bucket_coord(hi + m, A.lo[a], A.inv_h[a], A.dims[a]);
    }
}

__global__ void k_loc_count(LocArgs A, int32_t *__restrict__ cnt, unsigned long long *__restrict__ total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.M) return;
    int b0[3], b1[3];
    loc_range(A, i, b0, b1);
    for (int x = b0[0]; x <= b1[0]; ++x)
        for (int y = b0[1]; y <= b1[1]; ++y)
            for (int z = b0[2]; z <= b1[2]; ++z) atomicAdd(&cnt[((int64_t)x * A.dims[1] + y) * A.dims[2] + z], 1);
    atomicAdd(total, (unsigned long long)(b1[0] - b0[0] + 1) * (b1[1] - b0[1] + 1) * (b1[2] - b0[2] + 1));
}

__global__ void k_loc_fill(LocArgs A, const int32_t *__restrict__ start, int32_t *__restrict__ cursor,
                           int32_t *__restrict__ cells)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.M) return;
    int b0[3], b1[3];
    loc_range(A, i, b0, b1);
    for (int x = b0[0]; x <= b1[0]; ++x)
        for (int y = b0[1]; y <= b1[1]; ++y)
            for (int z = b0[2]; z <= b1[2]; ++z) {
                const int64_t k = ((int64_t)x * A.dims[1] + y) * A.dims[2] + z;
                cells[start[k] + atomicAdd(&cursor[k], 1)] = (int32_t)i;
            }
}

// Directed lists -> CSR (dir_start from a scan of cnt). slot[i] >= 0 marks a
// site redone by the second pass; its list is in big_nbr at that slot.
__global__ void k_gather_dir(const int32_t *__restrict__ nbr, const int32_t *__restrict__ cnt,
                             const int32_t *__restrict__ dir_start, const int32_t *__restrict__ slot, int64_t M,
                             const int32_t *__restrict__ big_nbr, int32_t *__restrict__ dir_col)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int n = cnt[i];
    int k = slot[i];
    const int32_t *src = (k < 0) ? nbr + i * kMaxNbr : big_nbr + (int64_t)k * kMaxNbrBig;
    int32_t *dst = dir_col + dir_start[i];
    for (int e = 0; e < n; ++e) dst[e] = src[e];
}

__device__ __forceinline__ bool row_has(const int32_t *__restrict__ col, int s, int n, int32_t x)
{
    for (int e = 0; e < n; ++e)
        if (col[s + e] == x) return true;
    return false;
}

// For every directed entry i -> j whose reverse is missing, count an extra
// entry for row j.
__global__ void k_symm_count(const int32_t *__restrict__ dir_col, const int32_t *__restrict__ dir_start,
                             const int32_t *__restrict__ cnt, int64_t M, int32_t *__restrict__ extra)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int s = dir_start[i], n = cnt[i];
    for (int e = 0; e < n; ++e) {
        int32_t j = dir_col[s + e];
        if (!row_has(dir_col, dir_start[j], cnt[j], (int32_t)i)) atomicAdd(&extra[j], 1);
    }
}

__global__ void k_total_counts(const int32_t *__restrict__ cnt, const int32_t *__restrict__ extra, int64_t M,
                               int32_t *__restrict__ total)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    total[i] = cnt[i] + extra[i];
}

// Copy each directed row to the front of its final row; cursor = its length.
__global__ void k_copy_rows(const int32_t *__restrict__ dir_col, const int32_t *__restrict__ dir_start,
                            const int32_t *__restrict__ cnt, const int32_t *__restrict__ start, int64_t M,
                            int32_t *__restrict__ col, int32_t *__restrict__ cursor)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int s = dir_start[i], n = cnt[i], o = start[i];
    for (int e = 0; e < n; ++e) col[o + e] = dir_col[s + e];
    cursor[i] = n;
}

// Append the missing reverse entries (same test as k_symm_count).
__global__ void k_symm_fill(const int32_t *__restrict__ dir_col, const int32_t *__restrict__ dir_start,
                            const int32_t *__restrict__ cnt, const int32_t *__restrict__ start, int64_t M,
                            int32_t *__restrict__ col, int32_t *__restrict__ cursor)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int s = dir_start[i], n = cnt[i];
    for (int e = 0; e < n; ++e) {
        int32_t j = dir_col[s + e];
        if (!row_has(dir_col, dir_start[j], cnt[j], (int32_t)i)) {
            int pos = atomicAdd(&cursor[j], 1);
            col[start[j] + pos] = (int32_t)i;
        }
    }
}

__global__ void k_row_sort(int32_t *__restrict__ col, const int32_t *__restrict__ start,
                           const int32_t *__restrict__ total, int64_t M)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int32_t *row = col + start[i];
    int n = total[i];
    for (int a = 1; a < n; ++a) {
        int32_t x = row[a];
        int k = a - 1;
        while (k >= 0 && row[k] > x) {
            row[k + 1] = row[k];
            --k;
        }
        row[k + 1] = x;
    }
}

__device__ __forceinline__ int wave_max_int(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Slots of a compact cell block: the header, then 12 bytes per neighbour
// (8-byte record + block offset), rounded up to whole slots. (Blocks start
// on any slot: starting them on 64- or 128-byte lines was measured slower.)
__global__ void k_compact_slots(const int32_t *__restrict__ total, int64_t M, int32_t *__restrict__ slots)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) slots[i] = kHdrSlots + (3 * total[i] + 3) / 4;
}

// The cell blocks and the FP64 records. Block i starts at blk_off[i]
// (compact) or block_of(row, i); each header records the start of the
// cell's FP64 row. FP32 blocks hold the offsets p_j - p_m rounded to FP32;
// compact blocks hold them as 21-bit integers against the cell's scale
// 2^(E - 19), E the smallest exponent with every offset component below
// 2^E (so |q| <= 2^19), but at least e_min, so that the box in the cell's
// units stays far inside the FP32 range; rounding to the nearest integer
// leaves each component within half a unit of the scale.
__global__ void k_fill_records(const Site *__restrict__ sites, const int32_t *__restrict__ col,
                               const int32_t *__restrict__ total, const int32_t *__restrict__ start, int64_t M,
                               int2 *__restrict__ rows, Rec64 *__restrict__ r64, Slot *__restrict__ blk,
                               const int32_t *__restrict__ blk_off, int compact, int e_min,
                               int *__restrict__ max_row)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0;
    if (i < M) {
        n = total[i];
        int s0 = start[i];
        rows[i] = make_int2(s0, n);
        const Site si = sites[i];
        const int32_t bo = blk_off ? blk_off[i] : block_of(make_int2(s0, n), (int32_t)i);
        int E = 0;
        if (compact) {
            double mc = 0.0;
            for (int e = 0; e < n; ++e) {
                const Site sj = sites[col[s0 + e]];
                mc = fmax(mc, fmax(fabs(sj.x - si.x), fmax(fabs(sj.y - si.y), fabs(sj.z - si.z))));
            }
            E = mc > 0.0 ? ilogb(mc) + 1 : e_min;
            E = E < e_min ? e_min : (E > 127 ? 127 : E);
        }
        BlockHdr h;
        h.x = si.x;
        h.y = si.y;
        h.z = si.z;
        h.uid = (int32_t)si.uid;
        h.j = (int32_t)i;
        h.len = n | (compact ? (E + kScaleBias) << 24 : 0);
        h.row = s0;
        h.rho = 0.0;
        *reinterpret_cast<BlockHdr *>(blk + bo) = h;
        float *rec = reinterpret_cast<float *>(blk + bo + kHdrSlots);           // FP32: n records of 3 floats
        uint2 *crec = reinterpret_cast<uint2 *>(blk + bo + kHdrSlots);          // compact: n records of 8 bytes
        int32_t *nb = compact ? reinterpret_cast<int32_t *>(crec + n) : reinterpret_cast<int32_t *>(rec + 3 * n);
        const double sc = ldexp(1.0, kQShift - E);
        for (int e = 0; e < n; ++e) {
            int32_t j = col[s0 + e];
            const Site sj = sites[j];
            Rec64 a;
            a.x = sj.x;
            a.y = sj.y;
            a.z = sj.z;
            a.j = j;
            a.uid = (int32_t)sj.uid;
            r64[s0 + e] = a;
            if (compact) {
                const uint64_t m21 = (1ull << kQBits) - 1;
                const uint64_t qx = (uint64_t)(int64_t)rint((sj.x - si.x) * sc) & m21;
                const uint64_t qy = (uint64_t)(int64_t)rint((sj.y - si.y) * sc) & m21;
                const uint64_t qz = (uint64_t)(int64_t)rint((sj.z - si.z) * sc) & m21;
                const uint64_t v = qx | (qy << kQBits) | (qz << (2 * kQBits));
                crec[e] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
            } else {
                rec[3 * e] = (float)(sj.x - si.x);
                rec[3 * e + 1] = (float)(sj.y - si.y);
                rec[3 * e + 2] = (float)(sj.z - si.z);
            }
            nb[e] = blk_off ? blk_off[j] : block_of(make_int2(start[j], 0), j);
        }
    }
    int m = wave_max_int(n);
    if ((threadIdx.x & 63) == 0) atomicMax(max_row, m);
}

// Slots of an FP64 cell block: the header, then 28 bytes per neighbour (its
// FP64 site and block offset), rounded up to whole slots.
__global__ void k_fp64_slots(const int2 *__restrict__ rows, int64_t M, int32_t *__restrict__ slots)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) slots[i] = kHdrSlots + (7 * rows[i].y + 3) / 4;
}

// FP64 cell blocks, what FP64-mode steps read: the header of the mixed-mode
// blocks, then the cell's n neighbour sites in FP64 (24 bytes each, in the
// row's order: ascending internal index), then the n neighbours' block
// offsets. Block i starts at blk64_off[i].
__global__ void k_fill_blk64(const Site *__restrict__ sites, const int2 *__restrict__ rows,
                             const Rec64 *__restrict__ r64, const int32_t *__restrict__ blk64_off, int64_t M,
                             Slot *__restrict__ blk64)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int2 rw = rows[i];
    const int32_t bo = blk64_off[i];
    const Site si = sites[i];
    BlockHdr h;
    h.x = si.x;
    h.y = si.y;
    h.z = si.z;
    h.rho = 0.0;
    h.uid = (int32_t)si.uid;
    h.j = (int32_t)i;
    h.len = rw.y;
    h.row = rw.x;
    *reinterpret_cast<BlockHdr *>(blk64 + bo) = h;
    double *rec = reinterpret_cast<double *>(blk64 + bo + kHdrSlots);
    int32_t *nb = reinterpret_cast<int32_t *>(rec + 3 * rw.y);
    for (int e = 0; e < rw.y; ++e) {
        const Rec64 a = r64[rw.x + e];
        rec[3 * e] = a.x;
        rec[3 * e + 1] = a.y;
        rec[3 * e + 2] = a.z;
        nb[e] = blk64_off[a.j];
    }
}

__global__ void k_export_counts(const int32_t *__restrict__ inv_perm, const int2 *__restrict__ rows,
                                const uint8_t *__restrict__ walls, int64_t M, int32_t *__restrict__ cnt)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= M) return;
    int32_t i = inv_perm[u];
    cnt[u] = rows[i].y + __popc((unsigned)walls[i]);
}

__global__ void k_export_fill(const int32_t *__restrict__ inv_perm, const int32_t *__restrict__ perm,
                              const int2 *__restrict__ rows, const Rec64 *__restrict__ r64,
                              const uint8_t *__restrict__ walls, int64_t M, const int64_t *__restrict__ row_ptr,
                              int32_t *__restrict__ col)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= M) return;
    int32_t i = inv_perm[u];
    int2 rw = rows[i];
    int32_t *out = col + row_ptr[u];
    for (int e = 0; e < rw.y; ++e) {
        int32_t x = r64[rw.x + e].uid;
        int k = e - 1;
        while (k >= 0 && out[k] > x) {
            out[k + 1] = out[k];
            --k;
        }
        out[k + 1] = x;
    }
    int n = rw.y;
    for (int w = 0; w < 6; ++w)
        if ((walls[i] >> w) & 1) out[n++] = -(w + 1);
}

// Device memory of a grid: from the caller's allocator when one is given
// (e.g. a framework's caching allocator), else hipMalloc.
struct DevBlock {
    void *p;
    size_t bytes;
};

struct DevAlloc {
    vor_allocator a{};
    bool custom = false;
    void *stream = nullptr;
    void *get(size_t bytes) const
    {
        if (custom) return a.alloc(bytes, a.ctx, stream);
        void *p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void put(const DevBlock &b) const
    {
        if (!b.p) return;
        if (custom) a.free(b.p, b.bytes, a.ctx, stream);
        else (void)hipFree(b.p);
    }
};

template <typename T>
T *dalloc(size_t n, vor_status &st, std::vector<DevBlock> &track, const DevAlloc &A)
{
    if (st != VOR_OK) return nullptr;
    const size_t bytes = n * sizeof(T) > 0 ? n * sizeof(T) : 1;
    void *p = A.get(bytes);
    if (!p) {
        st = VOR_ENOMEM;
        return nullptr;
    }
    track.push_back(DevBlock{p, bytes});
    return (T *)p;
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

// Cell blocks of more than this many bytes in the FP32 layout do not stay in
// the last-level cache; the automatic layout makes them compact.
constexpr int64_t kCompactAutoBytes = 512ll << 20;

// The smallest scale exponent of a compact block: 2^40 below the box
// diagonal, so that points of the box in a cell's units stay below 2^60
// (their squares inside the FP32 range); and at least -126.
static int compact_min_exp(const double box[6])
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (box[a + 3] - box[a]) * (box[a + 3] - box[a]);
    const int e = d2 > 0.0 ? ilogb(sqrt(d2)) - 40 : -126;
    return e < -126 ? -126 : (e > 127 ? 127 : e);
}

struct vor_grid {
    vrt::Grid g;
    DevAlloc alloc;                 // where its arrays came from
    std::vector<DevBlock> owned;    // ... and the arrays, returned by vor_grid_free
};

extern "C" vor_status vor_build_grid(const double *sites, int64_t M, const double *box, const vor_build_opts *opts,
                                     const vor_allocator *allocator, void *stream, vor_grid **out)
{
    if (out) *out = nullptr;
    if (!sites || !box || !out || M < 1 || M >= 0x7fffffffLL) return VOR_EINVAL;
    if (allocator && (!allocator->alloc || !allocator->free)) return VOR_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(box[a]) || !std::isfinite(box[a + 3]) || !(box[a] < box[a + 3])) return VOR_EINVAL;
    double occ = (opts && opts->bucket_occupancy > 0) ? opts->bucket_occupancy : 2.0;
    const bool want_loc = opts && opts->block_lists;
    const double locc = (opts && opts->block_occupancy > 0) ? opts->block_occupancy : 0.25;
    if (opts && (opts->block_lists < 0 || opts->block_lists > 1 || !(opts->block_occupancy >= 0))) return VOR_EINVAL;
    const int layout = opts ? opts->record_layout : VOR_RECORDS_AUTO;
    if (layout < VOR_RECORDS_AUTO || layout > VOR_RECORDS_COMPACT) return VOR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();

    vor_grid *G = new (std::nothrow) vor_grid;
    if (!G) return VOR_ENOMEM;
    Grid &g = G->g;
    G->alloc.custom = allocator != nullptr;
    if (allocator) G->alloc.a = *allocator;
    G->alloc.stream = stream;
    const DevAlloc &A = G->alloc;
    (void)hipGetDevice(&g.device);
    if (hipDeviceGetAttribute(&g.cus, hipDeviceAttributeMultiprocessorCount, g.device) != hipSuccess || g.cus < 1) {
        delete G;
        return VOR_EDEVICE;
    }
    g.M = M;
    for (int a = 0; a < 6; ++a) g.box[a] = box[a];

    vor_status rc = VOR_OK;
    std::vector<DevBlock> tmp, &keep = G->owned;
    BoxArg ba;
    for (int a = 0; a < 3; ++a) {
        ba.lo[a] = box[a];
        ba.hi[a] = box[a + 3];
    }
    double ext = std::max(box[3] - box[0], std::max(box[4] - box[1], box[5] - box[2]));
    double hscale = (double)(1 << kHilbertBits) / ext;

    int64_t hist_len = vrt_radix_hist_len(M);
    uint32_t *keys = dalloc<uint32_t>(M, rc, tmp, A);
    int32_t *vals = dalloc<int32_t>(M, rc, tmp, A);
    uint32_t *keys2 = dalloc<uint32_t>(M, rc, tmp, A);
    int32_t *vals2 = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *hist = dalloc<int32_t>(2 * hist_len + 1, rc, tmp, A);
    int *err = dalloc<int>(4, rc, tmp, A);
    g.sites = dalloc<Site>(M, rc, keep, A);
    g.perm = dalloc<int32_t>(M, rc, keep, A);
    g.inv_perm = dalloc<int32_t>(M, rc, keep, A);
    g.wall_mask = dalloc<uint8_t>(M, rc, keep, A);
    g.volume = dalloc<double>(M, rc, keep, A);
    g.rho_int = dalloc<double>(M, rc, keep, A);
    g.bucket_sites = dalloc<Site>(M, rc, keep, A);
    if (want_loc) g.bbox = dalloc<double>((size_t)M * 6, rc, keep, A);

    // bucket grid dimensions: about `occ` sites per bucket, cube-like buckets
    double vol = (box[3] - box[0]) * (box[4] - box[1]) * (box[5] - box[2]);
    double hb = std::cbrt(vol * occ / (double)M);
    int64_t B = 1;
    for (int a = 0; a < 3; ++a) {
        double e = box[a + 3] - box[a];
        int n = (int)std::ceil(e / hb);
        n = std::max(1, std::min(n, 1024));
        g.dims[a] = n;
        g.h[a] = e / n;
        g.inv_h[a] = n / e;
        B *= n;
    }
    int32_t *bcount = dalloc<int32_t>(B, rc, tmp, A);
    g.bucket_start = dalloc<int32_t>(B + 1, rc, keep, A);
    int32_t *nbr0 = dalloc<int32_t>((size_t)M * kMaxNbr, rc, tmp, A);
    int32_t *cnt0 = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *retry = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *slot = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *dir_start = dalloc<int32_t>(M + 1, rc, tmp, A);
    int32_t *extra = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *total = dalloc<int32_t>(M, rc, tmp, A);
    int32_t *start = dalloc<int32_t>(M + 1, rc, tmp, A);
    int *hdr = nullptr;

    auto fail = [&](vor_status s) {
        (void)hipStreamSynchronize(st);
        for (const DevBlock &b : tmp) A.put(b);
        for (const DevBlock &b : keep) A.put(b);
        delete G;
        return s;
    };
    if (rc != VOR_OK) return fail(rc);
    if (hipMemsetAsync(err, 0, 4 * sizeof(int), st) != hipSuccess) return fail(VOR_EDEVICE);

    const int T = 256;
    hipLaunchKernelGGL(k_validate_keys, dim3(blocks_for(M, T)), dim3(T), 0, st, sites, M, ba, hscale, keys, vals, err);
    int herr = 0;
    if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VOR_EDEVICE);
    if (herr & ERR_OUTSIDE) return fail(VOR_EOUTSIDE);

    rc = vrt_radix_sort_pairs(keys, vals, keys2, vals2, M, 3 * kHilbertBits, hist, hist_len, st);
    if (rc != VOR_OK) return fail(rc);
    hipLaunchKernelGGL(k_gather_sites, dim3(blocks_for(M, T)), dim3(T), 0, st, sites, vals, M, g.sites, g.perm,
                       g.inv_perm);

    // bucket the Hilbert-ordered sites (stable: within a bucket, Hilbert order)
    GridArg ga;
    for (int a = 0; a < 3; ++a) {
        ga.lo[a] = box[a];
        ga.inv_h[a] = g.inv_h[a];
        ga.dims[a] = g.dims[a];
    }
    if (hipMemsetAsync(bcount, 0, sizeof(int32_t) * B, st) != hipSuccess) return fail(VOR_EDEVICE);
    hipLaunchKernelGGL(k_bucket_keys, dim3(blocks_for(M, T)), dim3(T), 0, st, g.sites, M, ga, keys, vals, bcount);
    int bbits = 1;
    while ((1ll << bbits) < B) ++bbits;
    rc = vrt_radix_sort_pairs(keys, vals, keys2, vals2, M, bbits, hist, hist_len, st);
    if (rc != VOR_OK) return fail(rc);
    rc = vrt_scan_i32_to_i32(bcount, B, g.bucket_start, st);
    if (rc != VOR_OK) return fail(rc);
    hipLaunchKernelGGL(k_bucket_fill, dim3(blocks_for(M, T)), dim3(T), 0, st, g.sites, vals, M, g.bucket_sites);

    // clip every cell: small cells first, the overflowing ones again with large cells
    ClipArgs ca;
    ca.sites = g.sites;
    ca.grid = bucket_view(g);
    ca.box = ba;
    ca.M = M;
    ca.nbr = nbr0;
    ca.cnt = cnt0;
    ca.walls = g.wall_mask;
    ca.retry = retry;
    ca.n_retry = err + 2;
    ca.err = err;
    ca.volume = g.volume;
    ca.bbox = g.bbox;
    if (hipMemsetAsync(slot, 0xff, sizeof(int32_t) * M, st) != hipSuccess) return fail(VOR_EDEVICE);
    hipLaunchKernelGGL(k_clip, dim3((unsigned)M), dim3(64), 0, st, ca);
    if (hipGetLastError() != hipSuccess) return fail(VOR_EDEVICE);
    int hflags[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(hflags, err, 4 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VOR_EDEVICE);
    if (hflags[0] & ERR_DUP) return fail(VOR_EDUP);
    if (hflags[0] & (ERR_CAPACITY | ERR_DEGENERATE)) return fail(VOR_ECAPACITY);
    const int n_retry = hflags[2];
    int32_t *big_nbr = nullptr;
    if (n_retry > 0) {
        big_nbr = dalloc<int32_t>((size_t)n_retry * kMaxNbrBig, rc, tmp, A);
        if (rc != VOR_OK) return fail(rc);
        hipLaunchKernelGGL(k_clip_big, dim3((unsigned)n_retry), dim3(64), 0, st, ca, big_nbr, slot);
        if (hipMemcpyAsync(hflags, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(VOR_EDEVICE);
        if (hflags[0] & ERR_DUP) return fail(VOR_EDUP);
        if (hflags[0] & (ERR_CAPACITY | ERR_DEGENERATE)) return fail(VOR_ECAPACITY);
    }
    g.n_big = n_retry;

    // directed lists as CSR
    rc = vrt_scan_i32_to_i32(cnt0, M, dir_start, st);
    if (rc != VOR_OK) return fail(rc);
    int32_t nnz_dir = 0;
    if (hipMemcpyAsync(&nnz_dir, dir_start + M, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VOR_EDEVICE);
    int32_t *dir_col = dalloc<int32_t>(std::max<int32_t>(nnz_dir, 1), rc, tmp, A);
    if (rc != VOR_OK) return fail(rc);
    hipLaunchKernelGGL(k_gather_dir, dim3(blocks_for(M, T)), dim3(T), 0, st, nbr0, cnt0, dir_start, slot, M, big_nbr,
                       dir_col);

    // symmetric lists: add the reverse of every one-sided entry, sort rows
    if (hipMemsetAsync(extra, 0, sizeof(int32_t) * M, st) != hipSuccess) return fail(VOR_EDEVICE);
    hipLaunchKernelGGL(k_symm_count, dim3(blocks_for(M, T)), dim3(T), 0, st, dir_col, dir_start, cnt0, M, extra);
    hipLaunchKernelGGL(k_total_counts, dim3(blocks_for(M, T)), dim3(T), 0, st, cnt0, extra, M, total);
    rc = vrt_scan_i32_to_i32(total, M, start, st);
    if (rc != VOR_OK) return fail(rc);
    int32_t nnz32 = 0;
    if (hipMemcpyAsync(&nnz32, start + M, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VOR_EDEVICE);
    g.nnz = nnz32;
    int32_t *col = dalloc<int32_t>(std::max<int32_t>(nnz32, 1), rc, tmp, A);
    if (rc != VOR_OK) return fail(rc);
    hipLaunchKernelGGL(k_copy_rows, dim3(blocks_for(M, T)), dim3(T), 0, st, dir_col, dir_start, cnt0, start, M, col,
                       extra);
    hipLaunchKernelGGL(k_symm_fill, dim3(blocks_for(M, T)), dim3(T), 0, st, dir_col, dir_start, cnt0, start, M, col,
                       extra);
    hipLaunchKernelGGL(k_row_sort, dim3(blocks_for(M, T)), dim3(T), 0, st, col, start, total, M);

    // cell blocks are addressed by 32-bit slot offsets; FP32 blocks take
    // kHdrSlots + n slots, compact ones kHdrSlots + ceil(3n / 4)
    int64_t nslots = g.nnz + (int64_t)kHdrSlots * M;
    if (nslots + kRecPad > 0x7fffffffLL) return fail(VOR_ECAPACITY);   // compact blocks take no more slots
    g.compact = layout == VOR_RECORDS_COMPACT || (layout == VOR_RECORDS_AUTO && nslots * 16 > kCompactAutoBytes);
    if (g.compact) {   // blocks not at rows[j].x + 3j: their starts are kept
        g.blk_off = dalloc<int32_t>(M + 1, rc, keep, A);
        if (rc != VOR_OK) return fail(rc);
        hipLaunchKernelGGL(k_compact_slots, dim3(blocks_for(M, T)), dim3(T), 0, st, total, M, slot);
        rc = vrt_scan_i32_to_i32(slot, M, g.blk_off, st);
        if (rc != VOR_OK) return fail(rc);
        int32_t ns = 0;
        if (hipMemcpyAsync(&ns, g.blk_off + M, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(VOR_EDEVICE);
        nslots = ns;
    }
    if (nslots + kRecPad > 0x7fffffffLL) return fail(VOR_ECAPACITY);
    g.rows = dalloc<int2>(M, rc, keep, A);
    g.rec64 = dalloc<Rec64>(g.nnz + kRecPad, rc, keep, A);
    g.blk = dalloc<Slot>(nslots + kRecPad, rc, keep, A);
    if (rc != VOR_OK) return fail(rc);
    if (hipMemsetAsync(g.rec64 + g.nnz, 0, sizeof(Rec64) * kRecPad, st) != hipSuccess ||
        hipMemsetAsync(g.blk + nslots, 0, sizeof(Slot) * kRecPad, st) != hipSuccess)
        return fail(VOR_EDEVICE);
    hdr = err + 1;   // longest row
    hipLaunchKernelGGL(k_fill_records, dim3(blocks_for(M, T)), dim3(T), 0, st, g.sites, col, total, start, M, g.rows,
                       g.rec64, g.blk, g.blk_off, (int)g.compact, compact_min_exp(g.box), hdr);
    // the FP64 blocks: at most 4 + 7n/4 slots per cell
    if ((int64_t)4 * M + 2 * g.nnz + kRecPad > 0x7fffffffLL) return fail(VOR_ECAPACITY);
    g.blk64_off = dalloc<int32_t>(M + 1, rc, keep, A);
    if (rc != VOR_OK) return fail(rc);
    hipLaunchKernelGGL(k_fp64_slots, dim3(blocks_for(M, T)), dim3(T), 0, st, g.rows, M, slot);
    rc = vrt_scan_i32_to_i32(slot, M, g.blk64_off, st);
    if (rc != VOR_OK) return fail(rc);
    int32_t ns64 = 0;
    if (hipMemcpyAsync(&ns64, g.blk64_off + M, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(VOR_EDEVICE);
    g.nslots64 = ns64;
    g.blk64 = dalloc<Slot>((int64_t)ns64 + kRecPad, rc, keep, A);
    if (rc != VOR_OK) return fail(rc);
    if (hipMemsetAsync(g.blk64 + ns64, 0, sizeof(Slot) * kRecPad, st) != hipSuccess) return fail(VOR_EDEVICE);
    hipLaunchKernelGGL(k_fill_blk64, dim3(blocks_for(M, T)), dim3(T), 0, st, g.sites, g.rows, g.rec64, g.blk64_off, M,
                       g.blk64);
    // size of the export with walls
    hipLaunchKernelGGL(k_export_counts, dim3(blocks_for(M, T)), dim3(T), 0, st, g.inv_perm, g.rows, g.wall_mask, M,
                       total);
    rc = vrt_scan_i32_to_i32(total, M, start, st);
    if (rc != VOR_OK) return fail(rc);
    int32_t nnzw = 0, mrow = 0;
    if (hipMemcpyAsync(&nnzw, start + M, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&mrow, hdr, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
        return fail(VOR_EDEVICE);
    g.nnz_walls = nnzw;
    g.max_row = mrow;

    if (want_loc) {
        // blocks: about M / locc of them, cube-like
        LocArgs la;
        la.bbox = g.bbox;
        la.M = M;
        const double hl = std::cbrt(vol * locc / (double)M);
        int64_t K = 1;
        for (int a = 0; a < 3; ++a) {
            const double e = box[a + 3] - box[a];
            const int n = std::max(1, std::min((int)std::ceil(e / hl), 1024));
            g.loc_dims[a] = la.dims[a] = n;
            g.loc_inv_h[a] = la.inv_h[a] = n / e;
            la.lo[a] = box[a];
            la.ext[a] = e;
            K *= n;
        }
        if (K >= 0x7fffffffLL) return fail(VOR_ECAPACITY);
        int32_t *lcnt = dalloc<int32_t>(K, rc, tmp, A);
        unsigned long long *ltot = dalloc<unsigned long long>(1, rc, tmp, A);
        g.loc_start = dalloc<int32_t>(K + 1, rc, keep, A);
        if (rc != VOR_OK) return fail(rc);
        if (hipMemsetAsync(lcnt, 0, sizeof(int32_t) * K, st) != hipSuccess ||
            hipMemsetAsync(ltot, 0, sizeof(unsigned long long), st) != hipSuccess)
            return fail(VOR_EDEVICE);
        hipLaunchKernelGGL(k_loc_count, dim3(blocks_for(M, T)), dim3(T), 0, st, la, lcnt, ltot);
        unsigned long long entries = 0;
        if (hipMemcpyAsync(&entries, ltot, sizeof(entries), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
            return fail(VOR_EDEVICE);
        if (entries >= 0x7fffffffULL) return fail(VOR_ECAPACITY);
        rc = vrt_scan_i32_to_i32(lcnt, K, g.loc_start, st);
        if (rc != VOR_OK) return fail(rc);
        g.loc_cells = dalloc<int32_t>(std::max<unsigned long long>(entries, 1), rc, keep, A);
        if (rc != VOR_OK) return fail(rc);
        if (hipMemsetAsync(lcnt, 0, sizeof(int32_t) * K, st) != hipSuccess) return fail(VOR_EDEVICE);
        hipLaunchKernelGGL(k_loc_fill, dim3(blocks_for(M, T)), dim3(T), 0, st, la, g.loc_start, lcnt, g.loc_cells);
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) return fail(VOR_EDEVICE);
        g.loc_entries = (int64_t)entries;
    }

    if (hipStreamSynchronize(st) != hipSuccess) return fail(VOR_EDEVICE);
    for (const DevBlock &b : tmp) A.put(b);
    tmp.clear();
    g.device_bytes = (int64_t)M * (sizeof(Site) * 2 + 4 * 2 + 1 + sizeof(int2) + 2 * sizeof(double)) + (B + 1) * 4 +
                     (g.nnz + kRecPad) * (int64_t)sizeof(Rec64) + (nslots + kRecPad) * (int64_t)sizeof(Slot) +
                     (g.blk_off ? (M + 1) * 4 : 0) + (g.nslots64 + kRecPad) * (int64_t)sizeof(Slot) + (M + 1) * 4;
    if (want_loc)
        g.device_bytes += (int64_t)M * 6 * (int64_t)sizeof(double) +
                          ((int64_t)g.loc_dims[0] * g.loc_dims[1] * g.loc_dims[2] + 1 + g.loc_entries) * 4;
    g.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = G;
    return VOR_OK;
}

extern "C" void vor_grid_free(vor_grid *G)
{
    if (!G) return;
    (void)hipDeviceSynchronize();
    for (const DevBlock &b : G->owned) G->alloc.put(b);
    delete G;
}

extern "C" vor_status vor_grid_get_info(const vor_grid *G, vor_grid_info *info)
{
    if (!G || !info) return VOR_EINVAL;
    const Grid &g = G->g;
    info->n_sites = g.M;
    info->nnz = g.nnz;
    info->nnz_with_walls = g.nnz_walls;
    info->max_row = g.max_row;
    for (int a = 0; a < 3; ++a) info->dims[a] = g.dims[a];
    for (int a = 0; a < 6; ++a) info->box[a] = g.box[a];
    info->build_ms = g.build_ms;
    info->device_bytes = g.device_bytes;
    for (int a = 0; a < 3; ++a) info->block_dims[a] = g.loc_dims[a];
    info->block_entries = g.loc_entries;
    info->record_layout = g.compact ? VOR_RECORDS_COMPACT : VOR_RECORDS_FP32;
    return VOR_OK;
}

extern "C" vor_status vor_grid_neighbors(const vor_grid *G, int64_t *row_ptr, int32_t *col, void *stream)
{
    if (!G || !row_ptr || (!col && G->g.nnz_walls > 0)) return VOR_EINVAL;
    const Grid &g = G->g;
    hipStream_t st = (hipStream_t)stream;
    // per-row counts are staged in col, which holds at least M entries
    // (every clipped cell has at least one face)
    if (g.nnz_walls < g.M) return VOR_EINVAL;
    const int T = 256;
    hipLaunchKernelGGL(k_export_counts, dim3(blocks_for(g.M, T)), dim3(T), 0, st, g.inv_perm, g.rows, g.wall_mask,
                       g.M, col);
    vor_status rc = vrt_scan_i32_to_i64(col, g.M, row_ptr, st);
    if (rc != VOR_OK) return rc;
    hipLaunchKernelGGL(k_export_fill, dim3(blocks_for(g.M, T)), dim3(T), 0, st, g.inv_perm, g.perm, g.rows, g.rec64,
                       g.wall_mask, g.M, row_ptr, col);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

extern "C" vor_status vor_grid_truncate_row(vor_grid *G, int64_t site, int32_t keep)
{
    if (!G || site < 0 || site >= G->g.M || keep < 0) return VOR_EINVAL;
    Grid &g = G->g;
    int32_t i = 0;
    int2 rw;
    if (hipMemcpy(&i, g.inv_perm + site, sizeof(i), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&rw, g.rows + i, sizeof(rw), hipMemcpyDeviceToHost) != hipSuccess)
        return VOR_EDEVICE;
    if (keep < rw.y) {
        // the block offsets follow the records (12 or 8 bytes each): move the
        // first keep of them to their place after the first keep records
        int32_t bo = block_of(rw, i);
        if (g.blk_off && hipMemcpy(&bo, g.blk_off + i, sizeof(bo), hipMemcpyDeviceToHost) != hipSuccess)
            return VOR_EDEVICE;
        char *rec = reinterpret_cast<char *>(g.blk + bo + kHdrSlots);
        const int rbytes = g.compact ? 8 : 12;
        std::vector<int32_t> nb(keep > 0 ? keep : 1);
        if (keep > 0 && (hipMemcpy(nb.data(), rec + rbytes * rw.y, sizeof(int32_t) * keep, hipMemcpyDeviceToHost) !=
                             hipSuccess ||
                         hipMemcpy(rec + rbytes * keep, nb.data(), sizeof(int32_t) * keep, hipMemcpyHostToDevice) !=
                             hipSuccess))
            return VOR_EDEVICE;
        BlockHdr *h = reinterpret_cast<BlockHdr *>(g.blk + bo);
        int32_t len = 0;
        if (hipMemcpy(&len, &h->len, sizeof(len), hipMemcpyDeviceToHost) != hipSuccess) return VOR_EDEVICE;
        len = (len & ~kLenMask) | keep;   // the scale exponent stays
        // the same in the FP64 block (24-byte records)
        int32_t bo64 = 0;
        if (hipMemcpy(&bo64, g.blk64_off + i, sizeof(bo64), hipMemcpyDeviceToHost) != hipSuccess) return VOR_EDEVICE;
        char *rec64 = reinterpret_cast<char *>(g.blk64 + bo64 + kHdrSlots);
        if (keep > 0 && (hipMemcpy(nb.data(), rec64 + 24 * rw.y, sizeof(int32_t) * keep, hipMemcpyDeviceToHost) !=
                             hipSuccess ||
                         hipMemcpy(rec64 + 24 * keep, nb.data(), sizeof(int32_t) * keep, hipMemcpyHostToDevice) !=
                             hipSuccess))
            return VOR_EDEVICE;
        BlockHdr *h64 = reinterpret_cast<BlockHdr *>(g.blk64 + bo64);
        rw.y = keep;
        if (hipMemcpy(g.rows + i, &rw, sizeof(rw), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(&h->len, &len, sizeof(len), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(&h64->len, &keep, sizeof(keep), hipMemcpyHostToDevice) != hipSuccess)
            return VOR_EDEVICE;
    }
    return VOR_OK;
}

__global__ void k_export_bboxes(const int32_t *__restrict__ perm, const double *__restrict__ bb, int64_t M,
                                double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int64_t u = perm[i];
    for (int a = 0; a < 6; ++a) out[6 * u + a] = bb[6 * i + a];
}

extern "C" vor_status vor_grid_bboxes(const vor_grid *G, double *bbox, void *stream)
{
    if (!G || !bbox || !G->g.bbox) return VOR_EINVAL;
    const Grid &g = G->g;
    const int T = 256;
    hipLaunchKernelGGL(k_export_bboxes, dim3(blocks_for(g.M, T)), dim3(T), 0, (hipStream_t)stream, g.perm, g.bbox,
                       g.M, bbox);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

__global__ void k_bind_density(Slot *__restrict__ blk, Slot *__restrict__ blk64, const int2 *__restrict__ rows,
                               const int32_t *__restrict__ blk_off, const int32_t *__restrict__ blk64_off,
                               const int32_t *__restrict__ perm, int64_t M, const double *__restrict__ density,
                               double *__restrict__ rho_int)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double r = density ? density[perm[i]] : 0.0;
    const int32_t bo = blk_off ? blk_off[i] : block_of(rows[i], (int32_t)i);
    reinterpret_cast<BlockHdr *>(blk + bo)->rho = r;
    reinterpret_cast<BlockHdr *>(blk64 + blk64_off[i])->rho = r;
    rho_int[i] = r;
}

extern "C" vor_status vor_grid_bind_density(vor_grid *G, const double *density, void *stream)
{
    if (!G) return VOR_EINVAL;
    Grid &g = G->g;
    const int T = 256;
    hipLaunchKernelGGL(k_bind_density, dim3(blocks_for(g.M, T)), dim3(T), 0, (hipStream_t)stream, g.blk, g.blk64,
                       g.rows, g.blk_off, g.blk64_off, g.perm, g.M, density, g.rho_int);
    if (hipGetLastError() != hipSuccess) return VOR_EDEVICE;
    g.rho_bound = density ? 1 : 0;
    return VOR_OK;
}

__global__ void k_export_volumes(const int32_t *__restrict__ perm, const double *__restrict__ vol, int64_t M,
                                 double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[perm[i]] = vol[i];
}

extern "C" vor_status vor_grid_volumes(const vor_grid *G, double *volume, void *stream)
{
    if (!G || !volume) return VOR_EINVAL;
    const Grid &g = G->g;
    const int T = 256;
    hipLaunchKernelGGL(k_export_volumes, dim3(blocks_for(g.M, T)), dim3(T), 0, (hipStream_t)stream, g.perm, g.volume,
                       g.M, volume);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

// accessor for the other translation units
const vrt::Grid &vrt_grid_of(const vor_grid *G) { return G->g; }
