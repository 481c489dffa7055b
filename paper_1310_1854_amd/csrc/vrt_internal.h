// vrt_internal.h -- device data layout and helpers shared by the HIP sources
// of libvoronoi_rt. Not part of the public ABI (include/voronoi_rt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define VRT_HD __host__ __device__

#include "../../include/voronoi_rt.h"

namespace vrt {

// FP64 neighbour record: the neighbour's site, its internal (Hilbert-order)
// index and its user index. A row of these per cell is all the exit-point
// search reads (Sect. 2.2: the current cell's neighbour indices and sites).
struct __align__(32) Rec64 {
    double x, y, z;
    int32_t j;    // internal index of the neighbour
    int32_t uid;  // user index of the neighbour
};

// The 16-byte slot of the cell blocks.
struct __align__(16) Slot {
    uint32_t w[4];
};

// Cell blocks of the mixed-precision search, one per cell in internal
// order, in 16-byte slots: a header of kHdrSlots slots, then the cell's row
// of n neighbours as n FP32 records of 12 bytes (the offset p_j - p_m
// rounded to FP32), then the n block offsets of those neighbours (int32):
// 48 + 16 n bytes, so the block of cell j starts at slot
// rows[j].x + kHdrSlots * j. The search reads the records only (8 of them
// are 6 aligned 16-byte loads) and the block offset of the winner alone.
// What a step needs of the cell it moves into (its FP64 site, indices, row
// and bound density) lies in the lines of its first records.
// A grid may instead use compact blocks (Grid::compact): the same header,
// then n records of 8 bytes -- the offset p_j - p_m as three 21-bit signed
// integers q (x in bits 0-20, y in 21-41, z in 42-62) with
// p_j - p_m ~= q * 2^(E - 19), E the cell's scale exponent (the largest
// offset component is below 2^E) -- then the n block offsets; each block is
// padded to whole slots and its start is kept in Grid::blk_off.
constexpr int kHdrSlots = 3;
struct __align__(16) BlockHdr {
    double x, y, z;   // the site
    double rho;       // the density bound to the grid (vor_grid_bind_density), 0 when none
    int32_t uid;      // user index
    int32_t j;        // internal index
    int32_t len;      // records that follow (bits 0-23); compact blocks: E + 128 in bits 24-31
    int32_t row;      // start of the cell's row of FP64 records (rows[j].x)
};
constexpr int32_t kLenMask = 0xffffff;
constexpr int kScaleBias = 128;
constexpr int kQBits = 21;     // bits per component of a compact record
constexpr int kQShift = 19;    // q = rint(offset * 2^(19 - E)), |q| <= 2^19
static_assert(sizeof(BlockHdr) == 16 * kHdrSlots, "a block header fills kHdrSlots slots");
static_assert(offsetof(BlockHdr, z) == 16 && offsetof(BlockHdr, rho) == 24 && offsetof(BlockHdr, uid) == 32 &&
                  offsetof(BlockHdr, j) == 36 && offsetof(BlockHdr, len) == 40,
              "the trace reads the header as three 16-byte slots");

__host__ __device__ inline int32_t block_of(int2 row, int32_t j) { return row.x + kHdrSlots * j; }

// Site in internal order with its user index (the w slot holds the index
// bits so that one 32-byte load fetches both).
struct __align__(32) Site {
    double x, y, z;
    int64_t uid;
};

// Records readable past the end of the last row (zeroed): the exit search
// loads whole batches and masks the entries past a row's end.
constexpr int kRecPad = 16;

struct Grid {
    int64_t M = 0;
    int64_t nnz = 0;
    int64_t nnz_walls = 0;
    int32_t max_row = 0;
    int32_t n_big = 0;     // cells built with the large capacity
    double box[6];
    // uniform bucket grid of sites
    int32_t dims[3];
    double inv_h[3];   // buckets per unit length on each axis
    double h[3];       // bucket side on each axis
    // device arrays (internal order unless stated)
    Site *sites = nullptr;          // [M]
    int32_t *perm = nullptr;        // [M] internal -> user
    int32_t *inv_perm = nullptr;    // [M] user -> internal
    int2 *rows = nullptr;           // [M] {start, count} into rec64
    Rec64 *rec64 = nullptr;         // [nnz + kRecPad]
    Slot *blk = nullptr;           // [nnz + kHdrSlots M + kRecPad] cell blocks (headers, FP32 records, block offsets)
    uint8_t *wall_mask = nullptr;   // [M] bit w set if wall -(w+1) is a face
    double *volume = nullptr;       // [M] volume of each clipped cell
    int32_t *bucket_start = nullptr;// [B + 1]
    Site *bucket_sites = nullptr;   // [M] sites grouped by bucket (uid holds the internal index)
    // the paper's locate structure (Sect. 2.3), built on request: a regular
    // grid of blocks over the box, each listing the cells whose bounding box
    // overlaps it
    double *bbox = nullptr;         // [6 M] cell bounding boxes {min xyz, max xyz}
    int32_t loc_dims[3] = {0, 0, 0};
    double loc_inv_h[3] = {0, 0, 0};
    int32_t *loc_start = nullptr;   // [K + 1] list of block k: loc_cells[loc_start[k] .. loc_start[k+1])
    int32_t *loc_cells = nullptr;   // internal cell indices
    int64_t loc_entries = 0;
    int32_t rho_bound = 0;          // a density is bound (block headers and rho_int)
    double *rho_int = nullptr;      // [M] the bound density in internal order (FP64 mode reads it here)
    int32_t compact = 0;            // cell blocks with 8-byte fixed-point records
    int32_t *blk_off = nullptr;     // [M + 1] compact blocks: the slot where each cell's block starts
    // FP64 cell blocks (FP64-mode steps): the same header, then the n
    // neighbour sites in FP64 (24 bytes each), then their FP64 block offsets
    Slot *blk64 = nullptr;          // [nslots64 + kRecPad]
    int32_t *blk64_off = nullptr;   // [M + 1] where each cell's FP64 block starts
    int64_t nslots64 = 0;
    double build_ms = 0;
    int64_t device_bytes = 0;
    int device = 0;
    int cus = 0;                    // compute units of that device (sizes the persistent launches)
};

// Per-ray status codes (same values as VOR_RAY_*).
constexpr uint8_t RAY_OK = 0, RAY_OUTSIDE = 1, RAY_BADDIR = 2, RAY_STEPLIMIT = 3, RAY_OVERFLOW = 4;

// Bucket coordinate of a point on one axis, clamped to the grid.
VRT_HD inline int bucket_coord(double x, double lo, double inv_h, int n)
{
    int b = (int)floor((x - lo) * inv_h);
    return b < 0 ? 0 : (b >= n ? n - 1 : b);
}

struct BucketGridView {
    double lo[3];
    double hi[3];
    double inv_h[3];
    double h[3];
    int32_t dims[3];
    const int32_t *start;
    const Site *items;
};

inline BucketGridView bucket_view(const Grid &g)
{
    BucketGridView v;
    for (int a = 0; a < 3; ++a) {
        v.lo[a] = g.box[a];
        v.hi[a] = g.box[a + 3];
        v.inv_h[a] = g.inv_h[a];
        v.h[a] = g.h[a];
        v.dims[a] = g.dims[a];
    }
    v.start = g.bucket_start;
    v.items = g.bucket_sites;
    return v;
}

// Lower bound on the distance from q to any point of the grid outside the
// block of buckets within Chebyshev distance r of bucket b. Sides of the
// block that reach the edge of the grid hold nothing beyond them and impose
// no bound; if every side does, the block covers the grid (returns -1).
VRT_HD inline double shell_bound(const BucketGridView &g, const double q[3], const int b[3], int r)
{
    double lb = 1e308;
    bool open = false;
    for (int a = 0; a < 3; ++a) {
        if (b[a] - r > 0) {
            double face = g.lo[a] + (double)(b[a] - r) * g.h[a];
            double d = q[a] - face;
            lb = fmin(lb, d);
            open = true;
        }
        if (b[a] + r < g.dims[a] - 1) {
            double face = g.lo[a] + (double)(b[a] + r + 1) * g.h[a];
            double d = face - q[a];
            lb = fmin(lb, d);
            open = true;
        }
    }
    if (!open) return -1.0;
    return lb < 0.0 ? 0.0 : lb;
}

// Visit every bucket at Chebyshev distance exactly r from b (clipped to the
// grid) and call f(bucket_linear_index).
template <typename F>
VRT_HD inline void for_shell(const BucketGridView &g, const int b[3], int r, F &&f)
{
    const int nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    int z0 = b[2] - r > 0 ? b[2] - r : 0, z1 = b[2] + r < nz - 1 ? b[2] + r : nz - 1;
    int y0 = b[1] - r > 0 ? b[1] - r : 0, y1 = b[1] + r < ny - 1 ? b[1] + r : ny - 1;
    int x0 = b[0] - r > 0 ? b[0] - r : 0, x1 = b[0] + r < nx - 1 ? b[0] + r : nx - 1;
    for (int z = z0; z <= z1; ++z) {
        bool zface = (z == b[2] - r) || (z == b[2] + r);
        for (int y = y0; y <= y1; ++y) {
            bool yface = (y == b[1] - r) || (y == b[1] + r);
            if (zface || yface || r == 0) {
                for (int x = x0; x <= x1; ++x) f((z * ny + y) * nx + x);
            } else {
                if (b[0] - r >= 0) f((z * ny + y) * nx + (b[0] - r));
                if (b[0] + r <= nx - 1 && r > 0) f((z * ny + y) * nx + (b[0] + r));
            }
        }
    }
}

// Exact nearest site (internal index) by ring search; squared distances in
// the same operation order as a plain (x-p)^2 sum; equal distances go to
// the lower user index. q must be inside the box.
// STOP_AT_SITE: end the search when the point is a site (no other is as
// near: the sites are distinct), as rays that start at sites do.
template <bool STOP_AT_SITE = false>
VRT_HD inline int32_t nearest_site(const BucketGridView &g, const double q[3], int32_t *uid_out)
{
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(q[a], g.lo[a], g.inv_h[a], g.dims[a]);
    double best = 1e308 * 10.0;  // +inf
    int32_t best_i = -1;
    int32_t best_u = 0x7fffffff;
    bool at_site = false;
    auto visit = [&](const Site &p) {
        double dx = q[0] - p.x, dy = q[1] - p.y, dz = q[2] - p.z;
        double d = dx * dx + dy * dy + dz * dz;
        int32_t idx = (int32_t)(p.uid & 0xffffffff);
        int32_t uid = (int32_t)(p.uid >> 32);
        if (d < best || (d == best && uid < best_u)) {
            best = d;
            best_i = idx;
            best_u = uid;
        }
        return dx == 0.0 && dy == 0.0 && dz == 0.0;
    };
    for (int r = 0;; ++r) {
        for_shell(g, b, r, [&](int bk) {
            int s0 = g.start[bk], s1 = g.start[bk + 1];
            if constexpr (STOP_AT_SITE) {   // four sites per round, loaded together
                for (int s = s0; s < s1 && !at_site; s += 4) {
                    const int n = (s1 - s < 4) ? s1 - s : 4;
                    Site p[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j < n) p[j] = g.items[s + j];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j < n) at_site |= visit(p[j]);
                }
            } else {
                for (int s = s0; s < s1; ++s) visit(g.items[s]);
            }
        });
        if (STOP_AT_SITE && at_site) break;
        double lb = shell_bound(g, q, b, r);
        if (lb < 0.0) break;
        // sites outside the block are at least lb away; the slack keeps a
        // rounding of lb from ending the search early
        double lb2 = lb * lb * (1.0 - 1e-12);
        if (best < lb2) break;
    }
    if (uid_out) *uid_out = best_u;
    return best_i;
}

constexpr int kHilbertBits10 = 10;   // bits per axis of the Hilbert keys

// Hilbert index of a point with kHilbertBits10-bit integer coordinates, by
// Skilling's transform ("Programming the Hilbert curve", AIP Conf. Proc.
// 707, 2004): undo the excess work of the recursion, Gray-encode, then
// interleave the bits of the three transposed coordinates.
__device__ __forceinline__ uint32_t hilbert_key(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t X[3] = {x, y, z};
    const uint32_t top = 1u << (kHilbertBits10 - 1);
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint32_t key = 0;
    for (int b = kHilbertBits10 - 1; b >= 0; --b)
        key = (key << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) | ((X[2] >> b) & 1u);
    return key;
}


inline bool cuda_ok(hipError_t e) { return e == hipSuccess; }

}  // namespace vrt

// scan.hip
vor_status vrt_scan_i32_to_i64(const int32_t *counts, int64_t N, int64_t *offsets, hipStream_t st);
vor_status vrt_scan_i32_to_i32(const int32_t *counts, int64_t N, int32_t *offsets, hipStream_t st);
// sort.hip: stable LSD radix sort of (key, value) pairs, 32-bit keys of `bits` significant bits
vor_status vrt_radix_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp,
                                int64_t n, int bits, int32_t *hist_scratch, int64_t hist_len, hipStream_t st);
int64_t vrt_radix_hist_len(int64_t n);
// dst[i] = src[idx[i]]
vor_status vrt_gather_u32(const uint32_t *src, const int32_t *idx, int64_t n, uint32_t *dst, hipStream_t st);
// trace.hip: whole paths from segment windows and spill chains into compact rows (vor_gather_paths)
vor_status vrt_gather_paths(const int32_t *n_seg, int64_t n, const int32_t *wcell, const double *wlen, int64_t stride,
                            const int64_t *first, const int32_t *next, const int32_t *pcell, const double *plen,
                            const int64_t *ray_off, int32_t *cell, double *len, hipStream_t st);
