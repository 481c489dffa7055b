// locate_core.h -- the cell-location function C(r) (Sect. 2.3) on the device,
// shared by the trace and the serving start passes: the paper's block lists
// and the bucket-grid ring search, per lane or for a point a whole wave
// shares.
#pragma once

#include "vrt_internal.h"

namespace vrt {

// C(r) through the paper's block lists (Sect. 2.3, steps 2-4), for a point
// inside the closed box: the block holding the point, then the nearest site
// among the cells listed for that block (equal distances: the lowest user
// index). The cell holding the point is listed there, so this is the
// nearest site of all. Returns the internal index (-1 for an empty list,
// which a point inside the box cannot meet) and the user index in *uid.
struct LocView {
    double lo[3], hi[3], inv_h[3];
    int32_t dims[3];
    const int32_t *start;   // null: the grid has no block lists
    const int32_t *cells;
    const Site *sites;
};

inline LocView loc_view(const Grid &g)
{
    LocView L;
    for (int a = 0; a < 3; ++a) {
        L.lo[a] = g.box[a];
        L.hi[a] = g.box[a + 3];
        L.inv_h[a] = g.loc_inv_h[a];
        L.dims[a] = g.loc_dims[a];
    }
    L.start = g.loc_start;
    L.cells = g.loc_cells;
    L.sites = g.sites;
    return L;
}

// STOP_AT_SITE: the search ends at a site the point coincides with (no
// other is as near), and takes the list four entries per round, their
// indices and sites loaded together (the minimum does not depend on the
// order the entries are seen in); the one-at-a-time loop of the other
// instance holds fewer registers in the kernels that inline it.
template <bool STOP_AT_SITE = false>
__device__ __forceinline__ int32_t nearest_in_blocks(const LocView &L, const double q[3], int32_t *uid)
{
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(q[a], L.lo[a], L.inv_h[a], L.dims[a]);
    const int64_t k = ((int64_t)b[0] * L.dims[1] + b[1]) * L.dims[2] + b[2];
    double best = __builtin_huge_val();
    int32_t best_u = -1, best_m = -1;
    auto visit = [&](int32_t m, const Site &p) {
        const double dx = q[0] - p.x, dy = q[1] - p.y, dz = q[2] - p.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        const int32_t u = (int32_t)p.uid;
        if (d2 < best || (d2 == best && u < best_u)) {
            best = d2;
            best_u = u;
            best_m = m;
        }
        return dx == 0.0 && dy == 0.0 && dz == 0.0;
    };
    const int s0 = L.start[k], s1 = L.start[k + 1];
    if constexpr (STOP_AT_SITE) {
#ifndef VRT_LOC_BATCH
#define VRT_LOC_BATCH 4
#endif
        constexpr int kBatch = VRT_LOC_BATCH;
        for (int s = s0; s < s1; s += kBatch) {
            int32_t m[kBatch];
            Site p[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) m[j] = (s + j < s1) ? L.cells[s + j] : -1;
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (m[j] >= 0) p[j] = L.sites[m[j]];
            bool at_site = false;
#pragma unroll
            for (int j = 0; j < kBatch; ++j)
                if (m[j] >= 0) at_site |= visit(m[j], p[j]);
            if (at_site) break;
        }
    } else {
        for (int s = s0; s < s1; ++s) {
            const int32_t m = L.cells[s];
            visit(m, L.sites[m]);
        }
    }
    *uid = best_u;
    return best_m;
}

// The same search by a whole wave for one point shared by its 64 lanes:
// the lanes take the list in turn, then the best (distance, user index) is
// reduced across the wave. Returns the internal index on every lane.
__device__ __forceinline__ int32_t nearest_in_blocks_wave(const LocView &L, const double q[3])
{
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(q[a], L.lo[a], L.inv_h[a], L.dims[a]);
    const int64_t k = ((int64_t)b[0] * L.dims[1] + b[1]) * L.dims[2] + b[2];
    double best = __builtin_huge_val();
    int32_t best_u = 0x7fffffff, best_m = -1;
    for (int s = L.start[k] + (int)(threadIdx.x & 63); s < L.start[k + 1]; s += 64) {
        const int32_t m = L.cells[s];
        const Site p = L.sites[m];
        const double dx = q[0] - p.x, dy = q[1] - p.y, dz = q[2] - p.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        const int32_t u = (int32_t)p.uid;
        if (d2 < best || (d2 == best && u < best_u)) {
            best = d2;
            best_u = u;
            best_m = m;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int32_t ou = __shfl_xor(best_u, off, 64);
        const int32_t om = __shfl_xor(best_m, off, 64);
        if (ob < best || (ob == best && ou < best_u)) {
            best = ob;
            best_u = ou;
            best_m = om;
        }
    }
    return best_m;
}

// nearest_site for a point shared by the whole wave: the sites of each
// bucket are split over the 64 lanes, and after each shell the lanes agree
// on the lexicographic minimum of (squared distance, user index). The
// shells visited, the distances and the minimum are those of nearest_site.
__device__ inline int32_t nearest_site_wave(const BucketGridView &g, const double q[3], int32_t *uid_out)
{
    const int lane = threadIdx.x & 63;
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(q[a], g.lo[a], g.inv_h[a], g.dims[a]);
    double best = 1e308 * 10.0;
    int32_t best_i = -1;
    int32_t best_u = 0x7fffffff;
    for (int r = 0;; ++r) {
        for_shell(g, b, r, [&](int bk) {
            const int s0 = g.start[bk], s1 = g.start[bk + 1];
            for (int s = s0 + lane; s < s1; s += 64) {
                const Site p = g.items[s];
                const double dx = q[0] - p.x, dy = q[1] - p.y, dz = q[2] - p.z;
                const double d = dx * dx + dy * dy + dz * dz;
                const int32_t idx = (int32_t)(p.uid & 0xffffffff);
                const int32_t uid = (int32_t)(p.uid >> 32);
                if (d < best || (d == best && uid < best_u)) {
                    best = d;
                    best_i = idx;
                    best_u = uid;
                }
            }
        });
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int32_t ou = __shfl_xor(best_u, off, 64);
            const int32_t oi = __shfl_xor(best_i, off, 64);
            if (ob < best || (ob == best && ou < best_u)) {
                best = ob;
                best_u = ou;
                best_i = oi;
            }
        }
        const double lb = shell_bound(g, q, b, r);
        if (lb < 0.0) break;
        const double lb2 = lb * lb * (1.0 - 1e-12);
        if (best < lb2) break;
    }
    if (uid_out) *uid_out = best_u;
    return best_i;
}

// The start cell of the ray on each lane, whose path starts at q (ok: the
// ray has a path; else -1): through the block lists when the grid has them
// (a point they cannot place falls back to the ring search), else the ring
// search; one cooperative search when all 64 lanes of the wave share the
// point (a point source), else one per lane. Every lane of the wave must
// call it. STOP_AT_SITE: a search ends at a site the point coincides with
// (rays that start at sites), which costs the calling kernel registers.
template <bool STOP_AT_SITE = true>
__device__ __forceinline__ int32_t start_cell(const BucketGridView &grid, const LocView &L, const double q[3], bool ok)
{
    const double q0 = __shfl(q[0], 0, 64), q1 = __shfl(q[1], 0, 64), q2 = __shfl(q[2], 0, 64);
    const bool same = ok && q[0] == q0 && q[1] == q1 && q[2] == q2;
    const bool shared = __ballot(true) == ~0ull && __ballot(same) == ~0ull;
    int32_t m = -1, uid;
    if (L.start) {
        if (shared) m = nearest_in_blocks_wave(L, q);
        else if (ok) m = nearest_in_blocks<STOP_AT_SITE>(L, q, &uid);
        if (ok && m < 0) m = nearest_site<STOP_AT_SITE>(grid, q, nullptr);   // empty list: not in the box
    } else if (shared) {
        m = nearest_site_wave(grid, q, nullptr);
    } else if (ok) {
        m = nearest_site<STOP_AT_SITE>(grid, q, nullptr);
    }
    return ok ? m : -1;
}

}  // namespace vrt
