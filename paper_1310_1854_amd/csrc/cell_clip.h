// cell_clip.h -- one site's Voronoi cell clipped out of the box, plane by
// plane, and the nearest-first candidate search that feeds it. Host and
// device code: the GPU builder runs it one site per lane, and it also
// compiles for the CPU.
#pragma once

#include "vrt_internal.h"

namespace vrt {

constexpr int kMaxCand = 96;       // candidates sorted per batch
constexpr int kMaxNbr = 64;        // neighbour-list capacity per site in the first pass
constexpr int kMaxNbrBig = 250;    // ... and in the retry pass for cells with many faces
constexpr int kHilbertBits = 10;   // per axis

enum : int { ERR_OUTSIDE = 1, ERR_DUP = 2, ERR_CAPACITY = 4, ERR_DEGENERATE = 8 };

struct BoxArg {
    double lo[3], hi[3];
};

// ---------------------------------------------------------------------------
// Per-site convex cell, clipped plane by plane.
//
// The cell is kept as the dual of its boundary: each vertex is a triangle of
// three plane slots (the faces meeting there), oriented so that the triple
// product of the three normals is positive; with simple vertices each
// polyhedron edge then appears once in each direction. Cutting by a plane
// removes the triangles whose vertex lies strictly outside; the edges of
// removed triangles whose reverse edge is not itself removed form the rim
// of the cut, and each rim edge (a, b) becomes a new triangle (a, b, P).
// Coordinates are relative to the site, so planes read n.x <= d with
// d = |n|^2 / 2 for a site at offset n.
//
// P plane slots (at most 255: slots are packed in 8 bits) and T vertices.
// The first pass uses a small cell in registers/private memory; the few
// cells that need more faces are redone with a large cell kept in a global
// workspace.
// ---------------------------------------------------------------------------

template <int P, int T>
struct CellT {
    static constexpr int kPlanes = P;
    static constexpr int kTris = T;
    double nx[P], ny[P], nz[P], d[P];
    int32_t id[P];            // internal site index, or -(w+1) for box wall w
    uint32_t tri[T];          // three 8-bit plane slots
    double vx[T], vy[T], vz[T];
    uint32_t rem[T];          // scratch: triangles removed by the current cut
    uint32_t rim[P];          // scratch: rim edges of the current cut
    int np, nt;
    double r2;                // largest squared vertex distance from the site
};

using CellSmall = CellT<64, 128>;
using CellBig = CellT<255, 512>;

VRT_HD inline uint32_t pack3(int a, int b, int c) { return (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16); }

template <class C>
VRT_HD bool vertex_of(const C &c, int a, int b, int p, double &x, double &y, double &z)
{
    // Cramer: x = (d_a (n_b x n_p) + d_b (n_p x n_a) + d_p (n_a x n_b)) / det
    double bxpx = c.ny[b] * c.nz[p] - c.nz[b] * c.ny[p];
    double bxpy = c.nz[b] * c.nx[p] - c.nx[b] * c.nz[p];
    double bxpz = c.nx[b] * c.ny[p] - c.ny[b] * c.nx[p];
    double pxax = c.ny[p] * c.nz[a] - c.nz[p] * c.ny[a];
    double pxay = c.nz[p] * c.nx[a] - c.nx[p] * c.nz[a];
    double pxaz = c.nx[p] * c.ny[a] - c.ny[p] * c.nx[a];
    double axbx = c.ny[a] * c.nz[b] - c.nz[a] * c.ny[b];
    double axby = c.nz[a] * c.nx[b] - c.nx[a] * c.nz[b];
    double axbz = c.nx[a] * c.ny[b] - c.ny[a] * c.nx[b];
    double det = c.nx[a] * bxpx + c.ny[a] * bxpy + c.nz[a] * bxpz;
    double inv = 1.0 / det;
    x = (c.d[a] * bxpx + c.d[b] * pxax + c.d[p] * axbx) * inv;
    y = (c.d[a] * bxpy + c.d[b] * pxay + c.d[p] * axby) * inv;
    z = (c.d[a] * bxpz + c.d[b] * pxaz + c.d[p] * axbz) * inv;
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

template <class C>
VRT_HD void cell_init(C &c, const double p[3], const BoxArg &box)
{
    for (int w = 0; w < 6; ++w) {
        int a = w >> 1;
        c.nx[w] = c.ny[w] = c.nz[w] = 0.0;
        double s = (w & 1) ? 1.0 : -1.0;
        if (a == 0) c.nx[w] = s;
        else if (a == 1) c.ny[w] = s;
        else c.nz[w] = s;
        c.d[w] = (w & 1) ? (box.hi[a] - p[a]) : (p[a] - box.lo[a]);
        c.id[w] = -(w + 1);
    }
    c.np = 6;
    c.nt = 0;
    c.r2 = 0.0;
    for (int sx = 0; sx < 2; ++sx)
        for (int sy = 0; sy < 2; ++sy)
            for (int sz = 0; sz < 2; ++sz) {
                int X = sx, Y = 2 + sy, Z = 4 + sz;
                int sign = (sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1);
                uint32_t t = sign > 0 ? pack3(X, Y, Z) : pack3(X, Z, Y);
                int k = c.nt++;
                c.tri[k] = t;
                c.vx[k] = sx ? c.d[1] : -c.d[0];
                c.vy[k] = sy ? c.d[3] : -c.d[2];
                c.vz[k] = sz ? c.d[5] : -c.d[4];
                double r2 = c.vx[k] * c.vx[k] + c.vy[k] * c.vy[k] + c.vz[k] * c.vz[k];
                c.r2 = fmax(c.r2, r2);
            }
}

// Cut by {x : n.x <= d}; returns 0, or an ERR_* flag.
template <class C>
VRT_HD int cell_clip(C &c, double nx, double ny, double nz, double d, int32_t id)
{
    // classify the vertices; move the removed ones to the scratch list and
    // compact the kept ones in place
    int nrem = 0, nt = 0;
    for (int t = 0; t < c.nt; ++t) {
        double f = nx * c.vx[t] + ny * c.vy[t] + nz * c.vz[t] - d;
        if (f > 0.0) {
            c.rem[nrem++] = c.tri[t];
        } else {
            c.tri[nt] = c.tri[t];
            c.vx[nt] = c.vx[t];
            c.vy[nt] = c.vy[t];
            c.vz[nt] = c.vz[t];
            ++nt;
        }
    }
    if (nrem == 0) return 0;
    if (nt == 0) return ERR_DEGENERATE;   // the site itself is always strictly inside
    // plane slot for the new face: a fresh one, or one no kept vertex uses
    int P = c.np;
    if (P >= C::kPlanes) {
        constexpr int W = (C::kPlanes + 63) / 64;
        uint64_t used[W];
        for (int w = 0; w < W; ++w) used[w] = 0;
        for (int t = 0; t < nt; ++t) {
            uint32_t tr = c.tri[t];
            int v[3] = {(int)(tr & 255), (int)((tr >> 8) & 255), (int)((tr >> 16) & 255)};
            for (int k = 0; k < 3; ++k) used[v[k] >> 6] |= 1ull << (v[k] & 63);
        }
        P = -1;
        for (int s = 0; s < C::kPlanes && P < 0; ++s)
            if (!((used[s >> 6] >> (s & 63)) & 1ull)) P = s;
        if (P < 0) return ERR_CAPACITY;
    }
    // rim: edges (a -> b) of removed triangles whose reverse (b -> a) is not
    // an edge of another removed triangle
    int nrim = 0;
    for (int r = 0; r < nrem; ++r) {
        uint32_t tr = c.rem[r];
        int v[3] = {(int)(tr & 255), (int)((tr >> 8) & 255), (int)((tr >> 16) & 255)};
        for (int k = 0; k < 3; ++k) {
            int a = v[k], b = v[(k + 1) % 3];
            bool inner = false;
            for (int q = 0; q < nrem && !inner; ++q) {
                uint32_t tq = c.rem[q];
                int w0 = tq & 255, w1 = (tq >> 8) & 255, w2 = (tq >> 16) & 255;
                inner = (w0 == b && w1 == a) || (w1 == b && w2 == a) || (w2 == b && w0 == a);
            }
            if (!inner) {
                if (nrim >= C::kPlanes) return ERR_CAPACITY;
                c.rim[nrim++] = (uint32_t)a | ((uint32_t)b << 8);
            }
        }
    }
    if (nt + nrim > C::kTris) return ERR_CAPACITY;
    c.nx[P] = nx;
    c.ny[P] = ny;
    c.nz[P] = nz;
    c.d[P] = d;
    c.id[P] = id;
    if (P == c.np) c.np++;
    double r2 = 0.0;
    for (int t = 0; t < nt; ++t) r2 = fmax(r2, c.vx[t] * c.vx[t] + c.vy[t] * c.vy[t] + c.vz[t] * c.vz[t]);
    for (int k = 0; k < nrim; ++k) {
        int a = c.rim[k] & 255, b = (c.rim[k] >> 8) & 255;
        double x, y, z;
        if (!vertex_of(c, a, b, P, x, y, z)) return ERR_DEGENERATE;
        c.tri[nt] = pack3(a, b, P);
        c.vx[nt] = x;
        c.vy[nt] = y;
        c.vz[nt] = z;
        r2 = fmax(r2, x * x + y * y + z * z);
        ++nt;
    }
    c.nt = nt;
    c.r2 = r2;
    return 0;
}

struct Cand {
    double d2;
    int32_t j;
};

VRT_HD inline void sort_cands(Cand *c, int n)
{
    for (int i = 1; i < n; ++i) {
        Cand x = c[i];
        int k = i - 1;
        while (k >= 0 && (c[k].d2 > x.d2 || (c[k].d2 == x.d2 && c[k].j > x.j))) {
            c[k + 1] = c[k];
            --k;
        }
        c[k + 1] = x;
    }
}

// Clip site i's cell: candidates come from rings of buckets around it,
// nearest-first within each ring, and the search ends once the rings left
// are farther than twice the largest vertex distance (no bisector plane of
// a farther site can reach the cell). Writes up to max_nbr neighbour
// indices to nbr (capacity max_nbr), the wall bit mask to *walls, returns the neighbour count
// (>= 0) or -ERR_* on failure.
template <class C>
VRT_HD int clip_site(const Site *sites, const BucketGridView &grid, const BoxArg &box, int64_t i, int32_t *nbr,
                     int max_nbr, uint8_t *walls, C &c, Cand *cand)
{
    const Site si = sites[i];
    const double p[3] = {si.x, si.y, si.z};
    cell_init(c, p, box);
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(p[a], grid.lo[a], grid.inv_h[a], grid.dims[a]);
    int err = 0;
    int ncand = 0;

    auto flush = [&]() {
        sort_cands(cand, ncand);
        for (int q = 0; q < ncand && !err; ++q) {
            if (cand[q].d2 >= 4.0 * c.r2) break;   // sorted: nothing farther can cut
            const Site sj = sites[cand[q].j];
            double nx = sj.x - p[0], ny = sj.y - p[1], nz = sj.z - p[2];
            double d = 0.5 * (nx * nx + ny * ny + nz * nz);
            err = cell_clip(c, nx, ny, nz, d, cand[q].j);
        }
        ncand = 0;
    };

    for (int r = 0; !err; ++r) {
        for_shell(grid, b, r, [&](int bk) {
            int s0 = grid.start[bk], s1 = grid.start[bk + 1];
            for (int s = s0; s < s1 && !err; ++s) {
                Site q = grid.items[s];
                int32_t j = (int32_t)(q.uid & 0xffffffff);
                if (j == (int32_t)i) continue;
                double dx = q.x - p[0], dy = q.y - p[1], dz = q.z - p[2];
                double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 == 0.0) {
                    err = ERR_DUP;
                    break;
                }
                if (d2 >= 4.0 * c.r2) continue;   // its bisector plane lies beyond every vertex
                if (ncand == kMaxCand) flush();
                cand[ncand].d2 = d2;
                cand[ncand].j = j;
                ++ncand;
            }
        });
        if (err) break;
        flush();
        if (err) break;
        double lb = shell_bound(grid, p, b, r);
        if (lb < 0.0) break;
        if (lb * lb > 4.0 * c.r2 * (1.0 + 1e-9)) break;
    }
    if (err) return -err;
    // faces = plane slots still used by some vertex
    int nn = 0;
    uint8_t wm = 0;
    uint64_t used = 0;
    for (int t = 0; t < c.nt; ++t) {
        uint32_t tr = c.tri[t];
        used |= (1ull << (tr & 255)) | (1ull << ((tr >> 8) & 255)) | (1ull << ((tr >> 16) & 255));
    }
    for (int sl = 0; sl < c.np; ++sl) {
        if (!((used >> sl) & 1ull)) continue;
        if (c.id[sl] < 0) {
            wm |= (uint8_t)(1u << (-c.id[sl] - 1));
        } else {
            if (nn >= max_nbr) return -ERR_CAPACITY;
            nbr[nn++] = c.id[sl];
        }
    }
    *walls = wm;
    return nn;
}

}  // namespace vrt
