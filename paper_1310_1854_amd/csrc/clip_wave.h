// clip_wave.h -- the neighbour-table builder's cell clipping, one 64-lane
// wave per site with the cell held in LDS.
//
// A site's Voronoi cell is the box cut by the bisector half-space of every
// other site (Sect. 2.1); only sites closer than twice the cell's largest
// vertex distance can cut it. Candidates come from rings of buckets around
// the site, nearest first; each cut is done by the whole wave:
//   - every lane classifies its share of the cell's vertices against the
//     plane (a vertex is cut off when it lies beyond the plane by more than
//     a relative tolerance, so planes that merely touch an edge or a vertex
//     leave no sliver face);
//   - kept and removed vertices are compacted with ballots;
//   - the rim of the cut (edges of removed vertices whose twin edge is kept)
//     is found in parallel, and each rim edge gives one new vertex on the
//     new face.
// The cell is stored as the dual of its boundary: each vertex is a triangle
// of three plane slots, oriented so that the normals' triple product is
// positive; each polyhedron edge then appears once in each direction.
// Coordinates are relative to the site: a site at offset n gives the plane
// n.x <= |n|^2/2. The faces left at the end are the site's neighbours.
#pragma once

#include "vrt_internal.h"

namespace vrt {

constexpr int kMaxNbr = 64;        // neighbour-list capacity per site in the first pass
constexpr int kMaxNbrBig = 250;    // ... and in the retry pass for cells with many faces
constexpr int kHilbertBits = 10;   // per axis

enum : int { ERR_OUTSIDE = 1, ERR_DUP = 2, ERR_CAPACITY = 4, ERR_DEGENERATE = 8 };

struct BoxArg {
    double lo[3], hi[3];
};

// P plane slots (<= 255, 8-bit packed), T vertices, NC candidates per batch.
template <int P, int T, int NC>
struct WaveCell {
    static constexpr int kPlanes = P;
    static constexpr int kTris = T;
    static constexpr int kCand = NC;
    static constexpr int kPerLane = T / 64;
    double nx[P], ny[P], nz[P], d[P];
    int32_t id[P];          // internal site index, or -(w+1) for box wall w
    uint32_t tri[T];
    double vx[T], vy[T], vz[T];
    uint32_t rem[T];        // triangles removed by the current cut
    uint32_t rim[P];        // rim edges of the current cut
    double cd2[NC];         // candidate squared distances
    int32_t cj[NC];         // candidate sites
    int ncand;              // LDS counter while collecting
    int nrim;
};

using WaveCellSmall = WaveCell<64, 128, 256>;
using WaveCellBig = WaveCell<255, 512, 256>;

__device__ __forceinline__ uint32_t wpack3(int a, int b, int c)
{
    return (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    int l = lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

__device__ __forceinline__ double wave_max_d(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v |= (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_excl_scan_i(int v)
{
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off, 64);
        if (lane_id() >= off) incl += u;
    }
    return incl - v;
}

// Vertex of planes a, b, p by Cramer's rule.
template <class C>
__device__ __forceinline__ bool wvertex(const C &c, int a, int b, int p, double &x, double &y, double &z)
{
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
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// The box as the initial cell (6 wall planes, 8 corner vertices).
// Returns the largest squared vertex distance.
template <class C>
__device__ double wcell_init(C &c, const double p[3], const BoxArg &box, int &np, int &nt)
{
    const int l = lane_id();
    if (l < 6) {
        int w = l, a = w >> 1;
        double s = (w & 1) ? 1.0 : -1.0;
        c.nx[w] = (a == 0) ? s : 0.0;
        c.ny[w] = (a == 1) ? s : 0.0;
        c.nz[w] = (a == 2) ? s : 0.0;
        c.d[w] = (w & 1) ? (box.hi[a] - p[a]) : (p[a] - box.lo[a]);
        c.id[w] = -(w + 1);
    }
    double r2 = 0.0;
    if (l < 8) {
        int sx = l & 1, sy = (l >> 1) & 1, sz = (l >> 2) & 1;
        int X = sx, Y = 2 + sy, Z = 4 + sz;
        int sign = (sx ? 1 : -1) * (sy ? 1 : -1) * (sz ? 1 : -1);
        c.tri[l] = sign > 0 ? wpack3(X, Y, Z) : wpack3(X, Z, Y);
        double x = sx ? (box.hi[0] - p[0]) : -(p[0] - box.lo[0]);
        double y = sy ? (box.hi[1] - p[1]) : -(p[1] - box.lo[1]);
        double z = sz ? (box.hi[2] - p[2]) : -(p[2] - box.lo[2]);
        c.vx[l] = x;
        c.vy[l] = y;
        c.vz[l] = z;
        r2 = x * x + y * y + z * z;
    }
    np = 6;
    nt = 8;
    __syncthreads();
    return wave_max_d(r2);
}

// Cut the cell by {x : n.x <= d} (plane id `id`). np, nt, r2 are
// wave-uniform. Returns 0 or an ERR_* flag.
template <class C>
__device__ int wcell_clip(C &c, double nx, double ny, double nz, double d, int32_t id, int &np, int &nt, double &r2)
{
    constexpr int K = C::kPerLane;
    const int l = lane_id();
    const uint64_t lt = lanemask_lt();
    // relative tolerance: the scale of the terms of n.v - d
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    const double tol = 1e-12 * (nn * sqrt(r2) + fabs(d));
    uint32_t tr[K];
    double x[K], y[K], z[K];
    bool out[K], have[K];
    int nrem = 0;
    uint64_t bal_out[K], bal_keep[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        int t = q * 64 + l;
        have[q] = t < nt;
        out[q] = false;
        if (have[q]) {
            tr[q] = c.tri[t];
            x[q] = c.vx[t];
            y[q] = c.vy[t];
            z[q] = c.vz[t];
            out[q] = (nx * x[q] + ny * y[q] + nz * z[q] - d) > tol;
        }
        bal_out[q] = __ballot(have[q] && out[q]);
        bal_keep[q] = __ballot(have[q] && !out[q]);
        nrem += __popcll(bal_out[q]);
    }
    if (nrem == 0) return 0;
    if (nrem == nt) return ERR_DEGENERATE;   // the site itself is always strictly inside
    // plane slot of the new face: a fresh one, or one no kept vertex uses
    int Pn = np;
    if (Pn >= C::kPlanes) {
        constexpr int W = (C::kPlanes + 63) / 64;
        uint64_t used[W];
        for (int w = 0; w < W; ++w) used[w] = 0;
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (have[q] && !out[q]) {
                int v0 = tr[q] & 255, v1 = (tr[q] >> 8) & 255, v2 = (tr[q] >> 16) & 255;
                used[v0 >> 6] |= 1ull << (v0 & 63);
                used[v1 >> 6] |= 1ull << (v1 & 63);
                used[v2 >> 6] |= 1ull << (v2 & 63);
            }
        Pn = -1;
        for (int w = 0; w < W && Pn < 0; ++w) {
            uint64_t u = wave_or_u64(used[w]);
            uint64_t freem = ~u;
            if (w == W - 1 && (C::kPlanes & 63)) freem &= (1ull << (C::kPlanes & 63)) - 1;
            if (freem) Pn = w * 64 + __ffsll((long long)freem) - 1;
        }
        if (Pn < 0) return ERR_CAPACITY;
    }
    // compact kept vertices in place and list the removed ones; every lane
    // holds its vertices in registers, so the moves cannot collide
    __syncthreads();
    int kbase = 0, rbase = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if (have[q]) {
            if (out[q]) {
                c.rem[rbase + __popcll(bal_out[q] & lt)] = tr[q];
            } else {
                int dst = kbase + __popcll(bal_keep[q] & lt);
                c.tri[dst] = tr[q];
                c.vx[dst] = x[q];
                c.vy[dst] = y[q];
                c.vz[dst] = z[q];
            }
        }
        kbase += __popcll(bal_keep[q]);
        rbase += __popcll(bal_out[q]);
    }
    const int nkeep = kbase;
    __syncthreads();
    // rim edges: (a -> b) of a removed triangle whose reverse (b -> a) is not
    // an edge of another removed triangle
    int nrim = 0;
    for (int r0 = 0; r0 < nrem; r0 += 64) {
        int r = r0 + l;
        bool act = r < nrem;
        uint32_t t = act ? c.rem[r] : 0u;
        int v[3] = {(int)(t & 255), (int)((t >> 8) & 255), (int)((t >> 16) & 255)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int a = v[k], b = v[(k + 1) % 3];
            bool rim_edge = false;
            if (act) {
                rim_edge = true;
                for (int s = 0; s < nrem && rim_edge; ++s) {
                    uint32_t u = c.rem[s];
                    int w0 = u & 255, w1 = (u >> 8) & 255, w2 = (u >> 16) & 255;
                    if ((w0 == b && w1 == a) || (w1 == b && w2 == a) || (w2 == b && w0 == a)) rim_edge = false;
                }
            }
            uint64_t bal = __ballot(rim_edge);
            int pos = nrim + __popcll(bal & lt);
            if (rim_edge && pos < C::kPlanes) c.rim[pos] = (uint32_t)a | ((uint32_t)b << 8);
            nrim += __popcll(bal);
        }
    }
    if (nrim > C::kPlanes) return ERR_CAPACITY;
    if (nkeep + nrim > C::kTris) return ERR_CAPACITY;
    if (l == 0) {
        c.nx[Pn] = nx;
        c.ny[Pn] = ny;
        c.nz[Pn] = nz;
        c.d[Pn] = d;
        c.id[Pn] = id;
    }
    __syncthreads();
    if (Pn == np) np++;
    // one new vertex per rim edge
    int bad = 0;
    for (int k0 = 0; k0 < nrim; k0 += 64) {
        int k = k0 + l;
        if (k < nrim) {
            uint32_t e = c.rim[k];
            int a = e & 255, b = (e >> 8) & 255;
            double vx, vy, vz;
            if (!wvertex(c, a, b, Pn, vx, vy, vz)) bad = 1;
            c.tri[nkeep + k] = wpack3(a, b, Pn);
            c.vx[nkeep + k] = vx;
            c.vy[nkeep + k] = vy;
            c.vz[nkeep + k] = vz;
        }
    }
    if (__ballot(bad)) return ERR_DEGENERATE;
    nt = nkeep + nrim;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        int t = q * 64 + l;
        if (t < nt) m = fmax(m, c.vx[t] * c.vx[t] + c.vy[t] * c.vy[t] + c.vz[t] * c.vz[t]);
    }
    r2 = wave_max_d(m);
    return 0;
}

// Bucket at position q of the Chebyshev shell of radius r around b (24 r^2
// + 2 positions: the two z faces, then the two y faces without their z
// edges, then the two x faces without either); -1 outside the grid.
__device__ __forceinline__ int shell_bucket(const BucketGridView &g, const int b[3], int r, int q)
{
    int dx, dy, dz;
    if (r == 0) {
        dx = dy = dz = 0;
    } else {
        const int n1 = 2 * r + 1, n2 = 2 * r - 1;
        if (q < 2 * n1 * n1) {
            dz = (q < n1 * n1) ? -r : r;
            int i = q % (n1 * n1);
            dx = i % n1 - r;
            dy = i / n1 - r;
        } else if ((q -= 2 * n1 * n1) < 2 * n1 * n2) {
            dy = (q < n1 * n2) ? -r : r;
            int i = q % (n1 * n2);
            dx = i % n1 - r;
            dz = i / n1 - (r - 1);
        } else {
            q -= 2 * n1 * n2;
            dx = (q < n2 * n2) ? -r : r;
            int i = q % (n2 * n2);
            dy = i % n2 - (r - 1);
            dz = i / n2 - (r - 1);
        }
    }
    int x = b[0] + dx, y = b[1] + dy, z = b[2] + dz;
    if (x < 0 || y < 0 || z < 0 || x >= g.dims[0] || y >= g.dims[1] || z >= g.dims[2]) return -1;
    return (z * g.dims[1] + y) * g.dims[0] + x;
}

// Sort the candidate batch by (squared distance, index) in LDS (bitonic).
template <class C>
__device__ void sort_candidates(C &c, int n)
{
    int m = 1;
    while (m < n) m <<= 1;
    const int l = lane_id();
    for (int i = n + l; i < m; i += 64) {
        c.cd2[i] = 1e308 * 10.0;
        c.cj[i] = 0x7fffffff;
    }
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = l; i < m; i += 64) {
                int p = i ^ j;
                if (p > i) {
                    bool up = (i & k) == 0;
                    double a = c.cd2[i], bb = c.cd2[p];
                    int ja = c.cj[i], jb = c.cj[p];
                    bool gt = (a > bb) || (a == bb && ja > jb);
                    if (gt == up) {
                        c.cd2[i] = bb;
                        c.cd2[p] = a;
                        c.cj[i] = jb;
                        c.cj[p] = ja;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Clip site i's cell. Writes the neighbour indices to nbr (capacity
// max_nbr) and the wall mask to *walls; returns the count or -ERR_*.
// All lanes of the wave call it with the same i.
// Volume of the clipped cell (nt vertices), by the whole wave. The cell is
// the union of the cones from the site (the origin here) to its faces, so
// V = sum over faces x of (h_x / 3) * area_x, with h_x = d_x / |n_x| the
// distance of plane x from the site. Around face x the vertices come in a
// cyclic order: from vertex t = (x, y, z) (oriented) the next is the vertex
// holding the reversed edge (y, x), the other end of the polyhedron edge
// between faces x and y; so 2 area_x = |sum over the face's vertices of
// n_x / |n_x| . (v_t x v_next)|, with one orientation for every face.
template <class C>
__device__ double wcell_volume(const C &c, int nt)
{
    double acc = 0.0;
    for (int t = lane_id(); t < nt; t += 64) {
        const uint32_t u = c.tri[t];
        const int corner[3] = {(int)(u & 255), (int)((u >> 8) & 255), (int)((u >> 16) & 255)};
        for (int e = 0; e < 3; ++e) {
            const int x = corner[e], y = corner[(e + 1) % 3];
            int t2 = -1;
            for (int s = 0; s < nt && t2 < 0; ++s) {
                const uint32_t w = c.tri[s];
                const int a = w & 255, b = (w >> 8) & 255, cc = (w >> 16) & 255;
                if ((a == y && b == x) || (b == y && cc == x) || (cc == y && a == x)) t2 = s;
            }
            if (t2 < 0) continue;   // cannot happen in a closed cell
            const double cx = c.vy[t] * c.vz[t2] - c.vz[t] * c.vy[t2];
            const double cy = c.vz[t] * c.vx[t2] - c.vx[t] * c.vz[t2];
            const double cz = c.vx[t] * c.vy[t2] - c.vy[t] * c.vx[t2];
            const double nn = c.nx[x] * c.nx[x] + c.ny[x] * c.ny[x] + c.nz[x] * c.nz[x];
            acc += c.d[x] / nn * (c.nx[x] * cx + c.ny[x] * cy + c.nz[x] * cz);
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return fabs(acc) / 6.0;
}

// Bounding box of the clipped cell from its vertices (Sect. 2.3: the cell
// is convex), absolute coordinates {xmin, ymin, zmin, xmax, ymax, zmax};
// every lane gets it.
template <class C>
__device__ void wcell_bbox(const C &c, int nt, const double p[3], double bb[6])
{
    double lo[3] = {__builtin_huge_val(), __builtin_huge_val(), __builtin_huge_val()};
    double hi[3] = {-__builtin_huge_val(), -__builtin_huge_val(), -__builtin_huge_val()};
    for (int t = lane_id(); t < nt; t += 64) {
        const double v[3] = {c.vx[t], c.vy[t], c.vz[t]};
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], v[a]);
            hi[a] = fmax(hi[a], v[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], off, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], off, 64));
        }
        bb[a] = p[a] + lo[a];
        bb[a + 3] = p[a] + hi[a];
    }
}

template <class C>
__device__ int wclip_site(C &c, const Site *__restrict__ sites, const BucketGridView &grid, const BoxArg &box,
                          int64_t i, int32_t *nbr, int max_nbr, uint8_t *walls, double *volume = nullptr,
                          double *bbox = nullptr)
{
    const int l = lane_id();
    const uint64_t lt = lanemask_lt();
    const Site si = sites[i];
    const double p[3] = {si.x, si.y, si.z};
    int np, nt;
    double r2 = wcell_init(c, p, box, np, nt);
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = bucket_coord(p[a], grid.lo[a], grid.inv_h[a], grid.dims[a]);
    int err = 0;

    for (int r = 0; !err; ++r) {
        const int nshell = (r == 0) ? 1 : 24 * r * r + 2;
        // candidates of this ring that may cut the cell: count per lane, rank
        const double lim = 4.0 * r2;
        int mine = 0;
        int dup = 0;
        for (int q = l; q < nshell; q += 64) {
            int bk = shell_bucket(grid, b, r, q);
            if (bk < 0) continue;
            for (int s = grid.start[bk]; s < grid.start[bk + 1]; ++s) {
                Site o = grid.items[s];
                int32_t j = (int32_t)(o.uid & 0xffffffff);
                if (j == (int32_t)i) continue;
                double dx = o.x - p[0], dy = o.y - p[1], dz = o.z - p[2];
                double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 == 0.0) dup = 1;
                if (d2 < lim) ++mine;
            }
        }
        if (__ballot(dup)) {
            err = ERR_DUP;
            break;
        }
        const int total = wave_sum_i(mine);
        const int first = wave_excl_scan_i(mine);
        // batches of at most kCand candidates, taken in rank order
        for (int b0 = 0; b0 < total && !err; b0 += C::kCand) {
            const int b1 = min(total, b0 + C::kCand);
            int k = first;
            for (int q = l; q < nshell && k < b1; q += 64) {
                int bk = shell_bucket(grid, b, r, q);
                if (bk < 0) continue;
                for (int s = grid.start[bk]; s < grid.start[bk + 1] && k < b1; ++s) {
                    Site o = grid.items[s];
                    int32_t j = (int32_t)(o.uid & 0xffffffff);
                    if (j == (int32_t)i) continue;
                    double dx = o.x - p[0], dy = o.y - p[1], dz = o.z - p[2];
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (!(d2 < lim)) continue;
                    if (k >= b0) {
                        c.cd2[k - b0] = d2;
                        c.cj[k - b0] = j;
                    }
                    ++k;
                }
            }
            __syncthreads();
            const int n = b1 - b0;
            sort_candidates(c, n);
            for (int q = 0; q < n && !err; ++q) {
                const double d2 = c.cd2[q];
                if (d2 >= 4.0 * r2) break;   // sorted: nothing farther can cut
                const int32_t j = c.cj[q];
                const Site sj = sites[j];
                double nx = sj.x - p[0], ny = sj.y - p[1], nz = sj.z - p[2];
                double dd = 0.5 * (nx * nx + ny * ny + nz * nz);
                err = wcell_clip(c, nx, ny, nz, dd, j, np, nt, r2);
            }
            __syncthreads();
        }
        if (err) break;
        double lb = shell_bound(grid, p, b, r);
        if (lb < 0.0) break;
        if (lb * lb > 4.0 * r2 * (1.0 + 1e-9)) break;
    }
    if (err) return -err;
    if (volume) *volume = wcell_volume(c, nt);
    if (bbox) wcell_bbox(c, nt, p, bbox);
    // faces: plane slots some vertex still uses
    constexpr int W = (C::kPlanes + 63) / 64;
    uint64_t used[W];
    for (int w = 0; w < W; ++w) used[w] = 0;
    for (int t = l; t < nt; t += 64) {
        uint32_t u = c.tri[t];
        int v0 = u & 255, v1 = (u >> 8) & 255, v2 = (u >> 16) & 255;
        used[v0 >> 6] |= 1ull << (v0 & 63);
        used[v1 >> 6] |= 1ull << (v1 & 63);
        used[v2 >> 6] |= 1ull << (v2 & 63);
    }
    for (int w = 0; w < W; ++w) used[w] = wave_or_u64(used[w]);
    int nn = 0;
    uint8_t wm = 0;
    for (int s0 = 0; s0 < np; s0 += 64) {
        int s = s0 + l;
        bool face = s < np && ((used[s >> 6] >> (s & 63)) & 1ull);
        int32_t id = face ? c.id[s] : 0;
        bool site = face && id >= 0;
        if (face && id < 0) wm |= (uint8_t)(1u << (-id - 1));
        uint64_t bal = __ballot(site);
        int pos = nn + __popcll(bal & lt);
        if (site && pos < max_nbr) nbr[pos] = id;
        nn += __popcll(bal);
    }
    for (int off = 32; off > 0; off >>= 1) wm |= (uint8_t)__shfl_xor((int)wm, off, 64);
    if (nn > max_nbr) return -ERR_CAPACITY;
    *walls = wm;
    return nn;
}

}  // namespace vrt
