// trace_core.h -- the per-ray work of the straight-path method (Sect. 2.2,
// Eqs. 1-5) shared by every tracing kernel: ray set-up, start cell, and one
// exit-point step in FP64 or mixed precision.
//
// Every crossing is measured from the ray's origin r0:
//     s_j = n.((p_j + p_m)/2 - r0) / (n.k),   n = p_j - p_m,
// which is Eq. 4 with the current point r = r0 + s_c k substituted and s
// counted from r0, so no position error builds up along the path. Only
// neighbours with n.k > 0 are evaluated (the sign argument of Sect. 2.2),
// the chord end L (Eq. 5 on every axis) is always a candidate, and a
// crossing at or behind the current position moves to that neighbour
// without emitting a segment.
#pragma once

#include "vrt_internal.h"

namespace vrt {

// A resident grid as the tracing code reads it.
struct GridRef {
    const Site *sites;
    const int2 *rows;
    const Rec64 *rec64;
    const Slot *blk;     // cell blocks (header, FP32 or compact records, neighbour block offsets)
    const int32_t *blk_off;  // where each cell's block starts when the grid keeps it (compact blocks; null: block_of)
    const Slot *blk64;       // FP64 cell blocks (header, FP64 neighbour sites, block offsets): FP64-mode steps
    const int32_t *blk64_off;
    const double *rho_int;   // the density bound to the grid, internal order
    BucketGridView grid;
    double lo[3], hi[3];
    int32_t max_steps;
    float eps_mix;
    float eps_abs;        // FP64 rounding allowance of the mixed-mode bound (2^-48 x coordinate scale)
    double eps_fb;        // no-exit fallback advance
};

// The rays' inputs.
struct RayIn {
    const double *origins;
    const double *dirs;
    const double *density;
    double kappa;
    int32_t enter;     // rays from outside the box start where they enter it
    int32_t grid_rho;  // densities from the cells' block headers (bound to the grid) instead of `density`
};

// Where segments go: a window per ray, then (optionally) a chain of spill
// chunks of kSpillChunk segments for the part of a path past its window.
constexpr int kSpillChunk = VOR_SPILL_CHUNK;

#ifndef VRT_VEC_STORE
#define VRT_VEC_STORE 1
#endif
#ifndef VRT_NT_STORE
#define VRT_NT_STORE 0
#endif
#ifndef VRT_LDS_STAGE
#define VRT_LDS_STAGE 1
#endif
#ifndef VRT_NT_STORE_SERVE
#define VRT_NT_STORE_SERVE 1
#endif

// A pool of spill chunks read from memory by the lane that takes a chunk: in
// the serving kernel the lanes of one wave may hold rays of different
// requests, each with a pool of its own. The pool's chunks lie in the
// window arrays themselves, after the windows: chunk k of the pool holds
// slots [(base_chunk + k) * kSpillChunk, ...) of SegOut's cell and len, so
// a lane stores its spill segments through the window pointers it already
// holds. first and next hold pool-relative chunk numbers k.
struct SpillPool {
    int32_t *next;
    int64_t *first;
    int64_t chunks;
    int64_t base_chunk;
    unsigned long long *head;
};

struct SegOut {
    int32_t *cell;                  // window slots
    double *len;
    int vec;                        // windows start on multiples of 8 slots (1) or 16 (2): groups of segments stored together
    int32_t *spill_cell;            // chunk c holds slots [c * kSpillChunk, (c + 1) * kSpillChunk)
    double *spill_len;
    int32_t *spill_next;            // next chunk of the same path, -1 at the end
    int64_t *spill_first;           // first chunk of each ray, -1 if none
    int64_t spill_chunks;           // capacity in chunks
    unsigned long long *chunk_head; // chunks handed out
    const SpillPool *pool;          // LP kernels: this lane's pool (in cell and len) instead of the spill arrays above
};

// The kernels' MODE: VOR_MODE_FP64, VOR_MODE_MIXED, or kModeCompact, mixed
// mode over a grid with compact records (vrt::Grid::compact).
constexpr int kModeCompact = 2;

// Smallest accepted eps of the mixed-mode bound (2^-20 = 16u): twice what
// the rounding analysis of exit_mixed needs.
constexpr double kEpsMixMin = 9.5367431640625e-07;

// Mixed mode keeps offsets, points and bounds in FP32: the box must lie
// well inside the FP32 range.
inline bool mixed_mode_fits(const Grid &g)
{
    for (int a = 0; a < 6; ++a)
        if (!(fabs(g.box[a]) < 1e30)) return false;
    return true;
}

// Optional transport outputs of a trace; all null when unused.
//   tau_stop  [N] the optical depth at which each path stops (the package
//             interacts there), or null for paths to the wall;
//   stop_cell [N] cell (user index) of the interaction point, -1 if the
//             path reached the wall first;  stop_s [N] its distance from the
//             origin (the chord L on escape), may be null;
//   tally_len, tally_abs [M] (user order, accumulated): w * length and
//             w * exp(-tau before) * (1 - exp(-kappa rho length)) per cell
//             along each path (cut at the interaction point);
//   weight    [N] w of each ray, or null (1).
struct Extras {
    const double *tau_stop;
    const double *weight;
    double *tally_len;
    double *tally_abs;
    int32_t *stop_cell;
    double *stop_s;
};

inline GridRef grid_ref(const Grid &g, int32_t max_steps, double eps_mix)
{
    GridRef G;
    G.sites = g.sites;
    G.rows = g.rows;
    G.rec64 = g.rec64;
    G.blk = g.blk;
    G.blk_off = g.blk_off;
    G.blk64 = g.blk64;
    G.blk64_off = g.blk64_off;
    G.rho_int = g.rho_int;
    G.grid = bucket_view(g);
    double diag = 0.0, cmax = 0.0;
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = g.box[a];
        G.hi[a] = g.box[a + 3];
        diag += (g.box[a + 3] - g.box[a]) * (g.box[a + 3] - g.box[a]);
        cmax = fmax(cmax, fmax(fabs(g.box[a]), fabs(g.box[a + 3])));
    }
    G.max_steps = max_steps > 0 ? max_steps : (int32_t)(g.M + 16 < 0x7fffffff ? g.M + 16 : 0x7fffffff);
    G.eps_mix = (float)(eps_mix > 0 ? eps_mix : kEpsMixMin);
    G.eps_abs = (float)(3.552713678800501e-15 * (2.0 * cmax + sqrt(diag)));   // 2^-48
    G.eps_fb = 1e-12 * sqrt(diag);
    return G;
}

#ifndef VRT_BATCH64
#define VRT_BATCH64 4
#endif
#ifndef VRT_DIAG
#define VRT_DIAG 0
#endif
#if VRT_DIAG
// Diagnostic build only: batches executed by each wave, counted by the
// wave's first active lane.
__device__ unsigned long long vrt_diag[4];
__device__ __forceinline__ void diag_count(int i)
{
    const uint64_t act = __ballot(true);
    if ((int)(threadIdx.x & 63) == __ffsll((long long)act) - 1) atomicAdd(&vrt_diag[i], 1ull);
}
#define VRT_DIAG_COUNT(i) diag_count(i)
#else
#define VRT_DIAG_COUNT(i)
#endif
#ifndef VRT_BATCH32
#define VRT_BATCH32 8
#endif
constexpr int kBatch64 = VRT_BATCH64;   // FP64 records loaded together per lane
constexpr int kBatch32 = VRT_BATCH32;   // FP32 records loaded together per lane
static_assert(kBatch64 - 1 <= kRecPad && 12 * kBatch32 <= 16 * kRecPad, "a batch may read past a row end");
static_assert(kBatch32 % 4 == 0, "a batch of FP32 records is a whole number of 16-byte loads");


// Crossing of one bisector plane in FP64, measured from r0 (Eqs. 1-4):
// n = p_j - p_m, s = n.((p_j + p_m)/2 - r0) / (n.k). Returns n.k in den.
__device__ __forceinline__ double cross_fp64(double qx, double qy, double qz, const double pm[3], const double r0[3],
                                             const double k[3], double &den)
{
    double n0 = qx - pm[0], n1 = qy - pm[1], n2 = qz - pm[2];
    den = n0 * k[0] + n1 * k[1] + n2 * k[2];
    double w0 = 0.5 * (qx + pm[0]) - r0[0];
    double w1 = 0.5 * (qy + pm[1]) - r0[1];
    double w2 = 0.5 * (qz + pm[2]) - r0[2];
    return (n0 * w0 + n1 * w1 + n2 * w2) / den;
}

// FP64 exit search over row rw of the current cell (site pm). Returns the
// winning record index, or -1 when the chord end L comes first, and the
// crossing in best. Tie rules: equal crossings go to the larger n.k (the
// cell nearest just after the crossing), then to the lower index; the wall
// wins a tie with a plane. Planes with n.k <= 0 are never crossed forwards.
__device__ __forceinline__ int exit_fp64(const Rec64 *__restrict__ rec, int2 rw, const double pm[3],
                                         const double r0[3], const double k[3], double L, double &best)
{
    best = L;
    double best_den = 1e308 * 10.0;
    int win = -1;
    int32_t win_j = 0x7fffffff;
    const int end = rw.x + rw.y;
    for (int e0 = rw.x; e0 < end; e0 += kBatch64) {
        VRT_DIAG_COUNT(1);
        Rec64 q[kBatch64];
#pragma unroll
        for (int u = 0; u < kBatch64; ++u) q[u] = rec[e0 + u];   // past the row end: padding or the next row, unused
#pragma unroll
        for (int u = 0; u < kBatch64; ++u) {
            double den;
            const double sj = cross_fp64(q[u].x, q[u].y, q[u].z, pm, r0, k, den);
            const bool take = e0 + u < end && den > 0.0 &&
                              (sj < best || (sj == best && win >= 0 &&
                                             (den > best_den || (den == best_den && q[u].j < win_j))));
            best = take ? sj : best;
            best_den = take ? den : best_den;
            win = take ? e0 + u : win;
            win_j = take ? q[u].j : win_j;
        }
    }
    return win;
}

// The FP64 exit search over the current cell's FP64 block (offset b, n
// records): exit_fp64's arithmetic and tie rules on the neighbour sites read
// from the block, 4 at a time as 6 aligned 16-byte loads (entries past the
// row end -- the block offsets, padding or the next block -- masked). A row
// lists its neighbours by ascending internal index, so the last tie rule
// (the lower index) is the earlier record. Returns the winner's place in the
// row, or -1 when the chord end comes first; the crossing in best.
__device__ __forceinline__ int exit_fp64_blk(const Slot *__restrict__ blk64, int32_t b, int n, const double pm[3],
                                             const double r0[3], const double k[3], double L, double &best)
{
    static_assert(kBatch64 == 4, "a batch of 4 FP64 sites is 6 aligned 16-byte loads");
    best = L;
    double best_den = 1e308 * 10.0;
    int win = -1;
    const double2 *rec = reinterpret_cast<const double2 *>(blk64 + b + kHdrSlots);
    for (int e0 = 0; e0 < n; e0 += 4) {
        VRT_DIAG_COUNT(1);
        double q[12];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const double2 x = rec[3 * e0 / 2 + u];
            q[2 * u] = x.x;
            q[2 * u + 1] = x.y;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double den;
            const double sj = cross_fp64(q[3 * u], q[3 * u + 1], q[3 * u + 2], pm, r0, k, den);
            const bool take = e0 + u < n && den > 0.0 && (sj < best || (sj == best && win >= 0 && den > best_den));
            best = take ? sj : best;
            best_den = take ? den : best_den;
            win = take ? e0 + u : win;
        }
    }
    return win;
}

// The block offsets that follow the n FP64 sites of the FP64 block at b.
__device__ __forceinline__ const int32_t *fp64_block_offsets(const Slot *blk64, int32_t b, int n)
{
    return reinterpret_cast<const int32_t *>(reinterpret_cast<const double *>(blk64 + b + kHdrSlots) + 3 * n);
}

// Mixed-precision exit search. Returns -1 when the chord end wins
// (best = L), else a non-negative value; redo is set when the step was
// decided in FP64 (then the return value is the winning record index in
// rec64 and best the FP64 crossing); otherwise j1 is the offset of the
// winner's cell block and the caller computes its FP64 crossing from the
// site in the block header. Either way the result equals exit_fp64's. The
// current cell's records (12-byte FP32 offsets, then the neighbours' block
// offsets) start at blk[b + kHdrSlots], rw is its row in rec64.
//
// Each plane is ranked in FP32 from its stored offset n = p_j - p_m
// (rounded once to FP32), the current point q = r - p_m and k (both
// rounded to FP32): t = n.(n/2 - q) / (n.k), with n/2 - q formed by one
// fused operation per axis and one hardware reciprocal (error <= 1 ulp) for
// 1/(n.k), and a bound on how far t can be from the crossing exit_fp64
// computes:
//   err = |n|_1 [c (|q| + |t|) + e_abs] / (n.k),   c = 3 eps
// (u = 2^-24; eps >= 16u). First order, the roundings of n, q, k, of n/2 - q
// and of the two three-term fused dot products move the numerator by at
// most 3u |n|^2 + 6u |n||q| and n.k by at most 5u |n| (also 5u |n|_1). The
// crossing point x = q + t k lies on the plane, n.x = |n|^2 / 2, so
// |n|^2 <= 2 |n| (|q| + |t|), and the error of t is at most
// 12u |n| (|q| + |t|) / (n.k) plus 3u |t| (reciprocal and product) --
// measured against the exact t; with the FP32 n.k trusted only above 4d,
// d = 8u |n|_1 (above the largest error of n.k), 12u |n| / (n.k) <= 0.38,
// so against the FP32 t it is at most 19.3u |n| (|q| + |t|) / (n.k) +
// 4.9u |t|. As |n| / (n.k) >= 1 the last term folds into the first, and
// with the roundings of the bound itself and of t - err, t + err the need
// is 25.2u |n| (|q| + |t|) / (n.k): c = 48u covers it 1.9 times over
// (|n|_1 >= |n|). The bound is linear in |t|: nearly parallel planes have a
// large t and must not get a wide bound. e_abs |n|_1 / (n.k) covers the
// FP64 roundings of exit_fp64 itself (2^-48 times twice the largest box
// coordinate plus the box diagonal). Planes with n.k > 4d have an FP64
// n.k > 0 and this bound; planes with n.k <= -4d have an FP64 n.k <= 0 and
// are skipped as exit_fp64 skips them; a plane in between (nearly parallel
// to the ray) forces the FP64 decision. 4d has a floor of the smallest
// normal float, so planes with a tiny n fall in between too. If the upper
// bound of the best candidate is below the lower bound of every other one
// (the wall included), the FP32 ranking is certain and only the winner's
// crossing is recomputed in FP64 (from its site, same arithmetic as
// exit_fp64); otherwise the step is redone in FP64.
// Records are loaded a whole batch at a time, unconditionally (the record
// arrays are padded for the last row); entries past the row end are masked.
// The current point and direction of a ray in FP32, with the constants of
// the mixed-mode bound.
struct Query32 {
    float qx, qy, qz;       // q = r - p_m
    float kx, ky, kz;
    float c, a;             // 3 eps and c |q| + e_abs (the FP64 allowance)
};

__device__ __forceinline__ Query32 query32(const double pm[3], const double r0[3], const double k[3], double s_c,
                                           float eps, float e_abs)
{
    double q64[3];
    for (int a = 0; a < 3; ++a) q64[a] = (r0[a] + s_c * k[a]) - pm[a];
    Query32 Q;
    Q.qx = (float)q64[0];
    Q.qy = (float)q64[1];
    Q.qz = (float)q64[2];
    Q.kx = (float)k[0];
    Q.ky = (float)k[1];
    Q.kz = (float)k[2];
    Q.c = 3.0f * eps;
    Q.a = fmaf(Q.c, sqrtf(Q.qx * Q.qx + Q.qy * Q.qy + Q.qz * Q.qz), e_abs);
    return Q;
}

// The wall (the chord end L) relative to the current point, and its bound.
__device__ __forceinline__ void wall32(double L, double s_c, float e_abs, float &tw, float &ew)
{
    tw = (float)(L - s_c);
    ew = 2.0f * 5.9604645e-8f * fabsf(tw) + e_abs;
}

// The current point of a ray in a compact cell's scaled units (offsets
// times qs = 2^(19 - E)), with the constants of the bound: as query32, plus
// aq, the quantisation term's part that depends on the point alone.
struct Query32q {
    float qx, qy, qz;
    float kx, ky, kz;
    float c, a, aq;
};

__device__ __forceinline__ Query32q query32q(const double pm[3], const double r0[3], const double k[3], double s_c,
                                             float eps, float e_abs_s, double qs)
{
    double q64[3];
    for (int a = 0; a < 3; ++a) q64[a] = ((r0[a] + s_c * k[a]) - pm[a]) * qs;
    Query32q Q;
    Q.qx = (float)q64[0];
    Q.qy = (float)q64[1];
    Q.qz = (float)q64[2];
    Q.kx = (float)k[0];
    Q.ky = (float)k[1];
    Q.kz = (float)k[2];
    Q.c = 3.0f * eps;
    Q.a = fmaf(Q.c, sqrtf(Q.qx * Q.qx + Q.qy * Q.qy + Q.qz * Q.qz), e_abs_s);
    Q.aq = 0.6667f * (fabsf(Q.qx) + fabsf(Q.qy) + fabsf(Q.qz) + 0.75f);
    return Q;
}

// The crossing of one plane of a compact cell (see exit_mixed): the stored
// offset n is exact in the scaled units and lies within half a unit of the
// true offset per component. With D = n.k and N = n.(n/2 - q), that moves
// N by at most (|n|_1 + 3/4 + |q|_1) / 2 and D by at most sqrt(3)/2 < 0.87,
// so t = N / D moves by at most (|dN| + |t_n| |dD|) / D_true, t_n the exact
// crossing of the stored plane. With D trusted above 4 (8u |n|_1 + 0.875)
// (so D_true >= 3/4 D, D >= 3.5) and |t_n| <= |t| + e, e the FP32 rounding
// bound of plane_bound32 (whose derivation holds for the exact offsets it is
// given here), that is at most
//   (4/3) ((|n|_1 + |q|_1 + 3/4) / 2 + 0.866 |t|) / D + 0.33 e,
// so err = 1.34 e + (0.6667 (|n|_1 + |q|_1 + 3/4) + 1.16 |t|) / D, the
// rounded coefficients covering the reciprocal's error. The grazing band
// widens by the same 0.875 of D, so a plane below -4 (...) has an FP64
// n.k < 0 as before. Offsets that round to nearly nothing (tiny against the
// cell's largest) fall in the band and force the FP64 decision.
__device__ __forceinline__ void plane_bound32q(float nx, float ny, float nz, const Query32q &Q, float &t,
                                               float &err, bool &pos, bool &maybe)
{
    const float den = fmaf(nx, Q.kx, fmaf(ny, Q.ky, nz * Q.kz));
    const float wx = fmaf(0.5f, nx, -Q.qx), wy = fmaf(0.5f, ny, -Q.qy), wz = fmaf(0.5f, nz, -Q.qz);
    const float num = fmaf(nx, wx, fmaf(ny, wy, nz * wz));
    const float n1 = fabsf(nx) + fabsf(ny) + fabsf(nz);
    const float d4 = fmaf(32.0f * 5.9604645e-8f, n1, 3.5f);   // 4 (8u |n|_1 + 0.875)
    pos = den > d4;
    maybe = den > -d4;
    const float rc = __builtin_amdgcn_rcpf(den);
    t = num * rc;
    const float e = (n1 * rc) * fmaf(Q.c, fabsf(t), Q.a);
    err = fmaf(1.34f, e, rc * fmaf(1.16f, fabsf(t), fmaf(0.6667f, n1, Q.aq)));
}

// FP32 crossing t of one plane and its error bound err (see exit_mixed);
// pos: the plane is approached and the bound holds; maybe: it may be
// approached in FP64 (nearly parallel) when pos is false.
__device__ __forceinline__ void plane_bound32(float nx, float ny, float nz, const Query32 &Q, float &t, float &err,
                                              bool &pos, bool &maybe)
{
    const float den = fmaf(nx, Q.kx, fmaf(ny, Q.ky, nz * Q.kz));
    const float wx = fmaf(0.5f, nx, -Q.qx), wy = fmaf(0.5f, ny, -Q.qy), wz = fmaf(0.5f, nz, -Q.qz);
    const float num = fmaf(nx, wx, fmaf(ny, wy, nz * wz));
    const float n1 = fabsf(nx) + fabsf(ny) + fabsf(nz);
    const float d4 = fmaf(32.0f * 5.9604645e-8f, n1, 1.17549435e-38f);   // 4d, floored
    pos = den > d4;
    maybe = den > -d4;
    const float rc = __builtin_amdgcn_rcpf(den);
    t = num * rc;
    err = (n1 * rc) * fmaf(Q.c, fabsf(t), Q.a);
}

// The mixed-mode exit search over a compact cell block: the same ranking
// and certificate as exit_mixed, in the cell's scaled units (everything
// times qs = 2^(19 - E), exact for a power of two), with each record decoded
// exactly from its 21-bit integers and the quantisation term in each bound
// (plane_bound32q). Eight records are four aligned 16-byte loads.
__device__ __forceinline__ int exit_mixed_compact(const Rec64 *__restrict__ rec64, int2 rw,
                                                  const Slot *__restrict__ blk, int32_t b, const double pm[3],
                                                  const double r0[3], const double k[3], double L, double s_c,
                                                  float eps, float e_abs, double &best, bool &redo, int32_t &j1,
                                                  double qs)
{
    const float e_abs_s = (float)((double)e_abs * qs);
    const Query32q Q = query32q(pm, r0, k, s_c, eps, e_abs_s, qs);
    const float inf = __builtin_huge_valf();
    const float tw = (float)((L - s_c) * qs);
    const float ew = 2.0f * 5.9604645e-8f * fabsf(tw) + e_abs_s;
    float t1 = tw, err1 = ew;
    int w1 = -1;
    float lo_a = tw - ew, lo_b = inf;
    bool graze = false;
    const int n = rw.y;
    const uint4 *rec = reinterpret_cast<const uint4 *>(blk + b + kHdrSlots);   // 8 records = 4 uint4
    for (int e0 = 0; e0 < n; e0 += kBatch32) {
        uint32_t w[2 * kBatch32];
#pragma unroll
        for (int u = 0; u < kBatch32 / 2; ++u) {   // past the row end: block offsets, padding or the next block, masked
            const uint4 x = rec[e0 / 2 + u];
            w[4 * u] = x.x;
            w[4 * u + 1] = x.y;
            w[4 * u + 2] = x.z;
            w[4 * u + 3] = x.w;
        }
        const int rem = n - e0;
#pragma unroll
        for (int v = 0; v < kBatch32; ++v) {
            const bool in = v < rem;
            const uint32_t lo = w[2 * v], hi = w[2 * v + 1];
            const int32_t ix = __builtin_amdgcn_sbfe((int32_t)lo, 0, kQBits);
            const int32_t iy = __builtin_amdgcn_sbfe((int32_t)__builtin_amdgcn_alignbit(hi, lo, kQBits), 0, kQBits);
            const int32_t iz = __builtin_amdgcn_sbfe((int32_t)hi, 2 * kQBits - 32, kQBits);
            float t, err;
            bool pos, maybe;
            plane_bound32q((float)ix, (float)iy, (float)iz, Q, t, err, pos, maybe);
            pos = pos && in;
            graze = graze || (maybe && in && !pos);
            const float lo_t = pos ? t - err : inf;
            const bool win = pos && t < t1;
            t1 = win ? t : t1;
            err1 = win ? err : err1;
            w1 = win ? e0 + v : w1;
            lo_b = __builtin_amdgcn_fmed3f(lo_a, lo_b, lo_t);
            lo_a = fminf(lo_a, lo_t);
        }
    }
    const float lo1 = t1 - err1;
    const float lo_other = (lo1 == lo_a) ? lo_b : lo_a;
    if (graze || !(t1 + err1 < lo_other)) {
        redo = true;
        j1 = -1;
        return exit_fp64(rec64, rw, pm, r0, k, L, best);
    }
    redo = false;
    if (w1 < 0) {
        j1 = -1;
        best = L;
        return -1;
    }
    j1 = reinterpret_cast<const int32_t *>(reinterpret_cast<const uint2 *>(rec) + n)[w1];
    return 0;
}

__device__ __forceinline__ int exit_mixed(const Rec64 *__restrict__ rec64, int2 rw, const Slot *__restrict__ blk,
                                          int32_t b, const double pm[3], const double r0[3], const double k[3],
                                          double L, double s_c, float eps, float e_abs, double &best, bool &redo,
                                          int32_t &j1)
{
    const Query32 Q = query32(pm, r0, k, s_c, eps, e_abs);
    const float inf = __builtin_huge_valf();
    float tw, ew;
    wall32(L, s_c, e_abs, tw, ew);
    float t1 = tw, err1 = ew;           // best estimate and its bound (the wall to begin with)
    int w1 = -1;                        // the winner's place in the row
    float lo_a = tw - ew, lo_b = inf;   // the two smallest lower bounds, lo_a <= lo_b
    bool graze = false;                 // a nearly parallel plane was met
    const int n = rw.y;
    const float4 *rec = reinterpret_cast<const float4 *>(blk + b + kHdrSlots);   // 8 records = 6 float4
    for (int e0 = 0; e0 < n; e0 += kBatch32) {
        float f[3 * kBatch32];
#pragma unroll
        for (int u = 0; u < 3 * kBatch32 / 4; ++u) {   // past the row end: the block offsets, padding or the next block, masked
            const float4 x = rec[3 * e0 / 4 + u];
            f[4 * u] = x.x;
            f[4 * u + 1] = x.y;
            f[4 * u + 2] = x.z;
            f[4 * u + 3] = x.w;
        }
        const int rem = n - e0;
        int ws = -1;   // the winner's slot in this batch, if it is in this batch
#pragma unroll
        for (int v = 0; v < kBatch32; ++v) {
            const bool in = v < rem;
            float t, err;
            bool pos, maybe;
            plane_bound32(f[3 * v], f[3 * v + 1], f[3 * v + 2], Q, t, err, pos, maybe);
            pos = pos && in;
            graze = graze || (maybe && in && !pos);
            const float lo = pos ? t - err : inf;
            // branch-free updates of the winner and of the two smallest lower bounds
            const bool w = pos && t < t1;
            t1 = w ? t : t1;
            err1 = w ? err : err1;
            ws = w ? v : ws;
            lo_b = __builtin_amdgcn_fmed3f(lo_a, lo_b, lo);
            lo_a = fminf(lo_a, lo);
        }
        w1 = ws >= 0 ? e0 + ws : w1;
    }
    // the winner's own lower bound, computed as in the loop; the smallest
    // lower bound of the others is lo_b if the winner holds the smallest
    const float lo1 = t1 - err1;
    const float lo_other = (lo1 == lo_a) ? lo_b : lo_a;
    if (graze || !(t1 + err1 < lo_other)) {
        redo = true;
        j1 = -1;
        return exit_fp64(rec64, rw, pm, r0, k, L, best);
    }
    redo = false;
    if (w1 < 0) {
        j1 = -1;
        best = L;
        return -1;
    }
    // the winner's block offset, stored after the records
    j1 = reinterpret_cast<const int32_t *>(reinterpret_cast<const float *>(rec) + 3 * n)[w1];
    return 0;
}

struct RayStats {
    int32_t cnt = 0, nfb = 0, nredo = 0, steps = 0, recs = 0;
};

// Ray set-up: normalised direction, chord length L (Eq. 5 on every axis),
// status, and s0, where the path starts (0, or with I.enter the distance at
// which a ray from outside enters the box: the largest over the axes of the
// distance to the near wall; it misses the box unless s0 < L).
// ENTER = false compiles the entry out (the kernels without the optional
// features, whose registers it would cost): every origin outside is OUTSIDE.
template <bool ENTER = true>
__device__ __forceinline__ uint8_t ray_setup(const GridRef &G, const RayIn &I, int64_t ray, double r0[3], double k[3],
                                             double &L, double &s0)
{
    for (int a = 0; a < 3; ++a) {
        r0[a] = I.origins[3 * ray + a];
        k[a] = I.dirs[3 * ray + a];
    }
    double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    bool inside = true;
    for (int a = 0; a < 3; ++a)
        if (!(r0[a] >= G.lo[a] && r0[a] <= G.hi[a])) inside = false;
    L = 0.0;
    s0 = 0.0;
    if (!(kn > 0.0) || !isfinite(kn)) return RAY_BADDIR;
    if (!inside && (!ENTER || !I.enter || !isfinite(r0[0]) || !isfinite(r0[1]) || !isfinite(r0[2])))
        return RAY_OUTSIDE;
    for (int a = 0; a < 3; ++a) k[a] /= kn;
    L = 1e308 * 10.0;
    for (int a = 0; a < 3; ++a) {
        if (k[a] > 0.0) {
            double s = (G.hi[a] - r0[a]) / k[a];
            if (s < L) L = s;
        } else if (k[a] < 0.0) {
            double s = (G.lo[a] - r0[a]) / k[a];
            if (s < L) L = s;
        }
    }
    if (ENTER && !inside) {
        for (int a = 0; a < 3; ++a) {
            if (k[a] > 0.0) {
                double s = (G.lo[a] - r0[a]) / k[a];
                if (s > s0) s0 = s;
            } else if (k[a] < 0.0) {
                double s = (G.hi[a] - r0[a]) / k[a];
                if (s > s0) s0 = s;
            } else if (r0[a] < G.lo[a] || r0[a] > G.hi[a]) {
                s0 = 1e308 * 10.0;
            }
        }
        if (!(s0 < L)) {
            L = 0.0;
            s0 = 0.0;
            return RAY_OUTSIDE;
        }
    }
    return RAY_OK;
}

// The point where the path starts.
__device__ __forceinline__ void start_point(const double r0[3], const double k[3], double s0, double q[3])
{
    for (int a = 0; a < 3; ++a) q[a] = s0 > 0.0 ? r0[a] + s0 * k[a] : r0[a];
}

// Per-lane state of a ray in flight.
struct RayState {
    double r0[3], k[3], pm[3];
    int2 rw;              // the current cell's row of neighbour records
    double L, s_c, tau;
    int64_t base, cap;    // window of this ray's first segments
    int32_t chunk;        // current spill chunk, -1 none yet, -2 spill exhausted
    int32_t ray;
#if VRT_VEC_STORE
    int32_t c0, c1, c2, c3, c4, c5, c6, c7;   // the last cells, oldest first, written 4, 8 or 16 at a time
    int32_t c8, c9, c10, c11, c12, c13, c14, c15;
    double l0, l1, l2, l3, l4, l5, l6, l7;    // the last lengths, written LG at a time
#endif
    int32_t m, uid;
    int32_t b;            // offset of the current cell's block
    int32_t qe;           // compact blocks: the current cell's scale exponent E
    double rho;           // the current cell's density from its block header (mixed mode with grid_rho)
    uint8_t st;
    double tstop, wgt, stop_s;   // transport outputs (kernels with Extras only)
    int32_t stop_uid;            // cell of the interaction point, -1 none yet
    int32_t dep_uid;             // deferred tally deposit of the last step: cell, -1 none
    double dep_len, dep_abs;     // ... and its two values
};

// Takes the wait for a loaded value here. The hardware counts a lane's
// loads and stores in one in-order counter, and where paths of a step merge
// the compiler waits for every load still outstanding on any of them: a
// value first used after the segment store would then hold the step until
// the store has completed as well.
template <class T>
__device__ __forceinline__ void settle(T &v)
{
    asm volatile("" : "+v"(v));
}

// The density held in the header of the block at offset b (FP64 mode: of
// the FP64 block).
template <int MODE>
__device__ __forceinline__ double block_rho(const GridRef &G, int32_t b)
{
    return reinterpret_cast<const BlockHdr *>((MODE == VOR_MODE_FP64 ? G.blk64 : G.blk) + b)->rho;
}

// The scale exponent E of a compact block from its header's length word.
__device__ __forceinline__ int32_t scale_exp(int32_t lenword) { return (int32_t)((uint32_t)lenword >> 24) - kScaleBias; }

// The block of the current cell R.m: where it starts (kept per cell when
// the grid has the starts, else derived from the row) and, for compact
// blocks, its scale exponent from the header. FP64 mode: its FP64 block.
template <int MODE>
__device__ __forceinline__ void enter_block(const GridRef &G, RayState &R)
{
    if (MODE == VOR_MODE_FP64) {
        R.b = G.blk64_off[R.m];
        return;
    }
    if (MODE != kModeCompact) {
        R.b = G.blk_off ? G.blk_off[R.m] : block_of(R.rw, R.m);
        return;
    }
    R.b = G.blk_off[R.m];
    R.qe = scale_exp(reinterpret_cast<const BlockHdr *>(G.blk + R.b)->len);
}

// The state a ray starts its first step with, settled (the loads of its
// set-up and start cell are waited for before the step, not after its
// first segment store).
__device__ __forceinline__ void settle_start(RayState &R)
{
    for (int a = 0; a < 3; ++a) {
        settle(R.r0[a]);
        settle(R.k[a]);
        settle(R.pm[a]);
    }
    settle(R.rw.x);
    settle(R.rw.y);
    settle(R.L);
    settle(R.s_c);
    settle(R.m);
    settle(R.uid);
    settle(R.b);
    settle(R.rho);
    settle(R.base);
    settle(R.cap);
}

template <int MODE>
__device__ __forceinline__ void ray_begin(const GridRef &G, RayState &R, double s0)
{
    R.s_c = s0;
    R.tau = 0.0;
    int32_t uid;
    double q[3];
    start_point(R.r0, R.k, s0, q);
    int32_t m = nearest_site(G.grid, q, &uid);
    Site sm = G.sites[m];
    R.m = m;
    R.uid = uid;
    R.pm[0] = sm.x;
    R.pm[1] = sm.y;
    R.pm[2] = sm.z;
    R.rw = G.rows[m];
    enter_block<MODE>(G, R);
}

// Start in cell m (internal index), found beforehand by nearest_site.
template <int MODE>
__device__ __forceinline__ void ray_begin_at(const GridRef &G, RayState &R, int32_t m, double s0)
{
    R.s_c = s0;
    R.tau = 0.0;
    const Site sm = G.sites[m];
    R.m = m;
    R.uid = (int32_t)sm.uid;
    R.pm[0] = sm.x;
    R.pm[1] = sm.y;
    R.pm[2] = sm.z;
    R.rw = G.rows[m];
    enter_block<MODE>(G, R);
}

// Slot of segment idx of the ray: its window, else its current spill chunk;
// null when the spill is exhausted or absent.
template <bool LP = false>
__device__ __forceinline__ int64_t segment_slot(const SegOut &O, const RayState &R, int64_t idx, bool &spill)
{
    if (idx < R.cap) {
        spill = false;
        return R.base + idx;
    }
    spill = true;
    if ((!LP && !O.spill_cell) || R.chunk < 0) return -1;
    return (int64_t)R.chunk * kSpillChunk + (idx - R.cap) % kSpillChunk;
}

// The arrays a slot from segment_slot indexes (LP: the pool's chunks follow
// the windows in the same arrays).
template <bool LP>
__device__ __forceinline__ int32_t *slot_cells(const SegOut &O, bool spill)
{
    return (spill && !LP) ? O.spill_cell : O.cell;
}
template <bool LP>
__device__ __forceinline__ double *slot_lens(const SegOut &O, bool spill)
{
    return (spill && !LP) ? O.spill_len : O.len;
}

// New spill chunks for the lanes that need one (need), each from its own
// pool (LP kernels, whose lanes may serve different pools): the lanes that
// share the first pending lane's pool take theirs with one atomic on the
// pool's counter, ranked by the ballot, and so on until every lane has one
// (or found its pool used up: chunk -2).
__device__ __forceinline__ void take_pool_chunks(const SpillPool *pool, RayState &R, bool need)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const unsigned long long me = (unsigned long long)(uintptr_t)pool;
    bool pend = need;
    for (uint64_t left = __ballot(pend); left; left = __ballot(pend)) {
        const int leader = __ffsll((long long)left) - 1;
        const unsigned long long lp = __shfl(me, leader, 64);
        const bool same = pend && me == lp;
        const uint64_t grp = __ballot(same);
        unsigned long long b = 0;
        if (lane == leader) b = atomicAdd(pool->head, (unsigned long long)__popcll(grp));
        b = __shfl(b, leader, 64);
        if (same) {
            const unsigned long long c = b + __popcll(grp & lt);
            if ((int64_t)c < pool->chunks) {
                const int64_t c0 = pool->base_chunk;
                pool->next[c] = -1;
                if (R.chunk < 0) pool->first[R.ray] = (int64_t)c;
                else pool->next[R.chunk - c0] = (int32_t)c;
                R.chunk = (int32_t)(c0 + (int64_t)c);   // in the window arrays' chunk numbering
            } else {
                R.chunk = -2;
            }
            pend = false;
        }
    }
}

// Store segment number idx of the ray: in its window, else in its spill
// chain. A new chunk is taken when a path reaches the first slot of one;
// lanes that do so in the same step share one atomic.
// Segments written together per lane: 16 cells (64 B) and 8 lengths (64 B),
// held in LDS until then (on windows that start on 8- but not 16-slot
// boundaries the cells go out 8 at a time), except in the FP64 kernels
// without the optional features, which write 4 of each (16 B and 32 B) from
// registers: measured, the wide groups made them slower (8% on a grid
// beyond the last-level cache), where they make the mixed and the
// transport kernels faster. Held in registers (VRT_LDS_STAGE = 0), the
// mixed-mode kernels without the optional features keep 16 and 8 and the
// others 4 of each, since more registers would cut their occupancy, and
// WIDE = false keeps 8 cells and 4 lengths (serving kernels).
template <int MODE, bool EXT>
constexpr bool narrow_fp64()
{
    return MODE == VOR_MODE_FP64 && !EXT;
}
template <int MODE, bool EXT, bool WIDE = true>
constexpr int cells_per_store()
{
    return (VRT_LDS_STAGE && WIDE && !narrow_fp64<MODE, EXT>()) ? 16
           : (MODE != VOR_MODE_FP64 && !EXT)                    ? (WIDE ? 16 : 8)
                                                                : 4;
}
template <int MODE, bool EXT, bool WIDE = true>
constexpr int lens_per_store()
{
    return (VRT_LDS_STAGE && WIDE && !narrow_fp64<MODE, EXT>()) ? 8
           : (WIDE && MODE != VOR_MODE_FP64 && !EXT)            ? 8
                                                                : 4;
}

// 16 bytes of segment output. The tracer stores them as ordinary stores:
// the L2 gathers a lane's 16-byte pieces of one line before writing it back,
// where non-temporal stores leave as separate partial writes. The serving
// kernel (LP: its spill chunks come from request pools) stores them
// non-temporal: its rays come in submission order, and there the records
// need the L2 more than the output lines do.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
template <bool LP, class V>
__device__ __forceinline__ void put16(V v, V *p)
{
    if (LP ? VRT_NT_STORE_SERVE : VRT_NT_STORE) __builtin_nontemporal_store(v, p);
    else *p = v;
}

#if VRT_VEC_STORE
// The groups of 16 cells and 8 lengths are held in LDS rather than in
// registers: a lane's segment number i goes to slot
// i mod 16 (cells) and i mod 8 (lengths) of its own column (slot-major, 256
// lanes of a block side by side), so a step writes one cell and one length
// there instead of shifting 32 registers, and the registers stay free for
// the exit search. 32 KB per block of 256 threads.
template <int CG, int LG, bool LP>
constexpr bool lds_stage()
{
    return VRT_LDS_STAGE && CG == 16 && LG == 8;
}
constexpr int kStageLanes = 256;   // threads per block of the kernels that stage
__device__ __forceinline__ int32_t *stage_cells()
{
    __shared__ int32_t s[16 * kStageLanes];
    return s;
}
__device__ __forceinline__ double *stage_lens()
{
    __shared__ double s[8 * kStageLanes];
    return s;
}

// Write the staged groups that end at segment idx (lengths when idx ends a
// group of 8; cells when it ends one of 16, or of 8 on windows that start
// on 8- but not 16-slot boundaries).
template <bool LP>
__device__ __forceinline__ void store_staged(const SegOut &O, const RayState &R, int64_t idx)
{
    const int t = threadIdx.x;
    const int32_t *sc = stage_cells();
    const double *sl = stage_lens();
    bool spill;
    const int64_t p = segment_slot<LP>(O, R, idx - 7, spill);
    if (p < 0) return;
    v2d *lp = reinterpret_cast<v2d *>(slot_lens<LP>(O, spill) + p);
    v4i *cp = reinterpret_cast<v4i *>(slot_cells<LP>(O, spill) + p);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        put16<LP>(v2d{sl[(2 * j) * kStageLanes + t], sl[(2 * j + 1) * kStageLanes + t]}, lp + j);
    if (O.vec < 2) {   // the last 8 cells
        const int b = (int)(idx & 8);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            put16<LP>(v4i{sc[(b + 4 * j) * kStageLanes + t], sc[(b + 4 * j + 1) * kStageLanes + t],
                          sc[(b + 4 * j + 2) * kStageLanes + t], sc[(b + 4 * j + 3) * kStageLanes + t]},
                      cp + j);
    } else if ((idx & 15) == 15) {   // the group of 16 started 8 slots earlier
#pragma unroll
        for (int j = 0; j < 4; ++j)
            put16<LP>(v4i{sc[(4 * j) * kStageLanes + t], sc[(4 * j + 1) * kStageLanes + t],
                          sc[(4 * j + 2) * kStageLanes + t], sc[(4 * j + 3) * kStageLanes + t]},
                      cp - 2 + j);
    }
}
#endif

template <int CG, int LG, bool LP = false>
__device__ __forceinline__ void store_segment(const SegOut &O, RayState &R, int64_t idx, int32_t cell, double len)
{
    if (LP) {
        const bool need = idx >= R.cap && ((idx - R.cap) % kSpillChunk) == 0 && R.chunk != -2;
        if (__ballot(need)) take_pool_chunks(O.pool, R, need);
    } else if (idx >= R.cap && O.spill_cell) {
        const int64_t k = idx - R.cap;
        const bool need = (k % kSpillChunk) == 0 && R.chunk != -2;
        const uint64_t bal = __ballot(need);
        if (bal) {
            const int lane = threadIdx.x & 63;
            const int leader = __ffsll((long long)bal) - 1;
            unsigned long long b = 0;
            if (lane == leader) b = atomicAdd(O.chunk_head, (unsigned long long)__popcll(bal));
            b = __shfl(b, leader, 64);
            if (need) {
                const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
                const int64_t c = (int64_t)b + __popcll(bal & lt);
                if (c < O.spill_chunks) {
                    O.spill_next[c] = -1;
                    if (R.chunk < 0) O.spill_first[R.ray] = c;
                    else O.spill_next[R.chunk] = (int32_t)c;
                    R.chunk = (int32_t)c;
                } else {
                    R.chunk = -2;
                }
            }
        }
    }
#if VRT_VEC_STORE
    if (lds_stage<CG, LG, LP>() && O.vec) {
        const int t = threadIdx.x;
        stage_cells()[(int)(idx & 15) * kStageLanes + t] = cell;
        stage_lens()[(int)(idx & 7) * kStageLanes + t] = len;
        if ((idx & 7) == 7) store_staged<LP>(O, R, idx);
        return;
    }
    if (O.vec) {
        // The cells go out CG and the lengths LG at a time: 64 B each with
        // CG = 16, LG = 8 (a partial write of the memory's write unit costs the
        // unit's read as well once the line leaves the L2 before the rest of
        // it is written).
        R.c0 = R.c1;
        R.c1 = R.c2;
        R.c2 = R.c3;
        if (CG >= 8) {
            R.c3 = R.c4;
            R.c4 = R.c5;
            R.c5 = R.c6;
            R.c6 = R.c7;
            if (CG == 16) {
                R.c7 = R.c8;
                R.c8 = R.c9;
                R.c9 = R.c10;
                R.c10 = R.c11;
                R.c11 = R.c12;
                R.c12 = R.c13;
                R.c13 = R.c14;
                R.c14 = R.c15;
                R.c15 = cell;
            } else {
                R.c7 = cell;
            }
        } else {
            R.c3 = cell;
        }
        R.l0 = R.l1;
        R.l1 = R.l2;
        R.l2 = R.l3;
        if (LG == 8) {
            R.l3 = R.l4;
            R.l4 = R.l5;
            R.l5 = R.l6;
            R.l6 = R.l7;
            R.l7 = len;
        } else {
            R.l3 = len;
        }
        if (LG == 8 && (idx & 7) == 7) {
            bool spill;
            const int64_t p = segment_slot<LP>(O, R, idx - 7, spill);
            if (p >= 0) {
                v2d *lp = reinterpret_cast<v2d *>(slot_lens<LP>(O, spill) + p);
                v4i *cp = reinterpret_cast<v4i *>(slot_cells<LP>(O, spill) + p);
                put16<LP>(v2d{R.l0, R.l1}, lp);
                put16<LP>(v2d{R.l2, R.l3}, lp + 1);
                put16<LP>(v2d{R.l4, R.l5}, lp + 2);
                put16<LP>(v2d{R.l6, R.l7}, lp + 3);
                if (CG == 8) {
                    put16<LP>(v4i{R.c0, R.c1, R.c2, R.c3}, cp);
                    put16<LP>(v4i{R.c4, R.c5, R.c6, R.c7}, cp + 1);
                } else if (O.vec < 2) {          // windows on 8-slot boundaries only: the last 8 cells
                    put16<LP>(v4i{R.c8, R.c9, R.c10, R.c11}, cp);
                    put16<LP>(v4i{R.c12, R.c13, R.c14, R.c15}, cp + 1);
                } else if ((idx & 15) == 15) {   // the group of 16 started 8 slots earlier
                    put16<LP>(v4i{R.c0, R.c1, R.c2, R.c3}, cp - 2);
                    put16<LP>(v4i{R.c4, R.c5, R.c6, R.c7}, cp - 1);
                    put16<LP>(v4i{R.c8, R.c9, R.c10, R.c11}, cp);
                    put16<LP>(v4i{R.c12, R.c13, R.c14, R.c15}, cp + 1);
                }
            }
        }
        if (LG == 4 && (idx & 3) == 3) {
            bool spill;
            const int64_t p = segment_slot<LP>(O, R, idx - 3, spill);   // groups of 8 never cross a window or chunk end
            if (p >= 0) {
                int32_t *cp = slot_cells<LP>(O, spill) + p;
                v2d *lp = reinterpret_cast<v2d *>(slot_lens<LP>(O, spill) + p);
                put16<LP>(v2d{R.l0, R.l1}, lp);
                put16<LP>(v2d{R.l2, R.l3}, lp + 1);
                if (CG == 4) {
                    put16<LP>(v4i{R.c0, R.c1, R.c2, R.c3}, reinterpret_cast<v4i *>(cp));
                } else if ((idx & 7) == 7) {
                    put16<LP>(v4i{R.c0, R.c1, R.c2, R.c3}, reinterpret_cast<v4i *>(cp - 4));
                    put16<LP>(v4i{R.c4, R.c5, R.c6, R.c7}, reinterpret_cast<v4i *>(cp));
                }
            }
        }
        return;
    }
#endif
    bool spill;
    const int64_t p = segment_slot<LP>(O, R, idx, spill);
    if (p >= 0) {
        slot_cells<LP>(O, spill)[p] = cell;
        slot_lens<LP>(O, spill)[p] = len;
    }
}

// Write the segments still held back when a path of n segments ends.
template <int CG, int LG, bool LP = false>
__device__ __forceinline__ void finish_segments(const SegOut &O, const RayState &R, int64_t n)
{
#if VRT_VEC_STORE
    if (!O.vec) return;
    const int cg = (CG == 16 && O.vec < 2) ? 8 : CG;                // 16 only on 16-slot windows
    const int rc = (int)(n & (cg - 1)), rl = (int)(n & (LG - 1));   // cells and lengths not yet written
    if (rc == 0) return;
    if (lds_stage<CG, LG, LP>()) {   // from the lane's LDS column
        const int t = threadIdx.x;
        for (int j = 0; j < rc; ++j) {
            const int64_t i = n - rc + j;
            bool spill;
            const int64_t p = segment_slot<LP>(O, R, i, spill);
            if (p >= 0) {
                slot_cells<LP>(O, spill)[p] = stage_cells()[(int)(i & 15) * kStageLanes + t];
                if (j >= rc - rl) slot_lens<LP>(O, spill)[p] = stage_lens()[(int)(i & 7) * kStageLanes + t];
            }
        }
        return;
    }
    // the held cells, right-aligned in 16 entries
    int32_t cs[16] = {R.c0, R.c1, R.c2, R.c3, R.c4, R.c5, R.c6, R.c7, R.c8, R.c9, R.c10, R.c11, R.c12, R.c13, R.c14, R.c15};
    if (CG == 8) {
        const int32_t t[8] = {R.c0, R.c1, R.c2, R.c3, R.c4, R.c5, R.c6, R.c7};
        for (int i = 0; i < 8; ++i) cs[8 + i] = t[i];
    } else if (CG == 4) {
        const int32_t t[4] = {R.c0, R.c1, R.c2, R.c3};
        for (int i = 0; i < 4; ++i) cs[12 + i] = t[i];
    }
    const double ls[8] = {LG == 8 ? R.l0 : 0.0, LG == 8 ? R.l1 : 0.0, LG == 8 ? R.l2 : 0.0, LG == 8 ? R.l3 : 0.0,
                          LG == 8 ? R.l4 : R.l0, LG == 8 ? R.l5 : R.l1, LG == 8 ? R.l6 : R.l2, LG == 8 ? R.l7 : R.l3};
#pragma unroll
    for (int j = 0; j < CG - 1; ++j) {
        if (j < rc) {
            bool spill;
            const int64_t p = segment_slot<LP>(O, R, n - rc + j, spill);
            if (p >= 0) {
                slot_cells<LP>(O, spill)[p] = cs[16 - rc + j];
                if (j >= rc - rl) slot_lens<LP>(O, spill)[p] = ls[8 - rc + j];
            }
        }
    }
#else
    (void)O;
    (void)R;
    (void)n;
#endif
}

// First part of a step: false once the path has ended (at the wall, or at
// the step limit, which sets the status).
__device__ __forceinline__ bool ray_step_begin(const GridRef &G, RayState &R, RayStats &S)
{
    if (!(R.L > 0.0)) return false;
    if (S.steps > G.max_steps) {
        R.st = RAY_STEPLIMIT;
        return false;
    }
    ++S.steps;
    S.recs += R.rw.y;
    return true;
}

// Rest of a step, given the exit search's result: record index win (-1: the
// chord end), best = the FP64 crossing when redo (or when win < 0), else the
// block offset j1 of the winner (its FP64 crossing is computed here from the
// site in the block header). Emits the segment, accumulates tau,
// moves to the next cell; the no-exit fallback of Sect. 2.2 when the current
// point lies beyond a plane of the cell. Returns false once the path ended.
// The absorbed fraction exp(-tau) (1 - exp(-dt)), kept out of line: inlined,
// the FP64 exp and expm1 raise the traversal kernel's register count past
// what three waves per SIMD allow.
__device__ __noinline__ double absorbed_fraction(double tau, double dt) { return exp(-tau) * -expm1(-dt); }

// Tallies of a segment of length l in the current cell (kr = kappa rho),
// with R.tau the optical depth before it: added at once, or (DEFER) kept in
// R.dep_* for the caller to add where the wave is converged.
template <bool DEFER>
__device__ __forceinline__ void deposit(const Extras &X, RayState &R, double l, double kr)
{
    const double vl = R.wgt * l;
    const double va = X.tally_abs ? R.wgt * absorbed_fraction(R.tau, kr * l) : 0.0;
    if (DEFER) {
        R.dep_uid = R.uid;
        R.dep_len = vl;
        R.dep_abs = va;
    } else {
        if (X.tally_len) atomicAdd(&X.tally_len[R.uid], vl);
        if (X.tally_abs) atomicAdd(&X.tally_abs[R.uid], va);
    }
}

// Transport set-up of a ray that has started (status known, start cell set).
__device__ __forceinline__ void ray_extras_begin(const Extras &X, int64_t ray, RayState &R)
{
    R.tstop = X.tau_stop ? X.tau_stop[ray] : 0.0;
    R.wgt = X.weight ? X.weight[ray] : 1.0;
    R.stop_uid = -1;
    R.stop_s = 0.0;
    R.dep_uid = -1;
    if (X.tau_stop && R.st == RAY_OK && R.tstop <= 0.0) {   // used up where the path starts: no segment
        R.stop_uid = R.uid;
        R.stop_s = R.s_c;
        R.L = 0.0;
    }
}

__device__ __forceinline__ void ray_extras_finish(const Extras &X, int64_t ray, const RayState &R)
{
    if (!X.tau_stop) return;
    X.stop_cell[ray] = R.stop_uid;
    if (X.stop_s) X.stop_s[ray] = R.stop_uid >= 0 ? R.stop_s : R.L;
}

template <int MODE, bool SEGS, bool EXT = false, bool DEFER = false, bool WIDE = true, bool LP = false>
__device__ __forceinline__ bool ray_step_end(const GridRef &G, const RayIn &I, RayState &R, RayStats &S,
                                             const SegOut &O, int win, double best, bool redo, int32_t j1,
                                             const Extras &X)
{
    // The current cell's density. Bound to the grid: mixed mode read it with
    // the cell's block header when the ray entered the cell; FP64 mode takes
    // it from the copy in internal order, whose lines neighbouring cells
    // share (carried in registers it would cost the FP64 kernel its fourth
    // wave per SIMD). Else from the caller's array, loaded before the
    // winner's header or record so that one wait covers both (loaded after
    // the segment store, its wait would also hold the step until the store
    // completed).
    const bool has_rho = I.grid_rho || I.density;
    double rho = 0.0, wrho = 0.0;
    if (I.grid_rho) rho = (MODE == VOR_MODE_FP64) ? G.rho_int[R.m] : R.rho;
    else if (I.density) rho = I.density[R.uid];
    int32_t wj = -1, wuid = 0;
    double wx = 0.0, wy = 0.0, wz = 0.0;
    int2 wrow = make_int2(0, 0);
    int32_t wqe = 0;
    if (win >= 0) {
        if (MODE != VOR_MODE_FP64 && redo) {
            const Rec64 w = G.rec64[win];
            wj = w.j;
            wuid = w.uid;
            wx = w.x;
            wy = w.y;
            wz = w.z;
            wrow = G.rows[wj];
            settle(wj);
            settle(wuid);
            settle(wx);
            settle(wy);
            settle(wz);
            settle(wrow.x);
            settle(wrow.y);
        } else {
            // the winner's block header as its three 16-byte slots: {x, y}, {z, rho},
            // {uid, j, len, row start}; in FP64 mode its FP64 block, whose offset
            // follows the current block's records
            const Slot *B = (MODE == VOR_MODE_FP64) ? G.blk64 : G.blk;
            if (MODE == VOR_MODE_FP64) j1 = fp64_block_offsets(G.blk64, R.b, R.rw.y)[win];
            const double2 s0 = *reinterpret_cast<const double2 *>(B + j1);
            const double2 s1 = *reinterpret_cast<const double2 *>(B + j1 + 1);
            const int4 s2 = *reinterpret_cast<const int4 *>(B + j1 + 2);
            wx = s0.x;
            wy = s0.y;
            wz = s1.x;
            if (MODE != VOR_MODE_FP64 && I.grid_rho) wrho = s1.y;
            wuid = s2.x;
            wj = s2.y;
            if (MODE == kModeCompact) {
                wrow = make_int2(s2.w, s2.z & kLenMask);
                wqe = scale_exp(s2.z);
            } else {
                wrow = make_int2(s2.w, s2.z);
            }
            if (MODE != VOR_MODE_FP64) {   // FP64 mode found it in the search
                double den;
                best = cross_fp64(wx, wy, wz, R.pm, R.r0, R.k, den);
            }
            settle(wrho);
        }
    }
    settle(rho);
    double len = best - R.s_c;
    if (len > 0.0) {
        if (EXT) {
            const double kr = has_rho ? I.kappa * rho : 0.0;
            if (X.tau_stop) {
                const double tn = R.tau + kr * len;
                if (kr > 0.0 && tn >= R.tstop) {   // the package interacts in this cell
                    const double lp = (R.tstop - R.tau) / kr;
                    if (SEGS) store_segment<cells_per_store<MODE, EXT, WIDE>(), lens_per_store<MODE, EXT, WIDE>(), LP>(O, R, S.cnt, R.uid, lp);
                    deposit<DEFER>(X, R, lp, kr);
                    R.tau = R.tau + kr * lp;
                    ++S.cnt;
                    R.stop_uid = R.uid;
                    R.stop_s = R.s_c + lp;
                    return false;
                }
            }
            deposit<DEFER>(X, R, len, kr);
        }
        if (has_rho) R.tau += I.kappa * rho * len;   // before the store: its wait then holds no store
        if (SEGS) store_segment<cells_per_store<MODE, EXT, WIDE>(), lens_per_store<MODE, EXT, WIDE>(), LP>(O, R, S.cnt, R.uid, len);
        ++S.cnt;
        R.s_c = best;
    } else if (len < -1e-9 * R.L) {
        // The current point lies well beyond a plane of this cell: the
        // neighbour table missed a cell. Advance a small distance without a
        // segment and locate the point again (the no-exit fallback of
        // Sect. 2.2).
        R.s_c += G.eps_fb;
        ++S.nfb;
        if (R.s_c >= R.L) return false;
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = R.r0[a] + R.s_c * R.k[a];
        int32_t uid;
        R.m = nearest_site(G.grid, r, &uid);
        R.uid = uid;
        Site sm = G.sites[R.m];
        R.pm[0] = sm.x;
        R.pm[1] = sm.y;
        R.pm[2] = sm.z;
        R.rw = G.rows[R.m];
        settle(R.pm[0]);
        settle(R.pm[1]);
        settle(R.pm[2]);
        settle(R.rw.x);
        settle(R.rw.y);
        enter_block<MODE>(G, R);
        if (MODE != VOR_MODE_FP64 && I.grid_rho) {
            R.rho = block_rho<MODE>(G, R.b);
            settle(R.rho);
        }
        return true;
    }
    if (wj < 0) return false;
    R.m = wj;
    R.uid = wuid;
    R.pm[0] = wx;
    R.pm[1] = wy;
    R.pm[2] = wz;
    R.rw = wrow;
    if (MODE == VOR_MODE_FP64) {
        R.b = j1;
    } else if (redo) {
        enter_block<MODE>(G, R);
        if (I.grid_rho) {
            R.rho = block_rho<MODE>(G, R.b);
            settle(R.rho);
        }
        if (MODE == kModeCompact) settle(R.qe);
    } else {
        R.b = j1;
        if (MODE == kModeCompact) R.qe = wqe;
        if (I.grid_rho) R.rho = wrho;
    }
    return true;
}

// One exit-point step (Sect. 2.2) with the exit search done by this lane
// alone. Returns false once the path has ended.
template <int MODE, bool SEGS, bool EXT = false, bool DEFER = false, bool WIDE = true, bool LP = false>
__device__ __forceinline__ bool ray_step(const GridRef &G, const RayIn &I, RayState &R, RayStats &S, const SegOut &O,
                                         const Extras &X = Extras{})
{
    if (!ray_step_begin(G, R, S)) return false;
    double best;
    bool redo = false;
    int32_t j1 = -1;
    int win;
    if (MODE == VOR_MODE_FP64) {
        win = exit_fp64_blk(G.blk64, R.b, R.rw.y, R.pm, R.r0, R.k, R.L, best);
    } else {
        if (MODE == kModeCompact)
            win = exit_mixed_compact(G.rec64, R.rw, G.blk, R.b, R.pm, R.r0, R.k, R.L, R.s_c, G.eps_mix, G.eps_abs,
                                     best, redo, j1, ldexp(1.0, kQShift - R.qe));
        else
            win = exit_mixed(G.rec64, R.rw, G.blk, R.b, R.pm, R.r0, R.k, R.L, R.s_c, G.eps_mix, G.eps_abs, best,
                             redo, j1);
        S.nredo += redo ? 1 : 0;
    }
    return ray_step_end<MODE, SEGS, EXT, DEFER, WIDE, LP>(G, I, R, S, O, win, best, redo, j1, X);
}

}  // namespace vrt
