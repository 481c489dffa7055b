// trace.hip -- vor_locate and vor_trace: the cell-location function C(r)
// (Sect. 2.3) and the straight-path loop (Sect. 2.2, Eqs. 1-5), one ray per
// lane.
//
// Every crossing is measured from the ray's origin r0:
//     s_j = n.((p_j + p_m)/2 - r0) / (n.k),   n = p_j - p_m,
// which is Eq. 4 with the current point r = r0 + s_c k substituted and s
// counted from r0, so no position error builds up along the path. Only
// neighbours with n.k > 0 are evaluated (the sign argument of Sect. 2.2),
// the chord end L (Eq. 5 on every axis) is always a candidate, and a
// crossing at or behind the current position moves to that neighbour
// without emitting a segment.
//
// Mixed mode ranks the neighbours with FP32 offsets and a rounding-error
// bound per crossing; when the bounds of the best and any other candidate
// overlap the whole step is redone in FP64, otherwise only the winner's
// crossing is recomputed in FP64. Either way the emitted values are the FP64
// ones.
#include "vrt_internal.h"

using namespace vrt;

const vrt::Grid &vrt_grid_of(const vor_grid *G);

namespace {

struct TraceArgs {
    const Site *sites;
    const int2 *rows;
    const Rec64 *rec64;
    const Rec32 *rec32;
    BucketGridView grid;
    double lo[3], hi[3];
    const double *origins;
    const double *dirs;
    int64_t N;
    const double *density;
    double kappa;
    int32_t max_steps;
    float eps_mix;
    double eps_fb;        // fallback advance
    double *tau;
    int32_t *n_seg;
    uint8_t *status;
    int32_t *n_fb;
    int32_t *seg_cell;
    double *seg_len;
    int64_t seg_stride;
    const int64_t *ray_off;
    unsigned long long *counters;
    // spill of paths longer than their window (stride mode)
    int64_t *work;        // [0] persistent queue head, [1] spill slots used, [2] spilled rays
    int32_t *spill_rays;
    int64_t *spill_off;
    int32_t *spill_cell;
    double *spill_len;
    int64_t spill_capacity;
};

constexpr int kBatch64 = 4;    // FP64 records loaded together
constexpr int kBatch32 = 8;    // FP32 records loaded together

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

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
        Rec64 q[kBatch64];
#pragma unroll
        for (int u = 0; u < kBatch64; ++u)
            if (e0 + u < end) q[u] = rec[e0 + u];
#pragma unroll
        for (int u = 0; u < kBatch64; ++u) {
            if (e0 + u >= end) break;
            double den;
            double sj = cross_fp64(q[u].x, q[u].y, q[u].z, pm, r0, k, den);
            if (!(den > 0.0)) continue;
            if (sj < best || (sj == best && win >= 0 && (den > best_den || (den == best_den && q[u].j < win_j)))) {
                best = sj;
                best_den = den;
                win = e0 + u;
                win_j = q[u].j;
            }
        }
    }
    return win;
}

// Mixed-precision exit search. Every plane is ranked with FP32 offsets and
// a bound on the FP32 rounding error of its crossing,
//   err = eps * (1.5 |n|^2 + 0.5 (|q| + |t|)^2) / (n.k) + 4u |t|,
// (q = current point - p_m, t = the FP32 crossing, u = 2^-24; eps >= 12u
// covers the rounding of n, q, k and of the products, the AM-GM step
// |n|(|q|+|t|) <= (|n|^2 + (|q|+|t|)^2)/2 turns the bound into this form).
// If the upper bound of the best candidate is below the lower bound of every
// other one (the wall included) the FP32 ranking is certain, and only the
// winner's crossing is recomputed in FP64 (from the FP64 record, same
// arithmetic as exit_fp64); otherwise the step is redone in FP64. Either way
// the result equals exit_fp64's.
__device__ __forceinline__ int exit_mixed(const Rec64 *__restrict__ rec64, const Rec32 *__restrict__ rec32, int2 rw,
                                          const double pm[3], const double r0[3], const double k[3], double L,
                                          double s_c, float eps, double &best, bool &redo)
{
    double q64[3];
    for (int a = 0; a < 3; ++a) q64[a] = (r0[a] + s_c * k[a]) - pm[a];
    const float qx = (float)q64[0], qy = (float)q64[1], qz = (float)q64[2];
    const float kx = (float)k[0], ky = (float)k[1], kz = (float)k[2];
    const float qa = sqrtf(qx * qx + qy * qy + qz * qz);
    const float u = 5.9604645e-8f;   // 2^-24
    const float tw = (float)(L - s_c);   // the wall, relative to the current point
    const float ew = 2.0f * u * fabsf(tw);
    float t1 = tw, hi1 = tw + ew;       // best estimate and its upper bound
    int e1 = -1;
    float lo_a = tw - ew, lo_b = 3.0e38f;   // two smallest lower bounds
    int ia = -1;
    const int end = rw.x + rw.y;
    for (int e0 = rw.x; e0 < end; e0 += kBatch32) {
        Rec32 r[kBatch32];
#pragma unroll
        for (int v = 0; v < kBatch32; ++v)
            if (e0 + v < end) r[v] = rec32[e0 + v];
#pragma unroll
        for (int v = 0; v < kBatch32; ++v) {
            if (e0 + v >= end) break;
            float den = r[v].nx * kx + r[v].ny * ky + r[v].nz * kz;
            if (!(den > 0.0f)) continue;
            float nn = r[v].nx * r[v].nx + r[v].ny * r[v].ny + r[v].nz * r[v].nz;
            float num = 0.5f * nn - (r[v].nx * qx + r[v].ny * qy + r[v].nz * qz);
            float t = num / den;
            float at = fabsf(t);
            float sq = qa + at;
            float err = eps * (1.5f * nn + 0.5f * sq * sq) / den + 4.0f * u * at;
            float lo = t - err;
            if (t < t1) {
                t1 = t;
                hi1 = t + err;
                e1 = e0 + v;
            }
            if (lo < lo_a) {
                lo_b = lo_a;
                lo_a = lo;
                ia = e0 + v;
            } else if (lo < lo_b) {
                lo_b = lo;
            }
        }
    }
    float lo_other = (ia == e1) ? lo_b : lo_a;
    if (!(hi1 < lo_other)) {
        redo = true;
        return exit_fp64(rec64, rw, pm, r0, k, L, best);
    }
    redo = false;
    if (e1 < 0) {
        best = L;
        return -1;
    }
    const Rec64 w = rec64[e1];
    double den;
    best = cross_fp64(w.x, w.y, w.z, pm, r0, k, den);
    return e1;
}

struct RayStats {
    int32_t cnt = 0, nfb = 0, nredo = 0, steps = 0, recs = 0;
};

// Ray set-up: normalised direction, chord length L (Eq. 5 on every axis),
// status. Returns false when the ray has no path.
__device__ __forceinline__ uint8_t ray_setup(const TraceArgs &A, int64_t ray, double r0[3], double k[3], double &L)
{
    for (int a = 0; a < 3; ++a) {
        r0[a] = A.origins[3 * ray + a];
        k[a] = A.dirs[3 * ray + a];
    }
    double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    bool inside = true;
    for (int a = 0; a < 3; ++a)
        if (!(r0[a] >= A.lo[a] && r0[a] <= A.hi[a])) inside = false;
    L = 0.0;
    if (!(kn > 0.0) || !isfinite(kn)) return RAY_BADDIR;
    if (!inside) return RAY_OUTSIDE;
    for (int a = 0; a < 3; ++a) k[a] /= kn;
    L = 1e308 * 10.0;
    for (int a = 0; a < 3; ++a) {
        if (k[a] > 0.0) {
            double s = (A.hi[a] - r0[a]) / k[a];
            if (s < L) L = s;
        } else if (k[a] < 0.0) {
            double s = (A.lo[a] - r0[a]) / k[a];
            if (s < L) L = s;
        }
    }
    return RAY_OK;
}

// Per-lane state of a ray in flight.
struct RayState {
    double r0[3], k[3], pm[3];
    double L, s_c, tau;
    int64_t base, cap;
    int64_t skip;         // segments with a smaller index are not written
    int32_t m, uid;
    uint8_t st;
};

__device__ __forceinline__ void ray_begin(const TraceArgs &A, RayState &R)
{
    R.s_c = 0.0;
    R.tau = 0.0;
    int32_t uid;
    int32_t m = nearest_site(A.grid, R.r0, &uid);
    Site sm = A.sites[m];
    R.m = m;
    R.uid = uid;
    R.pm[0] = sm.x;
    R.pm[1] = sm.y;
    R.pm[2] = sm.z;
}

// One exit-point step (Sect. 2.2). Returns false once the path has ended.
template <int MODE, bool SEGS>
__device__ __forceinline__ bool ray_step(const TraceArgs &A, RayState &R, RayStats &S, int32_t *seg_cell,
                                         double *seg_len)
{
    if (!(R.L > 0.0)) return false;
    if (S.steps > A.max_steps) {
        R.st = RAY_STEPLIMIT;
        return false;
    }
    ++S.steps;
    const int2 rw = A.rows[R.m];
    S.recs += rw.y;
    double best;
    int win;
    if (MODE == VOR_MODE_FP64) {
        win = exit_fp64(A.rec64, rw, R.pm, R.r0, R.k, R.L, best);
    } else {
        bool redo;
        win = exit_mixed(A.rec64, A.rec32, rw, R.pm, R.r0, R.k, R.L, R.s_c, A.eps_mix, best, redo);
        S.nredo += redo ? 1 : 0;
    }
    double len = best - R.s_c;
    if (len > 0.0) {
        if (SEGS && S.cnt < R.cap && S.cnt >= R.skip) {
            seg_cell[R.base + S.cnt] = R.uid;
            seg_len[R.base + S.cnt] = len;
        }
        if (A.density) R.tau += A.kappa * A.density[R.uid] * len;
        ++S.cnt;
        R.s_c = best;
    } else if (len < -1e-9 * R.L) {
        // The current point lies well beyond a plane of this cell: the
        // neighbour table missed a cell. Advance a small distance without a
        // segment and locate the point again (the no-exit fallback of
        // Sect. 2.2).
        R.s_c += A.eps_fb;
        ++S.nfb;
        if (R.s_c >= R.L) return false;
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = R.r0[a] + R.s_c * R.k[a];
        int32_t uid;
        R.m = nearest_site(A.grid, r, &uid);
        R.uid = uid;
        Site sm = A.sites[R.m];
        R.pm[0] = sm.x;
        R.pm[1] = sm.y;
        R.pm[2] = sm.z;
        return true;
    }
    if (win < 0) return false;
    const Rec64 w = A.rec64[win];
    R.m = w.j;
    R.uid = w.uid;
    R.pm[0] = w.x;
    R.pm[1] = w.y;
    R.pm[2] = w.z;
    return true;
}

// Output window of ray `ray` in the main pass.
template <bool SEGS>
__device__ __forceinline__ void ray_window(const TraceArgs &A, int64_t ray, RayState &R)
{
    R.base = 0;
    R.cap = 0;
    R.skip = 0;
    if (SEGS) {
        if (A.seg_stride > 0) {
            R.base = ray * A.seg_stride;
            R.cap = A.seg_stride;
        } else {
            R.base = A.ray_off[ray];
            R.cap = A.ray_off[ray + 1] - R.base;
        }
    }
}

// Results of a finished ray; a path longer than its stride window gets a
// slot range in the spill (when one is given) for the part past the
// window, which the spill pass writes.
template <bool SEGS>
__device__ __forceinline__ void ray_finish(const TraceArgs &A, int64_t ray, RayState &R, const RayStats &S)
{
    if (SEGS && R.st == RAY_OK && S.cnt > R.cap) {
        bool spilled = false;
        if (A.spill_cell && A.seg_stride > 0) {
            const int64_t tail = S.cnt - R.cap;
            unsigned long long off = atomicAdd((unsigned long long *)&A.work[1], (unsigned long long)tail);
            if ((int64_t)off + tail <= A.spill_capacity) {
                A.spill_off[ray] = (int64_t)off;
                unsigned long long idx = atomicAdd((unsigned long long *)&A.work[2], 1ull);
                A.spill_rays[idx] = (int32_t)ray;
                spilled = true;
            }
        }
        if (!spilled) R.st = RAY_OVERFLOW;
    }
    A.tau[ray] = R.tau;
    A.n_seg[ray] = S.cnt;
    if (A.status) A.status[ray] = R.st;
    if (A.n_fb) A.n_fb[ray] = S.nfb;
}

__device__ __forceinline__ void flush_counters(const TraceArgs &A, const RayStats &S)
{
    if (!A.counters) return;
    unsigned long long c0 = wave_sum((unsigned long long)S.cnt);
    unsigned long long c1 = wave_sum((unsigned long long)S.nfb);
    unsigned long long c2 = wave_sum((unsigned long long)S.nredo);
    unsigned long long c3 = wave_sum((unsigned long long)S.steps);
    unsigned long long c4 = wave_sum((unsigned long long)S.recs);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&A.counters[0], c0);
        if (c1) atomicAdd(&A.counters[1], c1);
        if (c2) atomicAdd(&A.counters[2], c2);
        atomicAdd(&A.counters[3], c3);
        atomicAdd(&A.counters[4], c4);
    }
}

// One ray per lane.
template <int MODE, bool SEGS>
__global__ void __launch_bounds__(256) k_trace(TraceArgs A)
{
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    RayStats S;
    if (ray < A.N) {
        RayState R;
        R.st = ray_setup(A, ray, R.r0, R.k, R.L);
        ray_window<SEGS>(A, ray, R);
        R.tau = 0.0;
        if (R.st == RAY_OK) {
            ray_begin(A, R);
            while (ray_step<MODE, SEGS>(A, R, S, A.seg_cell, A.seg_len)) {
            }
        }
        ray_finish<SEGS>(A, ray, R, S);
    }
    flush_counters(A, S);
}

// Persistent waves: every lane keeps a ray in flight; when rays end, the
// wave's idle lanes take the next rays from the work queue together (one
// atomic per wave, ranks from the ballot).
template <int MODE, bool SEGS>
__global__ void __launch_bounds__(256) k_trace_persistent(TraceArgs A)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    RayStats S, T;   // S: current ray, T: totals of this lane
    RayState R;
    int64_t ray = -1;
    bool live = false;
    unsigned long long *head = (unsigned long long *)&A.work[0];
    bool drained = false;   // wave-uniform: the queue has run out
    for (;;) {
        bool need = !live;
        uint64_t want = __ballot(need);
        if (want && !drained) {
            int n = __popcll(want);
            unsigned long long base0 = 0;
            if (lane == __ffsll((long long)want) - 1) base0 = atomicAdd(head, (unsigned long long)n);
            base0 = __shfl(base0, __ffsll((long long)want) - 1, 64);
            if (need) {
                ray = (int64_t)(base0 + __popcll(want & lt));
                if (ray < A.N) {
                    S = RayStats();
                    R.st = ray_setup(A, ray, R.r0, R.k, R.L);
                    ray_window<SEGS>(A, ray, R);
                    R.tau = 0.0;
                    live = true;
                    if (R.st == RAY_OK) ray_begin(A, R);
                    else R.L = 0.0;
                } else {
                    ray = -1;
                }
            }
            drained = __ballot(need && ray < 0) != 0ull;
        }
        if (__ballot(live) == 0ull) break;   // the queue is drained and every ray has ended
        if (live) {
            if (!ray_step<MODE, SEGS>(A, R, S, A.seg_cell, A.seg_len)) {
                ray_finish<SEGS>(A, ray, R, S);
                T.cnt += S.cnt;
                T.nfb += S.nfb;
                T.nredo += S.nredo;
                T.steps += S.steps;
                T.recs += S.recs;
                live = false;
            }
        }
    }
    flush_counters(A, T);
}

// Spill pass: rays whose path outgrew their stride window are traced again
// and write the segments past the window at their spill offset. Grid-stride
// over the spilled rays counted by the main pass.
template <int MODE>
__global__ void __launch_bounds__(256) k_trace_spill(TraceArgs A)
{
    const int64_t n = A.work[2];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ray = A.spill_rays[i];
        RayState R;
        RayStats S;
        R.st = ray_setup(A, ray, R.r0, R.k, R.L);
        R.skip = A.seg_stride;
        R.base = A.spill_off[ray] - A.seg_stride;
        R.cap = 1ll << 62;
        if (R.st == RAY_OK) {
            ray_begin(A, R);
            while (ray_step<MODE, true>(A, R, S, A.spill_cell, A.spill_len)) {
            }
        }
    }
}

__global__ void k_zero_i64(int64_t *p, int n)
{
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_locate(BucketGridView g, double lo0, double lo1, double lo2, double hi0,
                                                double hi1, double hi2, const double *__restrict__ pts, int64_t N,
                                                int32_t *__restrict__ cell)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double q[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    if (!(q[0] >= lo0 && q[0] <= hi0 && q[1] >= lo1 && q[1] <= hi1 && q[2] >= lo2 && q[2] <= hi2)) {
        cell[i] = -1;
        return;
    }
    int32_t uid;
    nearest_site(g, q, &uid);
    cell[i] = uid;
}

}  // namespace

extern "C" vor_status vor_locate(const vor_grid *G, const double *pts, int64_t N, int32_t *cell, void *stream)
{
    if (!G || N < 0 || (N > 0 && (!pts || !cell))) return VOR_EINVAL;
    if (N == 0) return VOR_OK;
    const Grid &g = vrt_grid_of(G);
    const int T = 256;
    int64_t blocks = (N + T - 1) / T;
    if (blocks > 0x7fffffff) return VOR_EINVAL;
    hipLaunchKernelGGL(k_locate, dim3((unsigned)blocks), dim3(T), 0, (hipStream_t)stream, bucket_view(g), g.box[0],
                       g.box[1], g.box[2], g.box[3], g.box[4], g.box[5], pts, N, cell);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

extern "C" vor_status vor_trace(const vor_grid *G, const double *origins, const double *dirs, int64_t N,
                                const double *density, double kappa, const vor_trace_opts *opts,
                                const vor_trace_out *out, void *stream)
{
    if (!G || N < 0 || !out) return VOR_EINVAL;
    if (N == 0) return VOR_OK;
    if (N > 0x7fffffffLL) return VOR_EINVAL;
    if (!origins || !dirs || !out->tau || !out->n_seg) return VOR_EINVAL;
    const bool segs = out->seg_cell != nullptr;
    if (segs && (!out->seg_len || (out->seg_stride <= 0 && !out->ray_off))) return VOR_EINVAL;
    if (!segs && out->seg_len) return VOR_EINVAL;
    if (out->seg_stride < 0) return VOR_EINVAL;
    const bool spill = out->spill_cell != nullptr;
    if (spill && (!segs || out->seg_stride <= 0 || !out->spill_len || !out->spill_off || !out->spill_rays ||
                  !out->work || out->spill_capacity < 0))
        return VOR_EINVAL;
    int mode = opts ? opts->mode : VOR_MODE_FP64;
    if (mode != VOR_MODE_FP64 && mode != VOR_MODE_MIXED) return VOR_EINVAL;
    if (opts && (opts->max_steps < 0 || opts->eps_mix < 0 || !(opts->eps_mix < 1.0))) return VOR_EINVAL;
    const bool persistent = opts && opts->persistent;
    if (persistent && !out->work) return VOR_EINVAL;
    const Grid &g = vrt_grid_of(G);
    TraceArgs A;
    A.sites = g.sites;
    A.rows = g.rows;
    A.rec64 = g.rec64;
    A.rec32 = g.rec32;
    A.grid = bucket_view(g);
    for (int a = 0; a < 3; ++a) {
        A.lo[a] = g.box[a];
        A.hi[a] = g.box[a + 3];
    }
    A.origins = origins;
    A.dirs = dirs;
    A.N = N;
    A.density = density;
    A.kappa = kappa;
    A.max_steps = (opts && opts->max_steps > 0) ? opts->max_steps : (int32_t)std::min<int64_t>(g.M + 16, 0x7fffffff);
    A.eps_mix = (float)((opts && opts->eps_mix > 0) ? opts->eps_mix : 1.9073486328125e-06);   // 2^-19
    double diag = 0.0;
    for (int a = 0; a < 3; ++a) diag += (g.box[a + 3] - g.box[a]) * (g.box[a + 3] - g.box[a]);
    A.eps_fb = 1e-12 * sqrt(diag);
    A.tau = out->tau;
    A.n_seg = out->n_seg;
    A.status = out->status;
    A.n_fb = out->n_fallback;
    A.seg_cell = out->seg_cell;
    A.seg_len = out->seg_len;
    A.seg_stride = out->seg_stride;
    A.ray_off = out->ray_off;
    A.counters = out->counters;
    A.work = out->work;
    A.spill_rays = out->spill_rays;
    A.spill_off = out->spill_off;
    A.spill_cell = out->spill_cell;
    A.spill_len = out->spill_len;
    A.spill_capacity = out->spill_capacity;
    hipStream_t st = (hipStream_t)stream;
    const int T = 256;
    if (A.work) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, A.work, 4);
    if (spill) {
        int64_t nb = std::min<int64_t>((N + T - 1) / T, 65535);
        hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)nb), dim3(T), 0, st, A.spill_off, N, (int64_t)-1);
    }
    dim3 block(T);
    if (persistent) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return VOR_EDEVICE;
        hipError_t e;
        if (mode == VOR_MODE_FP64)
            e = segs ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<VOR_MODE_FP64, true>, T, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<VOR_MODE_FP64, false>, T, 0);
        else
            e = segs ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<VOR_MODE_MIXED, true>, T, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_persistent<VOR_MODE_MIXED, false>, T, 0);
        if (e != hipSuccess || per_cu < 1) per_cu = 1;
        int64_t blocks = std::min<int64_t>((int64_t)cus * per_cu, (N + T - 1) / T);
        dim3 grid((unsigned)std::max<int64_t>(blocks, 1));
        if (mode == VOR_MODE_FP64) {
            if (segs) hipLaunchKernelGGL((k_trace_persistent<VOR_MODE_FP64, true>), grid, block, 0, st, A);
            else hipLaunchKernelGGL((k_trace_persistent<VOR_MODE_FP64, false>), grid, block, 0, st, A);
        } else {
            if (segs) hipLaunchKernelGGL((k_trace_persistent<VOR_MODE_MIXED, true>), grid, block, 0, st, A);
            else hipLaunchKernelGGL((k_trace_persistent<VOR_MODE_MIXED, false>), grid, block, 0, st, A);
        }
    } else {
        dim3 grid((unsigned)((N + T - 1) / T));
        if (mode == VOR_MODE_FP64) {
            if (segs) hipLaunchKernelGGL((k_trace<VOR_MODE_FP64, true>), grid, block, 0, st, A);
            else hipLaunchKernelGGL((k_trace<VOR_MODE_FP64, false>), grid, block, 0, st, A);
        } else {
            if (segs) hipLaunchKernelGGL((k_trace<VOR_MODE_MIXED, true>), grid, block, 0, st, A);
            else hipLaunchKernelGGL((k_trace<VOR_MODE_MIXED, false>), grid, block, 0, st, A);
        }
    }
    if (spill) {
        dim3 grid(1024);
        if (mode == VOR_MODE_FP64) hipLaunchKernelGGL((k_trace_spill<VOR_MODE_FP64>), grid, block, 0, st, A);
        else hipLaunchKernelGGL((k_trace_spill<VOR_MODE_MIXED>), grid, block, 0, st, A);
    }
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

extern "C" const char *vor_status_str(vor_status s)
{
    switch (s) {
    case VOR_OK: return "ok";
    case VOR_EINVAL: return "invalid argument";
    case VOR_EDUP: return "coincident sites";
    case VOR_EOUTSIDE: return "site outside the box or not finite";
    case VOR_ENOMEM: return "device allocation failed";
    case VOR_EDEVICE: return "HIP runtime or launch failure";
    case VOR_ECAPACITY: return "cell exceeds the builder's face capacity";
    case VOR_EBUDGET: return "request exceeds the memory budget";
    }
    return "unknown status";
}

extern "C" const char *vor_version(void) { return "voronoi_rt 0.1 (gfx950)"; }
