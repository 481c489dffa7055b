// trace.hip -- vor_locate and vor_trace: the cell-location function C(r)
// (Sect. 2.3) and the straight-path loop (Sect. 2.2, Eqs. 1-5), one ray per
// lane (the per-ray work is in trace_core.h).
//
// Mixed mode ranks the neighbours with FP32 offsets and a rounding-error
// bound per crossing; when the bounds of the best and any other candidate
// overlap the whole step is redone in FP64, otherwise only the winner's
// crossing is recomputed in FP64. Either way the emitted values are the FP64
// ones.
#include <mutex>

#include "trace_core.h"
#include "locate_core.h"

using namespace vrt;

const vrt::Grid &vrt_grid_of(const vor_grid *G);

namespace {

struct TraceArgs {
    GridRef G;
    LocView loc;          // the grid's block lists (loc.start null if it has none)
    RayIn I;
    SegOut O;
    int64_t N;
    double *tau;
    int32_t *n_seg;
    uint8_t *status;
    int32_t *n_fb;
    int64_t seg_stride;
    const int64_t *ray_off;
    const int32_t *order;
    unsigned long long *counters;
    int64_t *work;        // [1] spill chunks asked for, [2] rays past their window, [kHead0 ..] work queues
    int32_t *start;       // start cell (internal) of every ray from k_start_cells, or null: located at ray start
    Extras X;             // interaction points and tallies (kernels with EXT only)
};

#ifndef VRT_REFILL_MIN
#define VRT_REFILL_MIN 48
#endif
#ifndef VRT_DEFER_FINISH
#define VRT_DEFER_FINISH 1
#endif
#ifndef VRT_WAVES_PER_EU
#define VRT_WAVES_PER_EU 0
#endif
#if VRT_WAVES_PER_EU
#define VRT_OCC __attribute__((amdgpu_waves_per_eu(VRT_WAVES_PER_EU)))
#else
#define VRT_OCC
#endif
constexpr int kRefillMin = VRT_REFILL_MIN;   // idle lanes that trigger a refill in the persistent kernel
// Work queues of the persistent kernel: the processing order is cut into
// kParts contiguous parts, one per XCD (workgroups are dispatched to the
// XCDs in turn, so block b runs on XCD b mod kParts). The waves of an XCD
// take rays from their own part first, so the rays in flight on it are
// neighbours in the coherent order and share its L2; a wave whose part has
// run out moves on to the next part. Queue heads: work[kHead0 + p].
constexpr int kParts = 8;
constexpr int kHead0 = 8;
static_assert(kHead0 + kParts <= VOR_WORK_WORDS, "work queue heads must fit the control words");

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Output window of ray `ray`.
template <bool SEGS>
__device__ __forceinline__ void ray_window(const TraceArgs &A, int64_t ray, RayState &R)
{
    R.base = 0;
    R.cap = 0;
    R.chunk = -1;
    R.ray = (int32_t)ray;
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

// Results of a finished ray.
template <bool SEGS, bool EXT, int MODE>
__device__ __forceinline__ void ray_finish(const TraceArgs &A, int64_t ray, RayState &R, const RayStats &S)
{
    if (EXT) ray_extras_finish(A.X, ray, R);
    if (SEGS) finish_segments<cells_per_store<MODE, EXT>(), lens_per_store<MODE, EXT>()>(A.O, R, S.cnt);
    if (SEGS && S.cnt > R.cap) {
        if (A.work) atomicAdd((unsigned long long *)&A.work[2], 1ull);
        if (R.st == RAY_OK && (!A.O.spill_cell || R.chunk == -2)) R.st = RAY_OVERFLOW;
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

template <bool EXT, int MODE>
__device__ __forceinline__ void ray_start(const TraceArgs &A, int64_t ray, RayState &R)
{
    double s0;
    R.st = ray_setup<EXT>(A.G, A.I, ray, R.r0, R.k, R.L, s0);
    R.tau = 0.0;
    if (R.st == RAY_OK) {
        if (A.start) ray_begin_at<MODE>(A.G, R, A.start[ray], s0);
        else ray_begin<MODE>(A.G, R, s0);
    } else {
        R.L = 0.0;
        R.s_c = 0.0;
    }
    if (EXT) ray_extras_begin(A.X, ray, R);
    R.rho = (MODE != VOR_MODE_FP64 && A.I.grid_rho && R.st == RAY_OK) ? block_rho<MODE>(A.G, R.b) : 0.0;
    settle_start(R);
}

// The start cell C(r0) of every ray (Sect. 2.3), in processing order, ahead
// of the traversal: the ring searches of neighbouring lanes run side by side
// here instead of interrupting the persistent waves at every refill. A wave
// whose 64 rays share one origin (a point source, rays in coherent order)
// searches once, cooperatively.
__global__ void __launch_bounds__(256) k_start_cells(TraceArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < A.N;
    const int64_t ray = valid ? (A.order ? (int64_t)A.order[i] : i) : 0;
    double r0[3] = {0.0, 0.0, 0.0}, k[3] = {1.0, 0.0, 0.0}, L, s0 = 0.0;
    const uint8_t st = valid ? ray_setup(A.G, A.I, ray, r0, k, L, s0) : (uint8_t)RAY_BADDIR;
    double q[3];
    start_point(r0, k, s0, q);
    const int32_t m = start_cell(A.G.grid, A.loc, q, valid && st == RAY_OK);
    if (valid) A.start[ray] = m;
}

// One ray per lane.
template <int MODE, bool SEGS, bool EXT>
__global__ void __launch_bounds__(256) VRT_OCC k_trace(TraceArgs A)
{
    const int64_t lane_ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    RayStats S;
    if (lane_ray < A.N) {
        const int64_t ray = A.order ? (int64_t)A.order[lane_ray] : lane_ray;
        RayState R;
        ray_window<SEGS>(A, ray, R);
        ray_start<EXT, MODE>(A, ray, R);
        while (ray_step<MODE, SEGS, EXT>(A.G, A.I, R, S, A.O, A.X)) {
        }
        ray_finish<SEGS, EXT, MODE>(A, ray, R, S);
    }
    flush_counters(A, S);
}

// Tally deposits of the wave's lanes (at most one each, from their last
// step), added where the wave is converged: the lanes depositing into the
// same cell as the first pending lane sum their values across the wave and
// one of them updates the tallies -- a cell met by many rays at once, such
// as one next to a point source, then takes one atomic per wave instead of
// one per lane. Up to VRT_DEP_ROUNDS such groups are formed (while a group
// has two lanes or more); the other lanes update directly.
#ifndef VRT_DEP_ROUNDS
#define VRT_DEP_ROUNDS 4
#endif
__device__ __forceinline__ void flush_deposits(const Extras &X, RayState &R)
{
    bool direct = R.dep_uid >= 0;
    const int lane = threadIdx.x & 63;
    for (int round = 0; round < VRT_DEP_ROUNDS; ++round) {
        const uint64_t pend = __ballot(direct);
        if (pend == 0ull) break;
        const int leader = __ffsll((long long)pend) - 1;
        const int32_t luid = __shfl(R.dep_uid, leader, 64);
        const bool same = direct && R.dep_uid == luid;
        if (__popcll(__ballot(same)) < 2) break;
        double vl = same ? R.dep_len : 0.0, va = same ? R.dep_abs : 0.0;
        for (int off = 32; off > 0; off >>= 1) {
            vl += __shfl_xor(vl, off, 64);
            va += __shfl_xor(va, off, 64);
        }
        if (lane == leader) {
            if (X.tally_len) atomicAdd(&X.tally_len[luid], vl);
            if (X.tally_abs) atomicAdd(&X.tally_abs[luid], va);
        }
        direct = direct && !same;
    }
    if (direct) {
        if (X.tally_len) atomicAdd(&X.tally_len[R.dep_uid], R.dep_len);
        if (X.tally_abs) atomicAdd(&X.tally_abs[R.dep_uid], R.dep_abs);
    }
    R.dep_uid = -1;
}

// Persistent waves: every lane keeps a ray in flight. Lanes whose ray has
// ended wait until at least kRefillMin of the wave's lanes are idle (or
// none is busy); then they take the next rays from the work queue of their
// part of the processing order together (one atomic per wave, ranks from
// the ballot) and start them side by side. A wave that finds its current
// part exhausted moves to the next one; after finding all kParts parts
// exhausted (exhaustion is permanent) the queue is drained for it.
template <int MODE, bool SEGS, bool EXT>
__global__ void __launch_bounds__(256) VRT_OCC k_trace_persistent(TraceArgs A)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    RayStats S, T;   // S: current ray, T: totals of this lane
    RayState R;
    R.dep_uid = -1;   // no deferred deposit before the first ray
    int64_t ray = -1;
    bool live = false;
    unsigned long long *heads = (unsigned long long *)&A.work[kHead0];
    int part = (int)(blockIdx.x % kParts), exhausted = 0;   // wave-uniform: current part, parts found empty
    bool drained = false;   // wave-uniform: every part has run out
    bool pending = false;   // this lane's ray has ended and its results are not yet written
    unsigned int wit = 0, wref = 0;   // wave-uniform: iterations with a live lane, refills
    for (;;) {
        const bool need = !live;
        const uint64_t want = __ballot(need);
        const uint64_t busy = ~want & __ballot(true);
        if (want && !drained && (__popcll(want) >= kRefillMin || busy == 0ull)) {
            ++wref;
#if VRT_DEFER_FINISH
            if (pending) {   // the ended rays of the wave write their results together
                ray_finish<SEGS, EXT, MODE>(A, ray, R, S);
                pending = false;
            }
#endif
            int n = __popcll(want);
            int leader = __ffsll((long long)want) - 1;
            const int64_t p0 = A.N * part / kParts, p1 = A.N * (part + 1) / kParts;
            unsigned long long base0 = 0;
            if (lane == leader) base0 = atomicAdd(&heads[part], (unsigned long long)n);
            base0 = __shfl(base0, leader, 64);
            if (need) {
                const unsigned long long r = base0 + __popcll(want & lt);
                const int64_t q = r < (unsigned long long)(p1 - p0) ? p0 + (int64_t)r : A.N;
                if (q < p1) {
                    ray = A.order ? (int64_t)A.order[q] : q;
                    S = RayStats();
                    ray_window<SEGS>(A, ray, R);
                    ray_start<EXT, MODE>(A, ray, R);
                    live = true;
                } else {
                    ray = -1;
                }
            }
            if (__ballot(need && ray < 0) != 0ull) {   // this part has run out
                part = part + 1 == kParts ? 0 : part + 1;
                drained = ++exhausted == kParts;
            }
        }
        if (__ballot(live) == 0ull) {
            if (drained) break;   // the queue is drained and every ray has ended
            continue;
        }
        ++wit;
        const bool more = live && ray_step<MODE, SEGS, EXT, EXT>(A.G, A.I, R, S, A.O, A.X);
        if (EXT && (A.X.tally_len || A.X.tally_abs)) flush_deposits(A.X, R);
        if (live) {
            if (!more) {
#if VRT_DEFER_FINISH
                pending = true;
#else
                ray_finish<SEGS, EXT, MODE>(A, ray, R, S);
#endif
                T.cnt += S.cnt;
                T.nfb += S.nfb;
                T.nredo += S.nredo;
                T.steps += S.steps;
                T.recs += S.recs;
                live = false;
            }
        }
    }
#if VRT_DEFER_FINISH
    if (pending) ray_finish<SEGS, EXT, MODE>(A, ray, R, S);
#endif
    flush_counters(A, T);
    if (A.counters && (threadIdx.x & 63) == 0) {
        atomicAdd(&A.counters[5], (unsigned long long)wit);
        atomicAdd(&A.counters[6], (unsigned long long)wref);
    }
}

// Sort keys of a ray: Hilbert index of its origin (10 bits per axis over the
// box) and of its direction ((k/|k| + 1)/2 over the unit cube), and its
// chord -- the distance to the wall it heads for (Eq. 5 on every axis) --
// as a key of up to 8 bits that is smallest for the longest chords (0 for
// rays without one).
struct OrderBox {
    double lo[3], hi[3], scale[3], diag;
};

#ifndef VRT_ORDER_KEY_BITS
#define VRT_ORDER_KEY_BITS 30
#endif
#ifndef VRT_CHORD_KEY_BITS
#define VRT_CHORD_KEY_BITS 8
#endif
// Bits of the origin and direction keys of the coherent order (the leading
// bits of 30-bit Hilbert keys: coarser cells), and of the chord key, which
// only has to rank the rays into a few chord groups (by its histogram). Keys
// of 24 and 18 bits were measured: the sort saves a pass per key, the trace
// kernel loses about as much to coarser coherence.
constexpr int kOrderKeyBits = VRT_ORDER_KEY_BITS;
constexpr int kChordKeyBits = VRT_CHORD_KEY_BITS;
static_assert(kOrderKeyBits % 3 == 0 && kOrderKeyBits <= 30 && kChordKeyBits <= 8, "key widths");

// Block 0 also clears the chord-key counts (ccount, 256 entries) that
// k_chord_counts fills after it.
__global__ void k_ray_keys(const double *__restrict__ origins, const double *__restrict__ dirs, int64_t N,
                           OrderBox B, uint32_t *__restrict__ okey, uint32_t *__restrict__ dkey,
                           uint32_t *__restrict__ lkey, int32_t *__restrict__ idx, int32_t *__restrict__ ccount)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ccount && blockIdx.x == 0 && threadIdx.x < 256) ccount[threadIdx.x] = 0;
    if (i >= N) return;
    uint32_t qo[3], qd[3];
    double k[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    if (!(kn > 0.0) || !isfinite(kn)) kn = 1.0;
    double L = 1e308 * 10.0;
    for (int a = 0; a < 3; ++a) {
        const double r = origins[3 * i + a];
        const double ka = k[a] / kn;
        double f = (r - B.lo[a]) * B.scale[a];
        double g = (ka + 1.0) * 512.0;
        qo[a] = (uint32_t)(f > 0.0 ? (f < 1023.0 ? f : 1023.0) : 0.0);
        qd[a] = (uint32_t)(g > 0.0 ? (g < 1023.0 ? g : 1023.0) : 0.0);
        if (ka > 0.0) L = fmin(L, (B.hi[a] - r) / ka);
        else if (ka < 0.0) L = fmin(L, (B.lo[a] - r) / ka);
    }
    const double frac = (L > 0.0 && L < 1e300) ? fmin(L / B.diag, 1.0) : 0.0;   // NaN origins give 0
    okey[i] = hilbert_key(qo[0], qo[1], qo[2]) >> (30 - kOrderKeyBits);
    dkey[i] = hilbert_key(qd[0], qd[1], qd[2]) >> (30 - kOrderKeyBits);
    lkey[i] = (uint32_t)((1.0 - frac) * (double)((1 << kChordKeyBits) - 1) + 0.5);
    idx[i] = (int32_t)i;
}

// How many rays have each chord key (an LDS histogram per block, then one
// atomic per block and key).
__global__ void __launch_bounds__(256) k_chord_counts(const uint32_t *__restrict__ ckey, int64_t N,
                                                      int32_t *__restrict__ ccount)
{
    __shared__ int32_t c[256];
    c[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&c[ckey[i] & 255u], 1);
    __syncthreads();
    if (c[threadIdx.x]) atomicAdd(&ccount[threadIdx.x], c[threadIdx.x]);
}

// The final sort key of the ray at rank r of the coherent order: its part
// of the order (the contiguous part a persistent launch gives one XCD),
// then its chord bin. The bin is the ray's rank in chord order (longest
// first) scaled to `bins`, every ray of one chord key taking the rank at the
// middle of its key's run: ((rays of smaller keys) + (rays of its key) / 2)
// * bins / N. Each block derives the 256 bins from the key counts.
__global__ void __launch_bounds__(256) k_part_bin_key(const int32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ ckey,
                                                      const int32_t *__restrict__ ccount, int64_t N, int parts,
                                                      int bins, uint32_t *__restrict__ key)
{
    __shared__ uint32_t bin_of[256];
    const int t = threadIdx.x, lane = t & 63;
    if (t < 64) {   // one wave scans the 256 counts, 4 per lane
        int64_t c[4], v = 0;
        for (int j = 0; j < 4; ++j) {
            c[j] = ccount[4 * lane + j];
            v += c[j];
        }
        int64_t incl = v;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int64_t u = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += u;
        }
        int64_t before = incl - v;
        for (int j = 0; j < 4; ++j) {
            bin_of[4 * lane + j] = (uint32_t)(((before + c[j] / 2) * bins) / N);
            before += c[j];
        }
    }
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + t;
    if (r < N) key[r] = (uint32_t)((r * parts) / N) * (uint32_t)bins + bin_of[ckey[order[r]] & 255u];
}

__global__ void k_iota(int32_t *__restrict__ idx, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) idx[i] = (int32_t)i;
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

__global__ void __launch_bounds__(256) k_locate_blocks(LocView L, const double *__restrict__ pts, int64_t N,
                                                       int32_t *__restrict__ cell)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double q[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    if (!(q[0] >= L.lo[0] && q[0] <= L.hi[0] && q[1] >= L.lo[1] && q[1] <= L.hi[1] && q[2] >= L.lo[2] &&
          q[2] <= L.hi[2])) {
        cell[i] = -1;
        return;
    }
    int32_t uid;
    nearest_in_blocks(L, q, &uid);
    cell[i] = uid;
}

}  // namespace

extern "C" vor_status vor_locate_blocks(const vor_grid *G, const double *pts, int64_t N, int32_t *cell,
                                        void *stream)
{
    if (!G || N < 0 || (N > 0 && (!pts || !cell))) return VOR_EINVAL;
    const Grid &g = vrt_grid_of(G);
    if (!g.loc_start) return VOR_EINVAL;
    if (N == 0) return VOR_OK;
    const int T = 256;
    const int64_t blocks = (N + T - 1) / T;
    if (blocks > 0x7fffffff) return VOR_EINVAL;
    const LocView L = loc_view(g);
    hipLaunchKernelGGL(k_locate_blocks, dim3((unsigned)blocks), dim3(T), 0, (hipStream_t)stream, L, pts, N, cell);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

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

// Resident blocks per compute unit of a persistent trace kernel (a property
// of the compiled kernel: queried once per process).
template <int MODE, bool SEGS, bool EXT>
int persistent_blocks_per_cu()
{
    static const int per_cu = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_trace_persistent<MODE, SEGS, EXT>, 256, 0) !=
                hipSuccess ||
            n < 1)
            n = 1;
        return n;
    }();
    return per_cu;
}

// Launch of the trace kernel: one ray per lane, or persistent waves (as
// many blocks as fit on the device at once; cus = the grid's device's
// compute units, read when the grid was built).
template <int MODE, bool SEGS, bool EXT>
vor_status launch_trace_ext(const TraceArgs &A, bool persistent, int cus, hipStream_t st)
{
    const int T = 256;
    if (persistent) {
        const int per_cu = persistent_blocks_per_cu<MODE, SEGS, EXT>();
        const int64_t blocks = std::min<int64_t>((int64_t)cus * per_cu, (A.N + T - 1) / T);
        hipLaunchKernelGGL((k_trace_persistent<MODE, SEGS, EXT>), dim3((unsigned)std::max<int64_t>(blocks, 1)),
                           dim3(T), 0, st, A);
    } else {
        hipLaunchKernelGGL((k_trace<MODE, SEGS, EXT>), dim3((unsigned)((A.N + T - 1) / T)), dim3(T), 0, st, A);
    }
    return VOR_OK;
}

template <int MODE, bool SEGS>
vor_status launch_trace(const TraceArgs &A, bool ext, bool persistent, int cus, hipStream_t st)
{
    return ext ? launch_trace_ext<MODE, SEGS, true>(A, persistent, cus, st)
               : launch_trace_ext<MODE, SEGS, false>(A, persistent, cus, st);
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
    if (spill && (!segs || out->seg_stride <= 0 || !out->spill_len || !out->spill_first || !out->spill_next ||
                  !out->work || out->spill_chunks < 0 || out->spill_chunks > 0x7fffffffLL))
        return VOR_EINVAL;
    int mode = opts ? opts->mode : VOR_MODE_FP64;
    if (mode != VOR_MODE_FP64 && mode != VOR_MODE_MIXED) return VOR_EINVAL;
    if (opts && (opts->max_steps < 0 || !(opts->eps_mix == 0.0 || (opts->eps_mix >= kEpsMixMin && opts->eps_mix <= 0.25))))
        return VOR_EINVAL;
    if (opts && !(opts->eps_fb >= 0.0 && opts->eps_fb < 1e300)) return VOR_EINVAL;   // NaN, negative or infinite
    const bool persistent = opts && opts->persistent;
    if (persistent && !out->work) return VOR_EINVAL;
    if (opts && opts->start_given && !out->start_cell) return VOR_EINVAL;
    if (!out->tau_stop != !out->stop_cell) return VOR_EINVAL;   // interaction points: input and cell output together
    if (out->stop_s && !out->tau_stop) return VOR_EINVAL;
    if (out->weight && !out->tally_len && !out->tally_abs) return VOR_EINVAL;
    const Grid &g = vrt_grid_of(G);
    if (mode == VOR_MODE_MIXED && !mixed_mode_fits(g)) return VOR_EINVAL;
    if (opts && opts->grid_density && (density || !g.rho_bound)) return VOR_EINVAL;
    TraceArgs A;
    A.G = grid_ref(g, opts ? opts->max_steps : 0, opts ? opts->eps_mix : 0.0);
    if (opts && opts->eps_fb > 0.0) A.G.eps_fb = opts->eps_fb;
    A.loc = loc_view(g);
    A.I.origins = origins;
    A.I.dirs = dirs;
    A.I.density = density;
    A.I.kappa = kappa;
    A.I.enter = opts ? opts->enter : 0;
    A.I.grid_rho = (opts && opts->grid_density) ? 1 : 0;
    A.N = N;
    A.tau = out->tau;
    A.n_seg = out->n_seg;
    A.status = out->status;
    A.n_fb = out->n_fallback;
    A.seg_stride = out->seg_stride;
    A.ray_off = out->ray_off;
    A.order = out->ray_order;
    A.counters = out->counters;
    A.work = out->work;
    A.O.cell = out->seg_cell;
    A.O.len = out->seg_len;
    A.O.vec = out->seg_stride <= 0 ? 0 : out->seg_stride % 16 == 0 ? 2 : out->seg_stride % 8 == 0 ? 1 : 0;
    A.O.spill_cell = spill ? out->spill_cell : nullptr;
    A.O.spill_len = out->spill_len;
    A.O.spill_next = out->spill_next;
    A.O.spill_first = out->spill_first;
    A.O.spill_chunks = out->spill_chunks;
    A.O.chunk_head = out->work ? (unsigned long long *)&out->work[1] : nullptr;
    A.start = out->start_cell;
    A.X.tau_stop = out->tau_stop;
    A.X.weight = out->weight;
    A.X.tally_len = out->tally_len;
    A.X.tally_abs = out->tally_abs;
    A.X.stop_cell = out->stop_cell;
    A.X.stop_s = out->stop_s;
    hipStream_t st = (hipStream_t)stream;
    const int T = 256;
    if (A.work) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, st, A.work, VOR_WORK_WORDS);
    if (A.start && !(opts && opts->start_given))
        hipLaunchKernelGGL(k_start_cells, dim3((unsigned)((N + T - 1) / T)), dim3(T), 0, st, A);
    if (spill) {
        int64_t nb = std::min<int64_t>((N + T - 1) / T, 65535);
        hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)nb), dim3(T), 0, st, A.O.spill_first, N, (int64_t)-1);
    }
    const bool ext = A.X.tau_stop || A.X.tally_len || A.X.tally_abs || A.I.enter;   // kernels with the optional features
    const vor_status rc = mode == VOR_MODE_FP64
                              ? (segs ? launch_trace<VOR_MODE_FP64, true>(A, ext, persistent, g.cus, st)
                                      : launch_trace<VOR_MODE_FP64, false>(A, ext, persistent, g.cus, st))
                          : g.compact ? (segs ? launch_trace<kModeCompact, true>(A, ext, persistent, g.cus, st)
                                              : launch_trace<kModeCompact, false>(A, ext, persistent, g.cus, st))
                              : (segs ? launch_trace<VOR_MODE_MIXED, true>(A, ext, persistent, g.cus, st)
                                      : launch_trace<VOR_MODE_MIXED, false>(A, ext, persistent, g.cus, st));
    if (rc != VOR_OK) return rc;
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

// ---------------------------------------------------------------------------
// vor_trace_noalloc: vor_trace with its scratch (the control words of the
// work queues and spill, then the start cells of up to VOR_NOALLOC_MAX_RAYS
// rays) in a fixed array of the library instead of caller buffers. Each GPU
// holds its own copy of the array; host code reaches it only through the
// device address hipGetSymbolAddress returns for that GPU, taken once per
// device on its first call there (the array's name in host code is a
// host-side stand-in, not that address).
constexpr int64_t kNoAllocWords = VOR_WORK_WORDS + (VOR_NOALLOC_MAX_RAYS + 1) / 2;
static __device__ __align__(256) int64_t scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (the current device).
vor_status device_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VOR_EDEVICE;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VOR_EDEVICE;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return VOR_OK;
}
}  // namespace

extern "C" vor_status vor_trace_noalloc(const vor_grid *G, const double *origins, const double *dirs, int64_t N,
                                        const double *density, double kappa, const vor_trace_opts *opts,
                                        const vor_trace_out *out, void *stream)
{
    if (!G || !out || N < 0) return VOR_EINVAL;
    if (out->work || out->start_cell || (opts && opts->start_given)) return VOR_EINVAL;   // the library's own scratch
    if (N > VOR_NOALLOC_MAX_RAYS) return VOR_ECAPACITY;
    if (N == 0) return VOR_OK;
    void *sp = nullptr;
    const vor_status rc = device_scratch(&sp);
    if (rc != VOR_OK) return rc;
    vor_trace_out o = *out;
    o.work = reinterpret_cast<int64_t *>(sp);                        // zeroed by vor_trace's first kernel
    o.start_cell = reinterpret_cast<int32_t *>(o.work + VOR_WORK_WORDS);   // written by its start pass
    return vor_trace(G, origins, dirs, N, density, kappa, opts, &o, stream);
}

// The processing order: the coherent order (origin, then direction) cut
// into the kParts contiguous parts that a persistent launch hands to its
// XCDs; inside each part the rays fall in kChordBins groups by chord length
// (ranked over the whole batch), the longest first, each group in coherent
// order. Long paths then start early and the end of a part is left to short
// ones, which shortens the drain where only a few lanes of a wave still
// work; the parts keep their spatial coherence.
constexpr int kChordBins = 8;
// Batches below 2^22 rays (a few rays per lane of a full launch, so the
// drain weighs more) use 16 groups.
constexpr int kChordBinsSmall = 16;
constexpr int64_t kChordBinsSmallMaxRays = 1 << 22;
#ifndef VRT_ORDER_MIN_RAYS
#define VRT_ORDER_MIN_RAYS (1 << 14)
#endif
// Below this many rays a batch keeps its own order: the sort's launches
// would cost more than coherence can save in so short a trace.
constexpr int64_t kOrderMinRays = VRT_ORDER_MIN_RAYS;
// Below this many rays a launch is too short for a drain to matter (and is
// launch-bound): the order is the coherent one alone.
constexpr int64_t kChordBinsMinRays = 1 << 17;

extern "C" int64_t vor_order_workspace_bytes(int64_t N)
{
    if (N < 0) return -1;
    int64_t hl = vrt_radix_hist_len(N);
    return 6 * N * (int64_t)sizeof(uint32_t) + (hl + 512) * (int64_t)sizeof(int32_t) + 1024;
}

extern "C" vor_status vor_order_rays(const vor_grid *G, const double *origins, const double *dirs, int64_t N,
                                     int32_t *order, void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!G || N < 0 || (N > 0 && (!origins || !dirs || !order || !workspace))) return VOR_EINVAL;
    if (N == 0) return VOR_OK;
    if (N > 0x7fffffffLL || workspace_bytes < vor_order_workspace_bytes(N)) return VOR_EINVAL;
    const Grid &g = vrt_grid_of(G);
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    uint32_t *okey = (uint32_t *)w;
    uint32_t *dkey = okey + N;
    uint32_t *ktmp = dkey + N;
    int32_t *vtmp = (int32_t *)(ktmp + N);
    uint32_t *lkey = (uint32_t *)(vtmp + N);
    uint32_t *bins = lkey + N;
    int32_t *hist = (int32_t *)(bins + N);
    const int64_t hl = vrt_radix_hist_len(N);
    OrderBox B;
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        B.lo[a] = g.box[a];
        B.hi[a] = g.box[a + 3];
        B.scale[a] = 1024.0 / (g.box[a + 3] - g.box[a]);
        d2 += (g.box[a + 3] - g.box[a]) * (g.box[a + 3] - g.box[a]);
    }
    B.diag = sqrt(d2);
    const int T = 256;
    const unsigned nb = (unsigned)((N + T - 1) / T);
    if (N < kOrderMinRays) {
        hipLaunchKernelGGL(k_iota, dim3(nb), dim3(T), 0, st, order, N);
        return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
    }
    const bool chords = N >= kChordBinsMinRays;
    int32_t *ccount = chords ? hist + hl + 256 : nullptr;   // past the sort's histogram and digit totals
    // chord keys go to `bins` (the final keys are written to lkey while they are read)
    hipLaunchKernelGGL(k_ray_keys, dim3(nb), dim3(T), 0, st, origins, dirs, N, B, okey, dkey, bins, order, ccount);
    vor_status rc = VOR_OK;
    if (chords)   // chord bins: how many rays have each chord key
        hipLaunchKernelGGL(k_chord_counts, dim3(256), dim3(T), 0, st, bins, N, ccount);
    // by direction, then stably by origin: rays from one place in similar directions end up together
    rc = vrt_radix_sort_pairs(dkey, order, ktmp, vtmp, N, kOrderKeyBits, hist, hl, st);
    if (rc != VOR_OK) return rc;
    // the origin keys must follow the same permutation before the second sort
    rc = vrt_gather_u32(okey, order, N, ktmp, st);
    if (rc != VOR_OK) return rc;
    rc = vrt_radix_sort_pairs(ktmp, order, okey, vtmp, N, kOrderKeyBits, hist, hl, st);
    if (rc != VOR_OK) return rc;
    // then stably by (part of the order, chord bin)
    static_assert(kParts * kChordBinsSmall <= 256, "one 8-bit pass sorts by part and bin");
    const int bins_n = N < kChordBinsSmallMaxRays ? kChordBinsSmall : kChordBins;
    if (chords) {
        hipLaunchKernelGGL(k_part_bin_key, dim3(nb), dim3(T), 0, st, order, bins, ccount, N, kParts, bins_n,
                           lkey);
        rc = vrt_radix_sort_pairs(lkey, order, ktmp, vtmp, N, 8, hist, hl, st);
        if (rc != VOR_OK) return rc;
    }
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

// Whole paths as compact rows (Sect. 2.2: a path is every cell to the
// wall), one wave per ray: its window's first min(n_seg, stride) slots,
// then its chain of spill chunks (one chunk = one wave-wide copy), go to
// [ray_off[i], ray_off[i] + n_seg[i]). Reads and writes of a row are
// contiguous across the wave's lanes. A chain that ends early (a ray whose
// spill ran out) leaves the rest of its row unwritten.
__global__ void __launch_bounds__(256) k_gather_paths(const int32_t *__restrict__ n_seg, int64_t n,
                                                      const int32_t *__restrict__ wcell,
                                                      const double *__restrict__ wlen, int64_t stride,
                                                      const int64_t *__restrict__ first,
                                                      const int32_t *__restrict__ next,
                                                      const int32_t *__restrict__ pcell,
                                                      const double *__restrict__ plen,
                                                      const int64_t *__restrict__ ray_off, int32_t *__restrict__ cell,
                                                      double *__restrict__ len)
{
    static_assert(kSpillChunk == 64, "a spill chunk is one wave-wide copy");
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const int64_t cnt = n_seg[i];
    const int64_t o = ray_off[i];
    const int64_t w = cnt < stride ? cnt : stride;
    for (int64_t j = lane; j < w; j += 64) {
        cell[o + j] = wcell[i * stride + j];
        len[o + j] = wlen[i * stride + j];
    }
    int64_t c = (cnt > stride && first) ? first[i] : -1;
    for (int64_t j = w; j < cnt && c >= 0; j += kSpillChunk) {
        if (lane < cnt - j) {
            cell[o + j + lane] = pcell[c * kSpillChunk + lane];
            len[o + j + lane] = plen[c * kSpillChunk + lane];
        }
        c = next[c];
    }
}

vor_status vrt_gather_paths(const int32_t *n_seg, int64_t n, const int32_t *wcell, const double *wlen, int64_t stride,
                            const int64_t *first, const int32_t *next, const int32_t *pcell, const double *plen,
                            const int64_t *ray_off, int32_t *cell, double *len, hipStream_t st)
{
    if (n == 0) return VOR_OK;
    const int64_t blocks = (n + 3) / 4;
    if (blocks > 0x7fffffffLL) return VOR_EINVAL;
    hipLaunchKernelGGL(k_gather_paths, dim3((unsigned)blocks), dim3(256), 0, st, n_seg, n, wcell, wlen, stride, first,
                       next, pcell, plen, ray_off, cell, len);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

extern "C" vor_status vor_gather_paths(const int32_t *n_seg, int64_t N, const int32_t *win_cell, const double *win_len,
                                       int64_t seg_stride, const int64_t *spill_first, const int32_t *spill_next,
                                       const int32_t *spill_cell, const double *spill_len, const int64_t *ray_off,
                                       int32_t *seg_cell, double *seg_len, void *stream)
{
    const bool any_spill = spill_first || spill_next || spill_cell || spill_len;
    const bool all_spill = spill_first && spill_next && spill_cell && spill_len;
    if (N < 0 || seg_stride <= 0 || (any_spill && !all_spill)) return VOR_EINVAL;
    if (N > 0 && (!n_seg || !win_cell || !win_len || !ray_off || !seg_cell || !seg_len)) return VOR_EINVAL;
    return vrt_gather_paths(n_seg, N, win_cell, win_len, seg_stride, spill_first, spill_next, spill_cell, spill_len,
                            ray_off, seg_cell, seg_len, (hipStream_t)stream);
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
    case VOR_ECAPACITY: return "capacity exceeded (a cell's faces, the neighbour tables, or vor_trace_noalloc's rays)";
    case VOR_EBUDGET: return "request exceeds the memory budget";
    case VOR_ETIMEOUT: return "timed out";
    }
    return "unknown status";
}

extern "C" const char *vor_version(void) { return "voronoi_rt 0.1 (gfx950)"; }

#if VRT_DIAG
// Diagnostic build only: read and clear the batch counters.
extern "C" int vor_diag_take(unsigned long long *out)
{
    unsigned long long z[4] = {0, 0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyFromSymbol(out, HIP_SYMBOL(vrt_diag), sizeof(z)) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(vrt_diag), z, sizeof(z)) != hipSuccess)
        return 1;
    return 0;
}
#endif
