// serve.hip -- continuous-batching path service: several grids resident in
// HBM, requests of uneven size admitted against a memory budget, and their
// rays traced together by persistent waves that refill lanes from a device
// work queue.
//
// Host side: one scheduler thread per server. Requests wait in a FIFO until
// their output buffers fit in the budget arena (first fit). Whenever one of
// the server's streams is free, every admitted request not yet launched goes
// into one launch: its rays are cut into chunks (sized so that the launch has
// a few chunks per wave), the request table and chunk list are copied to the
// device and a persistent kernel drains them. Launches on different streams
// overlap: the blocks of a later launch start as those of an earlier one
// retire. A request is complete as soon as its last chunk is: the kernel
// publishes that to a flag in host memory, which the scheduler polls, so a
// small request does not wait for the large ones launched with it, and its
// memory returns to the budget at once.
//
// Device side: each wave works in one context (grid and precision class,
// uniform across the wave) and keeps its lanes busy with rays of the chunks
// it takes from the queue; lanes of one wave may hold rays of different
// requests of the same context. A wave that takes a chunk of another context
// lets its running rays finish before starting it. The per-ray work is the
// same code as vor_trace, so a ray's result does not depend on what else is
// in the launch.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "locate_core.h"
#include "trace_core.h"

using namespace vrt;

const vrt::Grid &vrt_grid_of(const vor_grid *G);

namespace {

constexpr int kMaxLaunchReqs = 1024;   // requests per launch
constexpr int kMaxLaunchChunks = 16384;
constexpr int kChunkMin = 64;          // rays per chunk, at least ...
constexpr int kChunkMax = 4096;        // ... and at most
constexpr int kChunksPerWave = 4;      // target chunks per wave of a launch
constexpr int kStreams = 3;
constexpr int kSlots = 64;             // chunks a wave may have open at once: one per lane, so a refill never waits
constexpr int kServeRefillMin = 48;    // idle lanes that trigger a refill

struct ReqDev {
    RayIn in;
    double *tau;
    int32_t *n_seg;
    uint8_t *status;
    int32_t *seg_cell;
    double *seg_len;
    int64_t seg_stride;
    SpillPool spill;      // the request's spill chunks (seg_stride > 0): paths longer than the window continue there
    int32_t *remaining;   // chunks of the request not yet complete (device memory)
    int32_t *overflow;    // rays whose spill chunks ran out (device memory)
    int32_t *done;        // completion flag (host memory, device address): 1 complete, 2 rerun with exact spill
};

// Per-request counters of a launch, zeroed when it starts.
struct ReqCount {
    unsigned long long spill_head;   // spill chunks handed out
    int32_t overflow;
    int32_t pad;
};

struct ChunkDev {
    int32_t req;    // index into the launch's request table
    int32_t first;  // first ray of the request in this chunk
    int32_t count;  // rays in the chunk (>= 1)
    int32_t ctx;    // 4 * grid + 2 * (densities bound to the grid) + (mode == mixed)
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Every ray of chunk slot's request chunk has been written by this wave:
// make the writes visible device-wide (a release fence: the wave's L2
// writes back, nothing is invalidated), count the chunk off its request,
// and the wave that completes the request's last chunk -- after an acquire
// fence, once per request -- raises its flag in host memory (release at
// system scope, so the flag is seen after the data): 1 when every path is
// whole, 2 when some ray found its request's spill chunks used up (the host
// then runs the request again with exactly the chunks its counts need). The
// overflow counts of other waves precede their release fences and chunk
// counts, which the acquire fence after the last count takes in. (A full
// fence or an acquire-release count here invalidated the L2 of the wave's
// XCD at every chunk.)
__device__ __forceinline__ void chunk_complete(const ReqDev *__restrict__ reqs, int q)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0) {
        const int prev = __hip_atomic_fetch_add(reqs[q].remaining, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int ovf = __hip_atomic_load(reqs[q].overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(reqs[q].done, ovf ? 2 : 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

#ifndef VRT_SERVE_WIDE
#define VRT_SERVE_WIDE VRT_LDS_STAGE
#endif
// Store groups of the serving kernels (see cells_per_store): the mixed
// kernels write 16 cells and 8 lengths at a time, held in LDS, or with
// VRT_SERVE_WIDE = 0 8 cells and 4 lengths held in registers.
constexpr bool kServeWide = VRT_SERVE_WIDE != 0;

// The serving kernel of one precision class (MODE): a launch runs the
// kernel of each class over the chunks of that class, so each holds the
// registers of one step only.
template <int MODE>
__global__ void __launch_bounds__(256) k_serve(const GridRef *__restrict__ grids, const LocView *__restrict__ locs,
                                               const ReqDev *__restrict__ reqs,
                                               const ChunkDev *__restrict__ chunks, int n_chunks,
                                               unsigned int *__restrict__ head,
                                               unsigned long long *__restrict__ counters)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    // Wave-uniform state.
    int ctx = -1;                     // context of the rays in flight
    GridRef G{};
    int cur_req = -1, cur_first = 0, cur_left = 0, cur_slot = 0;   // chunk being handed out
    int p_req = -1, p_first = 0, p_count = 0, p_ctx = -1;         // chunk taken, not yet started
    bool have_p = false, drained = false;
    // Open chunks of each wave of the block, in LDS: request, rays not yet
    // finished (0: the slot is free). Lane s owns slot s when searching.
    __shared__ int32_t s_req[4][kSlots], s_left[4][kSlots];
    int32_t *slot_req = s_req[threadIdx.x >> 6];
    int32_t *slot_left = s_left[threadIdx.x >> 6];
    slot_req[lane] = -1;
    slot_left[lane] = 0;
    __builtin_amdgcn_wave_barrier();   // the wave's lanes exchange slot data through LDS: keep its accesses in order
    // Per-lane state.
    bool live = false;
    bool pending = false;   // the lane's ray has ended; its results are written at the next refill
    int slot = -1, q = -1;
    int64_t ray = 0;
    const double *dens = nullptr;
    double kappa = 0.0;
    int32_t *cellp = nullptr;
    double *lenp = nullptr;
    int vec = 0;
    RayState R;
    RayStats S, T;
    for (;;) {
        const bool need = !live;
        const uint64_t want = __ballot(need);
        uint64_t busy = ~want & __ballot(true);
        if (want && (__popcll(want) >= kServeRefillMin || busy == 0ull)) {
            // The rays that ended since the last refill write their results together (one pass for the
            // wave instead of one per ray) and are counted off their chunks.
            if (__ballot(pending)) {
                if (pending) {
                    SegOut O{};
                    O.cell = cellp;
                    O.len = lenp;
                    O.vec = vec;
                    O.pool = &reqs[q].spill;
                    finish_segments<cells_per_store<MODE, false, kServeWide>(), lens_per_store<MODE, false, kServeWide>(),
                                    true>(O, R, S.cnt);
                    const ReqDev &rq = reqs[q];
                    if (R.cap > 0 && R.st == RAY_OK && S.cnt > R.cap && R.chunk == -2) {   // its spill chunks ran out
                        R.st = RAY_OVERFLOW;
                        atomicAdd(rq.overflow, 1);
                    }
                    rq.tau[ray] = R.tau;
                    rq.n_seg[ray] = S.cnt;
                    rq.status[ray] = R.st;
                }
                // count the ended rays off their chunks, one chunk at a time
                for (uint64_t left = __ballot(pending); left; left = __ballot(pending)) {
                    const int leader = __ffsll((long long)left) - 1;
                    const int s = uniform(__shfl(slot, leader, 64));
                    const uint64_t grp = __ballot(pending && slot == s);
                    int rest = 0;
                    if (lane == leader) {
                        rest = slot_left[s] - __popcll(grp);
                        slot_left[s] = rest;
                    }
                    __builtin_amdgcn_wave_barrier();
                    rest = uniform(__shfl(rest, leader, 64));
                    if (rest == 0) chunk_complete(reqs, uniform(slot_req[s]));
                    pending = pending && slot != s;
                }
            }
            uint64_t pend = want;
            // Each pass starts a chunk or hands out rays; eight passes serve
            // every idle lane but in the rarest cases (the rest wait).
            for (int pass = 0; pass < 8 && pend; ++pass) {
                if (cur_left == 0) {
                    if (!have_p) {
                        if (drained) break;
                        unsigned int c = 0;
                        if (lane == 0) c = atomicAdd(head, 1u);
                        const int cu = uniform((int)c);
                        if (cu >= n_chunks) {
                            drained = true;
                            break;
                        }
                        const ChunkDev ch = chunks[cu];
                        p_req = uniform(ch.req);
                        p_first = uniform(ch.first);
                        p_count = uniform(ch.count);
                        p_ctx = uniform(ch.ctx);
                        have_p = true;
                    }
                    if (p_ctx != ctx && busy != 0ull) break;   // let the other context's rays finish first
                    const uint64_t free = __ballot(slot_left[lane] == 0);
                    if (free == 0ull) break;                    // every slot open (cannot happen with a slot per lane)
                    const int fs = __ffsll((long long)free) - 1;
                    if (lane == fs) {
                        slot_req[fs] = p_req;
                        slot_left[fs] = p_count;
                    }
                    __builtin_amdgcn_wave_barrier();
                    cur_req = p_req;
                    cur_first = p_first;
                    cur_left = p_count;
                    cur_slot = fs;
                    if (p_ctx != ctx) {
                        ctx = p_ctx;
                        G = grids[ctx >> 2];
                    }
                    have_p = false;
                }
                const int take = min(__popcll(pend), cur_left);
                const int rank = __popcll(pend & lt);
                const bool mine = ((pend >> lane) & 1ull) && rank < take;
                double s0 = 0.0;
                if (mine) {
                    const ReqDev &rq = reqs[cur_req];
                    q = cur_req;
                    slot = cur_slot;
                    ray = cur_first + rank;
                    dens = rq.in.density;
                    kappa = rq.in.kappa;
                    cellp = rq.seg_cell;
                    lenp = rq.seg_len;
                    vec = !rq.seg_cell ? 0 : rq.seg_stride % 16 == 0 ? 2 : rq.seg_stride % 8 == 0 ? 1 : 0;
                    if (rq.spill.first) rq.spill.first[ray] = -1;   // no chunk yet (taking one overwrites it)
                    S = RayStats();
                    R.st = ray_setup<false>(G, rq.in, ray, R.r0, R.k, R.L, s0);
                    R.tau = 0.0;
                    R.chunk = rq.seg_cell ? -1 : -2;   // tau only: no spill chunk is ever taken
                    R.ray = (int32_t)ray;
                    R.base = ray * rq.seg_stride;
                    R.cap = rq.seg_cell ? rq.seg_stride : 0;
                }
                // the start cells C(r0) (Sect. 2.3) of the rays just handed out, side by side
                // (every lane takes part: one cooperative search when all 64 share a point)
                {
                    double qp[3] = {0.0, 0.0, 0.0};
                    if (mine) start_point(R.r0, R.k, s0, qp);
                    const bool ok = mine && R.st == RAY_OK;
                    const int32_t m0 = start_cell<false>(G.grid, locs[ctx >> 2], qp, ok);   // (registers: no early stop)
                    if (mine) {
                        if (ok) {
                            ray_begin_at<MODE>(G, R, m0, s0);
                            R.rho = (MODE != VOR_MODE_FP64 && (ctx & 2)) ? block_rho<MODE>(G, R.b) : 0.0;   // mixed mode carries it
                            settle(R.rho);
                        } else {
                            R.L = 0.0;
                        }
                        live = true;
                    }
                }
                const uint64_t taken = __ballot(mine);
                pend &= ~taken;
                busy |= taken;
                cur_first += take;
                cur_left -= take;
            }
        }
        if (__ballot(live) == 0ull) {
            if (drained && !have_p && cur_left == 0) break;   // queue drained, every ray ended
            continue;
        }
        if (live) {
            const RayIn I{nullptr, nullptr, dens, kappa, 0, (ctx >> 1) & 1};
            SegOut O{};
            O.cell = cellp;
            O.len = lenp;
            O.vec = vec;
            O.pool = &reqs[q].spill;
            const bool more = ray_step<MODE, true, false, false, kServeWide, true>(G, I, R, S, O);
            if (!more) {
                T.cnt += S.cnt;
                T.nfb += S.nfb;
                T.nredo += S.nredo;
                live = false;
                pending = true;
            }
        }
    }
    const unsigned long long a = wave_sum_u64((unsigned long long)T.cnt);
    const unsigned long long b = wave_sum_u64((unsigned long long)T.nfb);
    const unsigned long long d = wave_sum_u64((unsigned long long)T.nredo);
    if (lane == 0) {
        atomicAdd(&counters[0], a);
        if (b) atomicAdd(&counters[1], b);
        if (d) atomicAdd(&counters[2], d);
    }
}

__global__ void k_zero_launch(unsigned int *head, unsigned long long *counters, ReqCount *rc, int n_req)
{
    if (threadIdx.x < 3) head[threadIdx.x] = 0;
    if (threadIdx.x < 4) counters[threadIdx.x] = 0;
    for (int q = threadIdx.x; q < n_req; q += blockDim.x) rc[q] = ReqCount{0ull, 0, 0};
}

using clk = std::chrono::steady_clock;

enum ReqState { Q_WAIT = 0, Q_ADMITTED, Q_RUNNING, Q_DONE, Q_RELEASED };

struct Request {
    int64_t id = 0;
    int grid = 0;
    int mode = 0;
    int64_t n = 0;
    RayIn in{};
    int64_t seg_stride = 0;
    int64_t spill_chunks = 0;
    size_t bytes = 0;
    size_t off = 0;   // arena offset
    ReqState state = Q_WAIT;
    vor_status err = VOR_OK;
    int runs = 0;     // launches that traced the request (2 when its spill chunks were sized again)
    clk::time_point t_submit, t_admit, t_done;
    // device outputs (in the arena)
    double *tau = nullptr;
    int32_t *n_seg = nullptr;
    uint8_t *status = nullptr;
    int32_t *seg_cell = nullptr;
    double *seg_len = nullptr;
    int64_t *spill_first = nullptr;
    int32_t *spill_next = nullptr;
    int32_t *spill_cell = nullptr;
    double *spill_len = nullptr;
    hipEvent_t ready = nullptr;    // recorded on the submitter's stream: the inputs are written
    hipStream_t src = nullptr;     // that stream
    hipEvent_t copied = nullptr;   // recorded after the caller's last vor_server_copy_result
};

// Output memory of a released request whose copies may still be running:
// it returns to the budget once `copied` has completed.
struct PendingFree {
    hipEvent_t copied;
    size_t off, bytes;
};

struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<int64_t> reqs;      // request ids, in table order
    std::vector<uint8_t> seen;      // completion already taken from the flag
    int open = 0;                   // requests of the launch not yet seen complete
    // staging (pinned) and device copies of the launch's tables
    ReqDev *h_reqs = nullptr, *d_reqs = nullptr;
    ChunkDev *h_chunks = nullptr, *d_chunks = nullptr;
    int32_t *h_remaining = nullptr, *d_remaining = nullptr;
    ReqCount *d_count = nullptr;                      // per-request spill counter and overflow count
    int32_t *h_flags = nullptr, *d_flags = nullptr;   // host memory, mapped for the device
    unsigned int *d_head = nullptr;                   // chunk queue heads of the FP64, mixed and compact kernels
    unsigned long long *d_counters = nullptr;
    unsigned long long *h_counters = nullptr;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Chunks of kSpillChunk slots that the windows of a request take: its spill
// chunks follow them in the same arrays.
int64_t window_chunks(int64_t n, int64_t stride) { return (n * stride + kSpillChunk - 1) / kSpillChunk; }

// Output memory of a request: tau, counts and statuses; with a window of
// `stride` slots per ray also the windows followed by `chunks` spill chunks
// (cells, lengths), the chunks' links and the first chunk of every ray.
size_t request_bytes(int64_t n, int64_t stride, int64_t chunks)
{
    size_t b = align_up(n * sizeof(double)) + align_up(n * sizeof(int32_t)) + align_up(n);
    if (stride > 0) {
        const size_t slots = (size_t)(window_chunks(n, stride) + chunks) * kSpillChunk;
        b += align_up(slots * sizeof(int32_t)) + align_up(slots * sizeof(double));
        b += align_up((size_t)n * sizeof(int64_t)) + align_up((size_t)chunks * sizeof(int32_t));
    }
    return b;
}

}  // namespace

struct vor_server {
    std::vector<GridRef> grid_refs;
    std::vector<const vor_grid *> grids;
    GridRef *d_grids = nullptr;
    LocView *d_locs = nullptr;         // each grid's block lists (start cells; null lists: the bucket grid)
    char *arena = nullptr;
    size_t budget = 0, used = 0;
    std::map<size_t, size_t> free_blocks;   // offset -> size
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int64_t> waiting;
    std::map<int64_t, Request> reqs;
    int64_t next_id = 1;
    Launch launches[kStreams];
    std::thread worker;
    std::atomic<bool> stop{false};
    int device = 0;
    int blocks = 1;     // resident blocks of the mixed serving kernel
    int blocks_c = 1;   // ... of the one for grids with compact records
    int blocks64 = 1;   // ... and of the FP64 one
    vor_status fault = VOR_OK;
    hipStream_t aux = nullptr;   // the scheduler's own copies (segment counts of requests run again)
    int32_t *h_counts = nullptr; // staging for those counts
    int64_t h_counts_len = 0;
    // statistics
    int64_t n_done = 0;
    int64_t reruns = 0;
    unsigned long long crossings = 0, redecisions = 0, fallbacks = 0;
    int64_t launches_done = 0;
    int launches_running = 0;
    std::deque<int64_t> done_queue;   // completed requests not yet taken by vor_server_next_done
    std::vector<PendingFree> pending_frees;
    clk::time_point t0;

    bool arena_alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                size_t rest = it->second - bytes;
                free_blocks.erase(it);
                if (rest) free_blocks[off + bytes] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }

    void arena_free(size_t off, size_t bytes)
    {
        used -= bytes;
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
    }

    // FIFO admission: the head of the queue waits until it fits, so later
    // requests never overtake it (no starvation).
    void admit_locked()
    {
        while (!waiting.empty()) {
            Request &r = reqs[waiting.front()];
            size_t off;
            if (!arena_alloc(r.bytes, off)) break;
            r.off = off;
            char *p = arena + off;
            r.tau = (double *)p;
            p += align_up(r.n * sizeof(double));
            r.n_seg = (int32_t *)p;
            p += align_up(r.n * sizeof(int32_t));
            r.status = (uint8_t *)p;
            p += align_up(r.n);
            if (r.seg_stride > 0) {
                const int64_t wc = window_chunks(r.n, r.seg_stride);
                const size_t slots = (size_t)(wc + r.spill_chunks) * kSpillChunk;
                r.seg_cell = (int32_t *)p;
                p += align_up(slots * sizeof(int32_t));
                r.seg_len = (double *)p;
                p += align_up(slots * sizeof(double));
                r.spill_first = (int64_t *)p;
                p += align_up((size_t)r.n * sizeof(int64_t));
                r.spill_next = (int32_t *)p;
                r.spill_cell = r.seg_cell + wc * kSpillChunk;   // the spill chunks follow the windows
                r.spill_len = r.seg_len + wc * kSpillChunk;
            }
            r.state = Q_ADMITTED;
            r.t_admit = clk::now();
            waiting.pop_front();
        }
    }

    // Launch every admitted request that is not yet running on a free stream.
    // Requests are grouped by context (grid, precision class) so that a wave
    // rarely has to switch; chunks are sized for a few per wave.
    // The kernel a request's chunks run in: 0 FP64, 1 mixed, 2 mixed over a
    // grid with compact records.
    int kernel_class(const Request &r) const
    {
        return r.mode == VOR_MODE_FP64 ? 0 : (grid_refs[r.grid].blk_off ? 2 : 1);
    }

    void launch_locked(Launch &L)
    {
        L.reqs.clear();
        int64_t rays = 0;
        for (auto &kv : reqs) {
            const Request &r = kv.second;
            if (r.state != Q_ADMITTED) continue;
            if ((int)L.reqs.size() >= kMaxLaunchReqs) break;
            L.reqs.push_back(r.id);
            rays += r.n;
        }
        if (L.reqs.empty()) return;
        const int64_t waves = (int64_t)blocks * 4;
        int64_t chunk = (rays + waves * kChunksPerWave - 1) / (waves * kChunksPerWave);
        chunk = std::min<int64_t>(std::max<int64_t>(chunk, kChunkMin), kChunkMax);
        // at most half the table for the rays, the rest covers one partial chunk per request
        chunk = std::max<int64_t>(chunk, (rays + kMaxLaunchChunks / 2 - 1) / (kMaxLaunchChunks / 2));
        chunk = (chunk + 63) / 64 * 64;
        // cap the launch so its chunks fit the table
        int64_t nch_total = 0;
        size_t keep = 0;
        for (; keep < L.reqs.size(); ++keep) {
            const Request &r = reqs[L.reqs[keep]];
            const int64_t need = (r.n + chunk - 1) / chunk;
            if (nch_total + need > kMaxLaunchChunks) break;
            nch_total += need;
        }
        L.reqs.resize(keep);
        if (L.reqs.empty()) return;   // cannot happen: the requests need at most kMaxLaunchChunks / 2 + kMaxLaunchReqs chunks
        // kernel class first (FP64, mixed, mixed over compact records: each
        // has a kernel of its own), then grid
        std::stable_sort(L.reqs.begin(), L.reqs.end(), [this](int64_t x, int64_t y) {
            const int ka = kernel_class(reqs[x]), kb = kernel_class(reqs[y]);
            return (ka != kb) ? ka < kb : reqs[x].grid < reqs[y].grid;
        });
        int nch = 0, ncls[3] = {0, 0, 0};   // chunks, and those of each kernel class
        for (size_t qi = 0; qi < L.reqs.size(); ++qi) {
            Request &r = reqs[L.reqs[qi]];
            const int q = (int)qi;
            const int need = (int)((r.n + chunk - 1) / chunk);
            ReqDev &d = L.h_reqs[q];
            d.in = r.in;
            d.tau = r.tau;
            d.n_seg = r.n_seg;
            d.status = r.status;
            d.seg_cell = r.seg_cell;
            d.seg_len = r.seg_len;
            d.seg_stride = r.seg_stride;
            d.spill = SpillPool{r.spill_next, r.spill_first, r.spill_chunks,
                                r.seg_stride > 0 ? window_chunks(r.n, r.seg_stride) : 0, &L.d_count[q].spill_head};
            d.remaining = L.d_remaining + q;
            d.overflow = &L.d_count[q].overflow;
            d.done = L.d_flags + q;
            ++r.runs;
            L.h_remaining[q] = need;
            L.h_flags[q] = 0;
            const int32_t ctx = 4 * r.grid + 2 * r.in.grid_rho + (r.mode == VOR_MODE_MIXED ? 1 : 0);
            ncls[kernel_class(r)] += need;
            for (int c = 0; c < need; ++c) {
                ChunkDev &ch = L.h_chunks[nch++];
                ch.req = q;
                ch.first = (int32_t)(c * chunk);
                ch.count = (int32_t)std::min<int64_t>(chunk, r.n - (int64_t)c * chunk);
                ch.ctx = ctx;
            }
            r.state = Q_RUNNING;
        }
        const int nreq = (int)L.reqs.size();
        L.seen.assign(nreq, 0);
        L.open = nreq;
        bool ok = true;
        // the launch starts once every request's inputs are written on its submitter's
        // stream: the newest of a stream's events covers the earlier ones
        {
            std::map<hipStream_t, const Request *> newest;
            for (int64_t id : L.reqs) {
                const Request &r = reqs[id];
                if (!r.ready) continue;
                const Request *&m = newest[r.src];
                if (!m || r.id > m->id) m = &r;
            }
            for (const auto &kv : newest) ok = ok && hipStreamWaitEvent(L.stream, kv.second->ready, 0) == hipSuccess;
        }
        ok = ok && hipMemcpyAsync(L.d_reqs, L.h_reqs, sizeof(ReqDev) * nreq, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
                  hipMemcpyAsync(L.d_chunks, L.h_chunks, sizeof(ChunkDev) * nch, hipMemcpyHostToDevice, L.stream) == hipSuccess &&
                  hipMemcpyAsync(L.d_remaining, L.h_remaining, sizeof(int32_t) * nreq, hipMemcpyHostToDevice,
                                 L.stream) == hipSuccess;
        hipLaunchKernelGGL(k_zero_launch, dim3(1), dim3(256), 0, L.stream, L.d_head, L.d_counters, L.d_count, nreq);
        if (ncls[0] > 0) {
            const int nb = std::max(1, std::min(blocks64, (ncls[0] + 3) / 4));
            hipLaunchKernelGGL(k_serve<VOR_MODE_FP64>, dim3(nb), dim3(256), 0, L.stream, d_grids, d_locs, L.d_reqs,
                               L.d_chunks,
                               ncls[0], L.d_head, L.d_counters);
        }
        if (ncls[1] > 0) {
            const int nb = std::max(1, std::min(blocks, (ncls[1] + 3) / 4));
            hipLaunchKernelGGL(k_serve<VOR_MODE_MIXED>, dim3(nb), dim3(256), 0, L.stream, d_grids, d_locs, L.d_reqs,
                               L.d_chunks + ncls[0], ncls[1], L.d_head + 1, L.d_counters);
        }
        if (ncls[2] > 0) {
            const int nb = std::max(1, std::min(blocks_c, (ncls[2] + 3) / 4));
            hipLaunchKernelGGL(k_serve<kModeCompact>, dim3(nb), dim3(256), 0, L.stream, d_grids, d_locs, L.d_reqs,
                               L.d_chunks + ncls[0] + ncls[1], ncls[2], L.d_head + 2, L.d_counters);
        }
        ok = ok && hipGetLastError() == hipSuccess &&
             hipMemcpyAsync(L.h_counters, L.d_counters, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            L.stream) == hipSuccess &&
             hipEventRecord(L.done, L.stream) == hipSuccess;
        if (!ok) fault = VOR_EDEVICE;
        L.busy = true;
        ++launches_running;
    }

    void mark_done_locked(int64_t id, clk::time_point now)
    {
        auto it = reqs.find(id);
        if (it == reqs.end() || it->second.state != Q_RUNNING) return;
        it->second.state = Q_DONE;
        it->second.t_done = now;
        ++n_done;
        done_queue.push_back(id);
    }

    // A request some of whose rays found its spill chunks used up: every ray
    // has its full segment count, so the chunks its paths need are known
    // exactly. Its outputs go back to the budget and it waits again, at the
    // head of the queue, with that many chunks; the second run cannot run
    // out (the paths are the same). A request whose exact need exceeds the
    // budget ends with VOR_EBUDGET.
    void rerun_locked(int64_t id, clk::time_point now)
    {
        auto it = reqs.find(id);
        if (it == reqs.end() || it->second.state != Q_RUNNING) return;
        Request &r = it->second;
        int64_t need = 0;
        if (h_counts_len < r.n) {
            if (h_counts) (void)hipHostFree(h_counts);
            h_counts = nullptr;
            h_counts_len = 0;
            if (hipHostMalloc((void **)&h_counts, sizeof(int32_t) * r.n, hipHostMallocDefault) != hipSuccess) {
                fault = VOR_ENOMEM;
                return;
            }
            h_counts_len = r.n;
        }
        if (hipMemcpyAsync(h_counts, r.n_seg, sizeof(int32_t) * r.n, hipMemcpyDeviceToHost, aux) != hipSuccess ||
            hipStreamSynchronize(aux) != hipSuccess) {
            fault = VOR_EDEVICE;
            return;
        }
        for (int64_t i = 0; i < r.n; ++i)
            if (h_counts[i] > r.seg_stride) need += (h_counts[i] - r.seg_stride + kSpillChunk - 1) / kSpillChunk;
        arena_free(r.off, r.bytes);
        r.spill_chunks = need;
        r.bytes = request_bytes(r.n, r.seg_stride, need);
        r.tau = nullptr;
        r.n_seg = nullptr;
        r.status = nullptr;
        r.seg_cell = nullptr;
        r.seg_len = nullptr;
        r.spill_first = nullptr;
        r.spill_next = nullptr;
        r.spill_cell = nullptr;
        r.spill_len = nullptr;
        ++reruns;
        if (r.bytes > budget) {
            r.err = VOR_EBUDGET;
            r.bytes = 0;
            r.state = Q_RUNNING;   // so that mark_done_locked takes it
            mark_done_locked(id, now);
            return;
        }
        r.state = Q_WAIT;
        waiting.push_front(id);
    }

    // Requests whose flag the kernel has raised. Returns true if any.
    bool poll_flags_locked(Launch &L)
    {
        if (L.open == 0) return false;
        bool any = false;
        const auto now = clk::now();
        for (size_t q = 0; q < L.reqs.size(); ++q) {
            if (L.seen[q]) continue;
            const int32_t f = __atomic_load_n(&L.h_flags[q], __ATOMIC_ACQUIRE);
            if (f != 0) {
                L.seen[q] = 1;
                --L.open;
                if (f == 2) rerun_locked(L.reqs[q], now);
                else mark_done_locked(L.reqs[q], now);
                any = true;
            }
        }
        return any;
    }

    // Released outputs whose copies have finished go back to the budget.
    bool reap_frees_locked()
    {
        bool any = false;
        for (size_t q = 0; q < pending_frees.size();) {
            if (hipEventQuery(pending_frees[q].copied) == hipSuccess) {
                arena_free(pending_frees[q].off, pending_frees[q].bytes);
                (void)hipEventDestroy(pending_frees[q].copied);
                pending_frees[q] = pending_frees.back();
                pending_frees.pop_back();
                any = true;
            } else {
                ++q;
            }
        }
        return any;
    }

    // The launch's kernel has ended: every request in it is complete (the
    // flags of all of them are visible now).
    void complete_locked(Launch &L)
    {
        poll_flags_locked(L);
        const auto now = clk::now();
        for (size_t q = 0; q < L.reqs.size(); ++q)
            if (!L.seen[q]) mark_done_locked(L.reqs[q], now);
        crossings += L.h_counters[0];
        fallbacks += L.h_counters[1];
        redecisions += L.h_counters[2];
        ++launches_done;
        --launches_running;
        L.reqs.clear();
        L.seen.clear();
        L.open = 0;
        L.busy = false;
    }

    void run()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop.load()) {
            bool progress = false;
            for (auto &L : launches) {
                if (!L.busy) continue;
                if (poll_flags_locked(L)) progress = true;
                if (hipEventQuery(L.done) == hipSuccess) {
                    complete_locked(L);
                    progress = true;
                }
            }
            if (!pending_frees.empty() && reap_frees_locked()) progress = true;
            if (progress) cv.notify_all();
            admit_locked();
            for (auto &L : launches) {
                if (!L.busy) {
                    launch_locked(L);
                    if (L.busy) progress = true;
                }
            }
            if (!progress) {
                if (launches_running > 0 || !pending_frees.empty()) {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                    lk.lock();
                } else {
                    cv.wait_for(lk, std::chrono::milliseconds(5));
                }
            }
        }
        // drain
        for (auto &L : launches)
            if (L.busy) {
                lk.unlock();
                (void)hipEventSynchronize(L.done);
                lk.lock();
                complete_locked(L);
            }
        cv.notify_all();
    }
};

extern "C" {

vor_status vor_server_create(const vor_grid *const *grids, int32_t n_grids, int64_t budget_bytes,
                             vor_server **out)
{
    if (out) *out = nullptr;
    if (!grids || n_grids < 1 || budget_bytes <= 0 || !out) return VOR_EINVAL;
    for (int i = 0; i < n_grids; ++i)
        if (!grids[i]) return VOR_EINVAL;
    vor_server *S = new (std::nothrow) vor_server;
    if (!S) return VOR_ENOMEM;
    (void)hipGetDevice(&S->device);
    for (int i = 0; i < n_grids; ++i) {
        S->grid_refs.push_back(grid_ref(vrt_grid_of(grids[i]), 0, 0.0));
        S->grids.push_back(grids[i]);
    }
    std::vector<LocView> locs;
    for (int i = 0; i < n_grids; ++i) locs.push_back(loc_view(vrt_grid_of(grids[i])));
    bool ok = hipMalloc(&S->d_grids, sizeof(GridRef) * n_grids) == hipSuccess &&
              hipMemcpy(S->d_grids, S->grid_refs.data(), sizeof(GridRef) * n_grids, hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&S->d_locs, sizeof(LocView) * n_grids) == hipSuccess &&
              hipMemcpy(S->d_locs, locs.data(), sizeof(LocView) * n_grids, hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&S->arena, (size_t)budget_bytes) == hipSuccess;
    for (auto &L : S->launches) {
        ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc((void **)&L.h_reqs, sizeof(ReqDev) * kMaxLaunchReqs, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void **)&L.h_chunks, sizeof(ChunkDev) * kMaxLaunchChunks, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void **)&L.h_counters, 4 * sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void **)&L.h_remaining, sizeof(int32_t) * kMaxLaunchReqs, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void **)&L.h_flags, sizeof(int32_t) * kMaxLaunchReqs,
                           hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
             hipHostGetDevicePointer((void **)&L.d_flags, L.h_flags, 0) == hipSuccess &&
             hipMalloc(&L.d_remaining, sizeof(int32_t) * kMaxLaunchReqs) == hipSuccess &&
             hipMalloc(&L.d_count, sizeof(ReqCount) * kMaxLaunchReqs) == hipSuccess &&
             hipMalloc(&L.d_reqs, sizeof(ReqDev) * kMaxLaunchReqs) == hipSuccess &&
             hipMalloc(&L.d_chunks, sizeof(ChunkDev) * kMaxLaunchChunks) == hipSuccess &&
             hipMalloc(&L.d_head, 3 * sizeof(unsigned int)) == hipSuccess &&
             hipMalloc(&L.d_counters, 4 * sizeof(unsigned long long)) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&S->aux, hipStreamNonBlocking) == hipSuccess;
    int cus = 0, per_cu = 0, per_cu64 = 0, per_cu_c = 0;
    ok = ok && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) == hipSuccess &&
         hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_serve<VOR_MODE_MIXED>, 256, 0) == hipSuccess &&
         hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_c, k_serve<kModeCompact>, 256, 0) == hipSuccess &&
         hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu64, k_serve<VOR_MODE_FP64>, 256, 0) == hipSuccess;
    if (!ok) {
        vor_server_destroy(S);
        return VOR_ENOMEM;
    }
    S->blocks = std::max(1, cus * std::max(1, per_cu));
    S->blocks64 = std::max(1, cus * std::max(1, per_cu64));
    S->blocks_c = std::max(1, cus * std::max(1, per_cu_c));
    S->budget = (size_t)budget_bytes;
    S->free_blocks[0] = S->budget;
    S->t0 = clk::now();
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return VOR_OK;
}

vor_status vor_server_submit(vor_server *S, int32_t grid, const double *origins, const double *dirs, int64_t n,
                             const double *density, double kappa, int32_t mode, int64_t seg_stride,
                             int64_t spill_chunks, void *stream, int64_t *req_id)
{
    if (req_id) *req_id = 0;
    const bool grid_rho = (mode & VOR_SERVE_GRID_DENSITY) != 0;
    mode &= ~VOR_SERVE_GRID_DENSITY;
    if (!S || !req_id || grid < 0 || grid >= (int32_t)S->grid_refs.size() || n < 1 || n > 0x7fffffffLL ||
        !origins || !dirs || seg_stride < 0 || (mode != VOR_MODE_FP64 && mode != VOR_MODE_MIXED) ||
        spill_chunks < 0 || spill_chunks > 0x7fffffffLL || (seg_stride == 0 && spill_chunks != 0))
        return VOR_EINVAL;
    if (grid_rho && (density || !vrt_grid_of(S->grids[grid]).rho_bound)) return VOR_EINVAL;
    size_t bytes = request_bytes(n, seg_stride, spill_chunks);
    if (bytes > S->budget) return VOR_EBUDGET;
    // the launch that traces the request waits for what the submitter's stream has enqueued so far
    hipEvent_t ready = nullptr;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return VOR_EDEVICE;
    if (hipEventRecord(ready, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(ready);
        return VOR_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fault != VOR_OK) {
        (void)hipEventDestroy(ready);
        return S->fault;
    }
    Request r;
    r.id = S->next_id++;
    r.grid = grid;
    r.mode = mode;
    r.n = n;
    r.in.origins = origins;
    r.in.dirs = dirs;
    r.in.density = density;
    r.in.kappa = kappa;
    r.in.enter = 0;
    r.in.grid_rho = grid_rho ? 1 : 0;
    r.seg_stride = seg_stride;
    r.spill_chunks = spill_chunks;
    r.bytes = bytes;
    r.ready = ready;
    r.src = (hipStream_t)stream;
    r.t_submit = clk::now();
    S->reqs[r.id] = r;
    S->waiting.push_back(r.id);
    *req_id = r.id;
    S->cv.notify_all();
    return VOR_OK;
}

vor_status vor_server_poll(vor_server *S, int64_t req, int32_t *done)
{
    if (!S || !done) return VOR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end() || it->second.state == Q_RELEASED) return VOR_EINVAL;
    *done = it->second.state == Q_DONE ? 1 : 0;
    return S->fault;
}

vor_status vor_server_wait(vor_server *S, int64_t req, double timeout_s)
{
    if (!S) return VOR_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
    for (;;) {
        auto it = S->reqs.find(req);
        if (it == S->reqs.end() || it->second.state == Q_RELEASED) return VOR_EINVAL;
        if (it->second.state == Q_DONE) return it->second.err;
        if (S->fault != VOR_OK) return S->fault;
        if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout && clk::now() >= deadline) {
            auto it2 = S->reqs.find(req);
            return (it2 != S->reqs.end() && it2->second.state == Q_DONE) ? it2->second.err : VOR_ETIMEOUT;
        }
    }
}

vor_status vor_server_next_done(vor_server *S, double timeout_s, int64_t *req_id)
{
    if (req_id) *req_id = 0;
    if (!S || !req_id) return VOR_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
    for (;;) {
        while (!S->done_queue.empty()) {
            const int64_t id = S->done_queue.front();
            S->done_queue.pop_front();
            auto it = S->reqs.find(id);
            if (it != S->reqs.end() && it->second.state == Q_DONE) {
                *req_id = id;
                return VOR_OK;
            }
        }
        if (S->fault != VOR_OK) return S->fault;
        if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout && clk::now() >= deadline && S->done_queue.empty())
            return VOR_ETIMEOUT;
    }
}

vor_status vor_server_result(vor_server *S, int64_t req, vor_trace_out *out, double *latency_s)
{
    if (!S || !out) return VOR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end() || it->second.state != Q_DONE) return VOR_EINVAL;
    const Request &r = it->second;
    if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
    if (r.err != VOR_OK) return r.err;
    *out = vor_trace_out{};
    out->tau = r.tau;
    out->n_seg = r.n_seg;
    out->status = r.status;
    out->seg_cell = r.seg_cell;
    out->seg_len = r.seg_len;
    out->seg_stride = r.seg_stride;
    out->spill_first = r.spill_first;
    out->spill_next = r.spill_next;
    out->spill_cell = r.spill_cell;
    out->spill_len = r.spill_len;
    out->spill_chunks = r.spill_chunks;
    return VOR_OK;
}

vor_status vor_server_copy_result(vor_server *S, int64_t req, double *tau, int32_t *n_seg, uint8_t *status,
                                  const int64_t *ray_off, int32_t *seg_cell, double *seg_len, void *stream)
{
    if (!S) return VOR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end() || it->second.state != Q_DONE) return VOR_EINVAL;
    Request &r = it->second;
    if (r.err != VOR_OK) return r.err;
    if ((seg_cell || seg_len) && (!seg_cell || !seg_len || !ray_off || r.seg_stride <= 0)) return VOR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    bool ok = r.copied || hipEventCreateWithFlags(&r.copied, hipEventDisableTiming) == hipSuccess;
    if (tau) ok = ok && hipMemcpyAsync(tau, r.tau, r.n * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (n_seg) ok = ok && hipMemcpyAsync(n_seg, r.n_seg, r.n * sizeof(int32_t), hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (status) ok = ok && hipMemcpyAsync(status, r.status, r.n, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (seg_cell)   // the request's chunks follow its windows in the same arrays (spill_cell / spill_len)
        ok = ok && vrt_gather_paths(r.n_seg, r.n, r.seg_cell, r.seg_len, r.seg_stride, r.spill_first, r.spill_next,
                                    r.spill_cell, r.spill_len, ray_off, seg_cell, seg_len, st) == VOR_OK;
    ok = ok && hipEventRecord(r.copied, st) == hipSuccess;   // release waits for this
    return ok ? VOR_OK : VOR_EDEVICE;
}

vor_status vor_server_release(vor_server *S, int64_t req)
{
    if (!S) return VOR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(req);
    if (it == S->reqs.end() || it->second.state != Q_DONE) return VOR_EINVAL;
    if (it->second.bytes == 0) {   // ended with an error: holds no memory
        if (it->second.copied) (void)hipEventDestroy(it->second.copied);
    } else if (it->second.copied && hipEventQuery(it->second.copied) != hipSuccess) {
        S->pending_frees.push_back(PendingFree{it->second.copied, it->second.off, it->second.bytes});
    } else {
        if (it->second.copied) (void)hipEventDestroy(it->second.copied);
        S->arena_free(it->second.off, it->second.bytes);
    }
    if (it->second.ready) (void)hipEventDestroy(it->second.ready);
    S->reqs.erase(it);
    // ids of released requests are skipped by vor_server_next_done; drop
    // them once they make up most of its queue (callers that only wait/poll)
    if (S->done_queue.size() > 2 * S->reqs.size() + 64) {
        std::deque<int64_t> keep;
        for (int64_t id : S->done_queue)
            if (S->reqs.count(id)) keep.push_back(id);
        S->done_queue.swap(keep);
    }
    S->cv.notify_all();
    return VOR_OK;
}

vor_status vor_server_get_stats(vor_server *S, vor_server_stats *st)
{
    if (!S || !st) return VOR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    st->completed = S->n_done;
    st->crossings = (int64_t)S->crossings;
    st->fp64_redecisions = (int64_t)S->redecisions;
    st->fallbacks = (int64_t)S->fallbacks;
    st->launches = S->launches_done;
    st->running = S->launches_running;
    st->waiting = (int64_t)S->waiting.size();
    st->budget_bytes = (int64_t)S->budget;
    st->used_bytes = (int64_t)S->used;
    st->uptime_s = std::chrono::duration<double>(clk::now() - S->t0).count();
    st->reruns = S->reruns;
    return S->fault;
}

void vor_server_destroy(vor_server *S)
{
    if (!S) return;
    if (S->worker.joinable()) {
        S->stop.store(true);
        S->cv.notify_all();
        S->worker.join();
    }
    for (auto &L : S->launches) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.h_reqs) (void)hipHostFree(L.h_reqs);
        if (L.h_chunks) (void)hipHostFree(L.h_chunks);
        if (L.h_counters) (void)hipHostFree(L.h_counters);
        if (L.h_remaining) (void)hipHostFree(L.h_remaining);
        if (L.h_flags) (void)hipHostFree(L.h_flags);
        if (L.d_remaining) (void)hipFree(L.d_remaining);
        if (L.d_count) (void)hipFree(L.d_count);
        if (L.d_reqs) (void)hipFree(L.d_reqs);
        if (L.d_chunks) (void)hipFree(L.d_chunks);
        if (L.d_head) (void)hipFree(L.d_head);
        if (L.d_counters) (void)hipFree(L.d_counters);
    }
    // copies of outputs still running finish before the arena goes
    for (auto &f : S->pending_frees) {
        (void)hipEventSynchronize(f.copied);
        (void)hipEventDestroy(f.copied);
    }
    for (auto &kv : S->reqs) {
        if (kv.second.copied) {
            (void)hipEventSynchronize(kv.second.copied);
            (void)hipEventDestroy(kv.second.copied);
        }
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    }
    if (S->aux) {
        (void)hipStreamSynchronize(S->aux);
        (void)hipStreamDestroy(S->aux);
    }
    if (S->h_counts) (void)hipHostFree(S->h_counts);
    if (S->arena) (void)hipFree(S->arena);
    if (S->d_grids) (void)hipFree(S->d_grids);
    if (S->d_locs) (void)hipFree(S->d_locs);
    delete S;
}

}  // extern "C"
