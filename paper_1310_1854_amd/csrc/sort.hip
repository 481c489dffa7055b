// sort.hip -- stable LSD radix sort of (uint32 key, int32 value) pairs, 8
// bits per pass. Used by the grid build (sites in Hilbert order) and by the
// coherent ray order.
//
// Per pass, three launches: a per-tile digit histogram (LDS atomics) laid
// out digit-major; one block per digit that scans its row along the tiles in
// place and leaves the digit's total; and a stable scatter. The scatter
// scans the 256 totals itself, so digit d of tile t starts at (keys of every
// smaller digit) + (keys of digit d in earlier tiles). In it each 64-lane
// wave ranks equal digits with eight ballots over its own quarter of the
// tile, the waves then combine their per-digit counts through LDS, and the
// tile is reordered in LDS so that its runs of equal digits are written out
// contiguously.
#include "vrt_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Keys per tile: 256 threads times 16 rounds, or times 4 below kSmallTileKeys
// keys, where tiles of 4096 would leave compute units idle.
constexpr int kRoundsBig = 16, kRoundsSmall = 4;
#ifndef VRT_SORT_SMALL_TILE_KEYS
#define VRT_SORT_SMALL_TILE_KEYS (1 << 22)
#endif
constexpr int64_t kSmallTileKeys = VRT_SORT_SMALL_TILE_KEYS;
inline int sort_rounds(int64_t n) { return n < kSmallTileKeys ? kRoundsSmall : kRoundsBig; }
inline int64_t sort_tiles(int64_t n)
{
    const int64_t tile = (int64_t)kThreads * sort_rounds(n);
    return (n + tile - 1) / tile;
}

template <int kRounds>
__global__ void __launch_bounds__(kThreads) k_digit_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                         int32_t *__restrict__ hist, int64_t ntiles)
{
    constexpr int kTile = kThreads * kRounds;
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        int64_t idx = base + (int64_t)r * kThreads + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of row d = blockIdx.x of the digit-major histogram, in
// place (the count of digit d in the tiles before each tile), and the row's
// total in tot[d]. Each thread takes 8 consecutive tiles per round.
__global__ void __launch_bounds__(kThreads) k_digit_rows(int32_t *__restrict__ hist, int64_t ntiles,
                                                         int32_t *__restrict__ tot)
{
    constexpr int kItems = 8;
    __shared__ int32_t wsum[kWaves];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    int32_t carry = 0;
    for (int64_t c = 0; c < ntiles; c += (int64_t)kThreads * kItems) {
        const int64_t first = c + (int64_t)tid * kItems;
        int32_t v[kItems];
        int32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            v[i] = (first + i < ntiles) ? row[first + i] : 0;
            sum += v[i];
        }
        int32_t incl = sum;   // inclusive scan over the wave
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int32_t u = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += u;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int32_t before = 0, round = 0;
        for (int w = 0; w < kWaves; ++w) {
            before += (w < wave) ? wsum[w] : 0;
            round += wsum[w];
        }
        __syncthreads();   // wsum is rewritten in the next round
        int32_t run = carry + before + incl - sum;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            if (first + i < ntiles) row[first + i] = run;
            run += v[i];
        }
        carry += round;
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one tile. Each wave ranks its own quarter of the tile
// (consecutive indices), 64 keys at a time: eight ballots group the lanes
// with equal digits, and the wave keeps its running count of each digit in
// LDS, so the waves need no barrier until their quarters are ranked. Then
// the per-digit counts of the waves are combined (a digit's keys of wave w
// follow those of the earlier waves: the order of the indices), the tile is
// put in digit order in LDS, and written out in that order, so that runs of
// equal digits leave contiguously.
template <int kRounds>
__global__ void __launch_bounds__(kThreads) k_digit_scatter(const uint32_t *__restrict__ kin,
                                                            const int32_t *__restrict__ vin, int64_t n, int shift,
                                                            const int32_t *__restrict__ rows,
                                                            const int32_t *__restrict__ tot, int64_t ntiles,
                                                            uint32_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    constexpr int kTile = kThreads * kRounds;
    constexpr int kQuarter = kTile / kWaves;        // keys a wave ranks
    constexpr int kWaveRounds = kQuarter / 64;
    __shared__ int32_t wcnt[kWaves][256];           // each wave's running count of each digit, then its offset
    __shared__ int32_t loc[256];                    // where each digit's run starts in the tile
    __shared__ int32_t dst[256];                    // where it starts in the output
    __shared__ uint32_t skey[kTile];
    __shared__ int32_t sval[kTile];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int cnt = (int)((n - base) < kTile ? (n - base) : kTile);
    int32_t *mine = wcnt[wave];
    for (int d = lane; d < 256; d += 64) mine[d] = 0;
    __builtin_amdgcn_wave_barrier();

    // phase 1: each wave ranks its quarter in index order, with no block barrier
    uint32_t key[kWaveRounds];
    int32_t val[kWaveRounds], pos[kWaveRounds];
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r) {
        const int i = wave * kQuarter + r * 64 + lane;
        const bool valid = i < cnt;
        key[r] = valid ? kin[base + i] : 0u;
        val[r] = valid ? vin[base + i] : 0;
        const uint32_t d = (key[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        pos[r] = valid ? mine[d] + rank : -1;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) mine[d] += __popcll(peers);   // one lane per digit group
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // phase 2: the tile's digit totals and the batch's, their exclusive scans (wave 0
    // the tile's, wave 1 the batch's: 4 digits per lane), and each wave's offset per digit
    {
        int t = 0;
        for (int w = 0; w < kWaves; ++w) t += wcnt[w][tid];
        loc[tid] = t;
        dst[tid] = tot[tid];
    }
    __syncthreads();
    if (tid < 128) {
        int32_t *a = (tid < 64) ? loc : dst;
        const int c0 = a[4 * lane], c1 = a[4 * lane + 1], c2 = a[4 * lane + 2], c3 = a[4 * lane + 3];
        int v = c0 + c1 + c2 + c3;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int u = __shfl_up(v, dd, 64);
            if (lane >= dd) v += u;
        }
        const int e = v - (c0 + c1 + c2 + c3);
        a[4 * lane] = e;
        a[4 * lane + 1] = e + c0;
        a[4 * lane + 2] = e + c0 + c1;
        a[4 * lane + 3] = e + c0 + c1 + c2;
    }
    __syncthreads();
    dst[tid] += rows[(int64_t)tid * ntiles + blockIdx.x];
    {
        int run = loc[tid];
        for (int w = 0; w < kWaves; ++w) {
            const int c = wcnt[w][tid];
            wcnt[w][tid] = run;
            run += c;
        }
    }
    __syncthreads();

    // phase 3: the tile in digit order in LDS
#pragma unroll
    for (int r = 0; r < kWaveRounds; ++r) {
        if (pos[r] >= 0) {
            const uint32_t d = (key[r] >> shift) & 255u;
            const int p = mine[d] + pos[r];
            skey[p] = key[r];
            sval[p] = val[r];
        }
    }
    __syncthreads();

    // phase 4: out in digit order: slot j of digit d goes after the smaller digits and the digit's earlier tiles
    for (int j = tid; j < cnt; j += kThreads) {
        const uint32_t k = skey[j];
        const uint32_t d = (k >> shift) & 255u;
        const int64_t q = (int64_t)dst[d] + (j - loc[d]);
        kout[q] = k;
        vout[q] = sval[j];
    }
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const int32_t *__restrict__ idx, int64_t n,
                             uint32_t *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

vor_status vrt_gather_u32(const uint32_t *src, const int32_t *idx, int64_t n, uint32_t *dst, hipStream_t st)
{
    if (n <= 0) return VOR_OK;
    hipLaunchKernelGGL(k_gather_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, idx, n, dst);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

int64_t vrt_radix_hist_len(int64_t n)
{
    int64_t ntiles = sort_tiles(n);
    if (ntiles < 1) ntiles = 1;
    return 256 * ntiles;
}

// hist_scratch must hold hist_len + 256 int32. The sorted pairs end in
// (keys, vals); keys_tmp / vals_tmp are ping-pong buffers of n entries.
vor_status vrt_radix_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int64_t n,
                                int bits, int32_t *hist_scratch, int64_t hist_len, hipStream_t st)
{
    if (n <= 1) return VOR_OK;
    if (n > 0x7fffffff) return VOR_EINVAL;
    const int64_t ntiles = sort_tiles(n);
    const bool small = sort_rounds(n) == kRoundsSmall;
    if (hist_len < 256 * ntiles) return VOR_EINVAL;
    int32_t *hist = hist_scratch;
    int32_t *tot = hist_scratch + hist_len;
    uint32_t *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        if (small)
            hipLaunchKernelGGL(k_digit_hist<kRoundsSmall>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, n, shift,
                               hist, ntiles);
        else
            hipLaunchKernelGGL(k_digit_hist<kRoundsBig>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, n, shift,
                               hist, ntiles);
        hipLaunchKernelGGL(k_digit_rows, dim3(256), dim3(kThreads), 0, st, hist, ntiles, tot);
        if (small)
            hipLaunchKernelGGL(k_digit_scatter<kRoundsSmall>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, va, n,
                               shift, hist, tot, ntiles, kb, vb);
        else
            hipLaunchKernelGGL(k_digit_scatter<kRoundsBig>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, va, n,
                               shift, hist, tot, ntiles, kb, vb);
        uint32_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        if (hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return VOR_EDEVICE;
    }
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}
