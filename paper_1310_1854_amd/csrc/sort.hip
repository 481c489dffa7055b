// sort.hip -- stable LSD radix sort of (uint32 key, int32 value) pairs, 8
// bits per pass. Used once per grid build to put the sites in Hilbert order.
//
// Per pass: a per-tile digit histogram (LDS atomics), an exclusive scan of
// the digit-major histogram (digit d's slot for tile t lands after every
// smaller digit and every earlier tile), and a stable scatter in which each
// 64-lane wave ranks equal digits with eight ballots and the waves of a
// block combine their per-digit counts through LDS.
#include "vrt_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;

__global__ void __launch_bounds__(kThreads) k_digit_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                         int32_t *__restrict__ hist, int64_t ntiles)
{
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

__global__ void __launch_bounds__(kThreads) k_digit_scatter(const uint32_t *__restrict__ kin,
                                                            const int32_t *__restrict__ vin, int64_t n, int shift,
                                                            const int32_t *__restrict__ off, int64_t ntiles,
                                                            uint32_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[kWaves][256];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    run[tid] = off[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        int64_t idx = base + (int64_t)r * kThreads + tid;
        bool valid = idx < n;
        uint32_t key = valid ? kin[idx] : 0u;
        int32_t val = valid ? vin[idx] : 0;
        uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
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
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles < 1) ntiles = 1;
    return 256 * ntiles;
}

// hist_scratch must hold 2 * hist_len + 1 int32. The sorted pairs end in
// (keys, vals); keys_tmp / vals_tmp are ping-pong buffers of n entries.
vor_status vrt_radix_sort_pairs(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int64_t n,
                                int bits, int32_t *hist_scratch, int64_t hist_len, hipStream_t st)
{
    if (n <= 1) return VOR_OK;
    if (n > 0x7fffffff) return VOR_EINVAL;
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (hist_len < 256 * ntiles) return VOR_EINVAL;
    int32_t *hist = hist_scratch;
    int32_t *off = hist_scratch + hist_len;
    uint32_t *ka = keys, *kb = keys_tmp;
    int32_t *va = vals, *vb = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, n, shift, hist, ntiles);
        vor_status s = vrt_scan_i32_to_i32(hist, 256 * ntiles, off, st);
        if (s != VOR_OK) return s;
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)ntiles), dim3(kThreads), 0, st, ka, va, n, shift, off,
                           ntiles, kb, vb);
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
