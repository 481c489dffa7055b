// scan.hip -- exclusive prefix sums of non-negative int32 counts, used for
// CSR row offsets, bucket offsets and per-ray segment offsets.
//
// Three launches and no temporary buffer: tile totals are parked in the
// output at the tile-end positions, scanned in place by one block, and each
// tile then writes its own prefix (the value it rewrites at its end position
// equals what the in-place scan left there, so neighbouring tiles can read
// it concurrently).
#include "vrt_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T *lds, T *total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < blockDim.x; off <<= 1) {
        T add = (t >= off) ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    T incl = lds[t];
    if (total) *total = lds[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

template <typename OutT>
__global__ void __launch_bounds__(kThreads) k_tile_totals(const int32_t *__restrict__ counts, int64_t n,
                                                          OutT *__restrict__ out)
{
    __shared__ OutT lds[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    OutT s = 0;
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
        if (idx < n) s += (OutT)counts[idx];
    }
    OutT total;
    block_exclusive_scan<OutT>(s, lds, &total);
    if (threadIdx.x == 0) {
        int64_t end = base + kTile;
        out[end < n ? end : n] = total;
    }
}

template <typename OutT>
__global__ void __launch_bounds__(1024) k_scan_totals(OutT *__restrict__ out, int64_t n, int64_t ntiles)
{
    __shared__ OutT lds[1024];
    OutT carry = 0;
    for (int64_t c = 0; c < ntiles; c += blockDim.x) {
        int64_t b = c + threadIdx.x;
        int64_t pos = (b + 1) * kTile;
        if (pos > n) pos = n;
        OutT v = (b < ntiles) ? out[pos] : OutT(0);
        OutT total;
        OutT ex = block_exclusive_scan<OutT>(v, lds, &total);
        if (b < ntiles) out[pos] = carry + ex + v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0;
}

template <typename OutT>
__global__ void __launch_bounds__(kThreads) k_tile_scan(const int32_t *__restrict__ counts, int64_t n,
                                                        OutT *__restrict__ out)
{
    __shared__ OutT lds[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    OutT tile_base = (blockIdx.x == 0) ? OutT(0) : out[base];
    // each thread owns kItems consecutive elements
    OutT v[kItems];
    OutT s = 0;
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
        v[i] = (idx < n) ? (OutT)counts[idx] : OutT(0);
        s += v[i];
    }
    OutT ex = block_exclusive_scan<OutT>(s, lds, nullptr);
    OutT run = tile_base + ex;
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
        run += v[i];
        if (idx < n) out[idx + 1] = run;
    }
}

template <typename OutT>
vor_status scan_impl(const int32_t *counts, int64_t n, OutT *out, hipStream_t st)
{
    if (n < 0 || (!out) || (n > 0 && !counts)) return VOR_EINVAL;
    if (n == 0) {
        OutT zero = 0;
        return hipMemcpyAsync(out, &zero, sizeof(OutT), hipMemcpyHostToDevice, st) == hipSuccess ? VOR_OK
                                                                                                   : VOR_EDEVICE;
    }
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles > 0x7fffffff) return VOR_EINVAL;
    hipLaunchKernelGGL(k_tile_totals<OutT>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, counts, n, out);
    hipLaunchKernelGGL(k_scan_totals<OutT>, dim3(1), dim3(1024), 0, st, out, n, ntiles);
    hipLaunchKernelGGL(k_tile_scan<OutT>, dim3((unsigned)ntiles), dim3(kThreads), 0, st, counts, n, out);
    return hipGetLastError() == hipSuccess ? VOR_OK : VOR_EDEVICE;
}

}  // namespace

vor_status vrt_scan_i32_to_i64(const int32_t *counts, int64_t n, int64_t *offsets, hipStream_t st)
{
    return scan_impl<int64_t>(counts, n, offsets, st);
}

vor_status vrt_scan_i32_to_i32(const int32_t *counts, int64_t n, int32_t *offsets, hipStream_t st)
{
    return scan_impl<int32_t>(counts, n, offsets, st);
}

extern "C" vor_status vor_exclusive_scan(const int32_t *counts, int64_t N, int64_t *offsets, void *stream)
{
    return vrt_scan_i32_to_i64(counts, N, offsets, (hipStream_t)stream);
}
