// Device-wide exclusive prefix sum of int32 counts (reduce, scan of tile
// sums, scan-and-apply).  The item count may live in device memory so the
// scan can follow kernels whose output size is only known on the device.
#include "dev_common.h"

namespace oc {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096
constexpr int kScanMaxTiles = 1024 * 64;

__device__ inline int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan of one value per thread over a block of kScanThreads
__device__ inline int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *__restrict__ in, const int *n_dev,
                                                              int64_t n_host, int32_t *__restrict__ tsum)
{
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int s = 0;
    if (base < n) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
            if (i < n) s += in[i];
        }
    }
    int tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// single block: exclusive scan of the tile sums in place, total at tsum[nt]
__global__ __launch_bounds__(1024) void k_scan_tiles(int32_t *tsum, int nt)
{
    __shared__ int wsum[16];
    const int per = (nt + 1023) / 1024;
    const int lo = threadIdx.x * per;
    int loc = 0;
    for (int k = 0; k < per; ++k)
        if (lo + k < nt) loc += tsum[lo + k];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = wave_incl_scan(loc);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    int run = off + inc - loc;
    for (int k = 0; k < per; ++k)
        if (lo + k < nt) {
            int v = tsum[lo + k];
            tsum[lo + k] = run;
            run += v;
        }
    if (threadIdx.x == 0) tsum[nt] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *__restrict__ in,
                                                             int32_t *__restrict__ out, const int *n_dev,
                                                             int64_t n_host, const int32_t *__restrict__ tsum,
                                                             int nt)
{
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tsum[nt];
    if (base >= n) return;
    // each thread owns kScanItems consecutive items
    int v[kScanItems];
    int s = 0;
    const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = my + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl_scan(s, &tot) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = my + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// Scan-and-apply that finds its tile's offset itself (the sum of the tile
// sums before it, and block 0 also the total): with few tiles this saves the
// separate tile-scan launch.
__device__ inline int block_sum(int v)
{
    __shared__ int bs[kScanThreads / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) bs[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) t += bs[w];
    return t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply_direct(const int32_t *__restrict__ in,
                                                                    int32_t *__restrict__ out, const int *n_dev,
                                                                    int64_t n_host, const int32_t *__restrict__ tsum,
                                                                    int nt)
{
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    if (blockIdx.x == 0) {
        int pt = 0;
        for (int t = threadIdx.x; t < nt; t += kScanThreads) pt += tsum[t];
        const int tot = block_sum(pt);
        if (threadIdx.x == 0) out[n] = tot;
    }
    if (base >= n) return;
    int pp = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kScanThreads) pp += tsum[t];
    const int pre = block_sum(pp);
    int v[kScanItems];
    int s = 0;
    const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = my + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl_scan(s, &tot) + pre;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = my + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// the direct apply has each block add the tile sums before it (at most
// this many: 32 KB of reads for the last block), so scans up to 32 M items
// need two launches, not three
constexpr int kScanDirectMaxTiles = 8192;

int64_t scan_tmp_ints(int64_t cap) { return (cap + kScanTile - 1) / kScanTile + 1; }
int64_t scan_max_items() { return (int64_t)kScanMaxTiles * kScanTile; }

// One block for short arrays: chunks of kSingleChunk items in order, each
// scanned by the block and offset by the running total (one launch instead
// of a reduce and an apply).
constexpr int kSingleThreads = 1024;
constexpr int kSingleItems = 4;
constexpr int kSingleChunk = kSingleThreads * kSingleItems;
constexpr int64_t kSingleMax = 4 * kSingleChunk;   // at most four chunks

__global__ __launch_bounds__(kSingleThreads) void k_scan_single(const int32_t *__restrict__ in,
                                                                int32_t *__restrict__ out, const int *n_dev,
                                                                int64_t n_host)
{
    __shared__ int wsum[kSingleThreads / 64];
    // the device count never exceeds the capacity the arrays were sized for
    const int64_t n = n_dev ? ((int64_t)*n_dev < n_host ? (int64_t)*n_dev : n_host) : n_host;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int run = 0;   // total of the chunks before (the same on every thread)
    for (int64_t base = 0; base < n; base += kSingleChunk) {
        int v[kSingleItems];
        int s = 0;
        const int64_t my = base + (int64_t)threadIdx.x * kSingleItems;
#pragma unroll
        for (int k = 0; k < kSingleItems; ++k) {
            v[k] = my + k < n ? in[my + k] : 0;
            s += v[k];
        }
        const int inc = wave_incl_scan(s);
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kSingleThreads / 64; ++w) {
            if (w < wid) off += wsum[w];
            tot += wsum[w];
        }
        __syncthreads();
        int r = run + off + inc - s;
#pragma unroll
        for (int k = 0; k < kSingleItems; ++k) {
            if (my + k < n) out[my + k] = r;
            r += v[k];
        }
        run += tot;
    }
    if (threadIdx.x == 0) out[n] = run;
}

oc_status scan_exclusive(oc_ctx *ctx, hipStream_t st, const int32_t *in, int32_t *out, int64_t cap,
                         const int *n_dev, int32_t *tmp)
{
    if (cap <= kSingleMax) {
        size_t slot;
        time_begin(ctx, st, "scan", &slot);
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kSingleThreads), 0, st, in, out, n_dev, cap);
        time_end(ctx, st, slot);
        OC_HIP(hipGetLastError());
        return OC_OK;
    }
    int64_t nt = (cap + kScanTile - 1) / kScanTile;
    if (nt < 1) nt = 1;
    if (nt > kScanMaxTiles) {
        set_error("scan: too many items");
        return OC_EINVAL;
    }
    size_t slot;
    time_begin(ctx, st, "scan", &slot);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(kScanThreads), 0, st, in, n_dev, cap, tmp);
    if (nt <= kScanDirectMaxTiles) {
        hipLaunchKernelGGL(k_scan_apply_direct, dim3((unsigned)nt), dim3(kScanThreads), 0, st, in, out, n_dev, cap,
                           tmp, (int)nt);
    } else {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tmp, (int)nt);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kScanThreads), 0, st, in, out, n_dev, cap, tmp,
                           (int)nt);
    }
    time_end(ctx, st, slot);
    OC_HIP(hipGetLastError());
    return OC_OK;
}

}  // namespace oc
