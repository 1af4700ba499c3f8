// Exclusive prefix sums of int32 arrays: one workgroup for small arrays, else three
// phases (tile scan, tile-offset scan, add).
#include "common.h"

namespace nair {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of one value per thread over a 256-thread block; returns the
// prefix and writes the block total to *total.
__device__ int block_exclusive_scan(int v, int *lds_waves, int *total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            int t = lds_waves[w];
            lds_waves[w] = run;
            run += t;
        }
        lds_waves[kScanThreads / 64] = run;
    }
    __syncthreads();
    int res = x - v + lds_waves[wave];
    *total = lds_waves[kScanThreads / 64];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int *__restrict__ in, int *__restrict__ out,
                                                            int n, int *__restrict__ tile_sums) {
    __shared__ int lds[kScanThreads / 64 + 1];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int total;
    int pre = block_exclusive_scan(s, lds, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One block scans the tile sums in chunks of 256 with a running carry.
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(int *__restrict__ tile_sums, int ntiles,
                                                                int *__restrict__ grand_total,
                                                                int *__restrict__ total_copy) {
    __shared__ int lds[kScanThreads / 64 + 1];
    int carry = 0;
    for (int c0 = 0; c0 < ntiles; c0 += kScanThreads) {
        int i = c0 + threadIdx.x;
        int v = (i < ntiles) ? tile_sums[i] : 0;
        int total;
        int pre = block_exclusive_scan(v, lds, &total);
        if (i < ntiles) tile_sums[i] = pre + carry;
        carry += total;
    }
    if (threadIdx.x == 0) {
        *grand_total = carry;
        if (total_copy) *total_copy = carry;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int *__restrict__ out, int n,
                                                          const int *__restrict__ tile_sums) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    const int add = tile_sums[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads) {
        int64_t i = base + k;
        if (i < n) out[i] += add;
    }
}

// Small arrays: one 1024-thread workgroup; wave w scans its contiguous chunk
// in strips of 64 (one coalesced load per lane and strip, a wave scan per
// strip with a running carry), after the chunk totals are scanned in LDS.
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallStrips = 16;                                  // strips of 64 per wave
constexpr int kSmallMax = kSmallWaves * kSmallStrips * 64;

__global__ __launch_bounds__(kSmallThreads) void k_scan_small(const int *__restrict__ in, int *__restrict__ out,
                                                             int n, int *__restrict__ total_copy) {
    __shared__ int wsum[kSmallWaves + 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int strips = (n + kSmallWaves * 64 - 1) / (kSmallWaves * 64);   // per wave, <= kSmallStrips
    const int lo = wave * strips * 64;
    int v[kSmallStrips];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kSmallStrips; ++j) {
        const int i = lo + j * 64 + lane;
        v[j] = (j < strips && i < n) ? in[i] : 0;
        s += v[j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) wsum[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < kSmallWaves; ++w) {
            const int t = wsum[w];
            wsum[w] = run;
            run += t;
        }
        wsum[kSmallWaves] = run;
    }
    __syncthreads();
    int carry = wsum[wave];
#pragma unroll
    for (int j = 0; j < kSmallStrips; ++j) {
        if (j >= strips) break;
        int x = v[j];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        const int i = lo + j * 64 + lane;
        if (i < n) out[i] = carry + x - v[j];
        carry += __shfl(x, 63, 64);
    }
    if (threadIdx.x == 0) {
        out[n] = wsum[kSmallWaves];
        if (total_copy) *total_copy = wsum[kSmallWaves];
    }
}

}  // namespace

void scan_exclusive(const int *in, int *out, int n, hipStream_t s, int *total_copy) {
    if (n <= 0) {
        NAIR_HIP(hipMemsetAsync(out, 0, sizeof(int), s));
        if (total_copy) NAIR_HIP(hipMemsetAsync(total_copy, 0, sizeof(int), s));
        return;
    }
    if (n <= kSmallMax) {
        k_scan_small<<<1, kSmallThreads, 0, s>>>(in, out, n, total_copy);
        NAIR_HIP(hipGetLastError());
        return;
    }
    const int ntiles = static_cast<int>((static_cast<int64_t>(n) + kScanTile - 1) / kScanTile);
    DBuf<int> tiles(ntiles);
    k_scan_tiles<<<ntiles, kScanThreads, 0, s>>>(in, out, n, tiles.get());
    k_scan_tile_sums<<<1, kScanThreads, 0, s>>>(tiles.get(), ntiles, out + n, total_copy);
    k_scan_add<<<ntiles, kScanThreads, 0, s>>>(out, n, tiles.get());
    NAIR_HIP(hipGetLastError());
    // `tiles` returns to the pool now; any later user of that memory is ordered after
    // these kernels on the same stream (the library runs one call at a time).
}

}  // namespace nair
