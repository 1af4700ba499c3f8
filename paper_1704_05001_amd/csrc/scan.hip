// Exclusive prefix sums of int32 arrays: one workgroup for small arrays, else three
// phases (tile scan, tile-offset scan, add).  Two arrays can be scanned by the
// same launches (the workgroup's grid index picks the array).
#include <algorithm>

#include "common.h"

namespace nair {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Up to two scans done together: in[k][0..n[k]) -> out[k] (out[k][n[k]] =
// total), the total also to total_copy[k] when that is not null.
struct ScanJobs {
    const int *in[2];
    int *out[2];
    int *total_copy[2];
    int *tiles[2];
    int n[2];
};

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

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(ScanJobs J) {
    __shared__ int lds[kScanThreads / 64 + 1];
    const int n = J.n[blockIdx.y];
    if (static_cast<int64_t>(blockIdx.x) * kScanTile >= n) return;   // past this array's tiles (whole block)
    const int *__restrict__ in = J.in[blockIdx.y];
    int *__restrict__ out = J.out[blockIdx.y];
    int *__restrict__ tile_sums = J.tiles[blockIdx.y];
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

// One block per array scans its tile sums in chunks of 256 with a running carry.
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(ScanJobs J) {
    __shared__ int lds[kScanThreads / 64 + 1];
    const int n = J.n[blockIdx.x];
    const int ntiles = static_cast<int>((static_cast<int64_t>(n) + kScanTile - 1) / kScanTile);
    int *__restrict__ tile_sums = J.tiles[blockIdx.x];
    int *__restrict__ grand_total = J.out[blockIdx.x] + n;
    int *__restrict__ total_copy = J.total_copy[blockIdx.x];
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

__global__ __launch_bounds__(kScanThreads) void k_scan_add(ScanJobs J) {
    const int n = J.n[blockIdx.y];
    if (static_cast<int64_t>(blockIdx.x) * kScanTile >= n) return;
    int *__restrict__ out = J.out[blockIdx.y];
    const int *__restrict__ tile_sums = J.tiles[blockIdx.y];
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

__global__ __launch_bounds__(kSmallThreads) void k_scan_small(ScanJobs J) {
    __shared__ int wsum[kSmallWaves + 1];
    const int n = J.n[blockIdx.x];
    const int *__restrict__ in = J.in[blockIdx.x];
    int *__restrict__ out = J.out[blockIdx.x];
    int *__restrict__ total_copy = J.total_copy[blockIdx.x];
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

namespace {

// Jobs with n <= 0 just get out[0] = 0 (and their total copy); the others share launches.
void scan_jobs(ScanJobs J, int njobs, hipStream_t s) {
    ScanJobs K{};
    int nk = 0, nmax = 0;
    for (int k = 0; k < njobs; ++k) {
        if (J.n[k] <= 0) {
            NAIR_HIP(hipMemsetAsync(J.out[k], 0, sizeof(int), s));
            if (J.total_copy[k]) NAIR_HIP(hipMemsetAsync(J.total_copy[k], 0, sizeof(int), s));
            continue;
        }
        K.in[nk] = J.in[k];
        K.out[nk] = J.out[k];
        K.total_copy[nk] = J.total_copy[k];
        K.n[nk] = J.n[k];
        nmax = std::max(nmax, J.n[k]);
        ++nk;
    }
    if (nk == 0) return;
    if (nmax <= kSmallMax) {
        k_scan_small<<<nk, kSmallThreads, 0, s>>>(K);
        NAIR_HIP(hipGetLastError());
        return;
    }
    const int ntiles = static_cast<int>((static_cast<int64_t>(nmax) + kScanTile - 1) / kScanTile);
    DBuf<int> tiles(static_cast<size_t>(ntiles) * nk);
    for (int k = 0; k < nk; ++k) K.tiles[k] = tiles.get() + static_cast<int64_t>(k) * ntiles;
    const dim3 grid(static_cast<unsigned>(ntiles), static_cast<unsigned>(nk));
    k_scan_tiles<<<grid, kScanThreads, 0, s>>>(K);
    k_scan_tile_sums<<<nk, kScanThreads, 0, s>>>(K);
    k_scan_add<<<grid, kScanThreads, 0, s>>>(K);
    NAIR_HIP(hipGetLastError());
    // `tiles` returns to the pool now; any later user of that memory is ordered after
    // these kernels on the same stream (the library runs one call at a time).
}

}  // namespace

void scan_exclusive(const int *in, int *out, int n, hipStream_t s, int *total_copy) {
    ScanJobs J{};
    J.in[0] = in;
    J.out[0] = out;
    J.total_copy[0] = total_copy;
    J.n[0] = n;
    scan_jobs(J, 1, s);
}

void scan_exclusive2(const int *in0, int *out0, int n0, int *total0, const int *in1, int *out1, int n1, int *total1,
                     hipStream_t s) {
    ScanJobs J{};
    J.in[0] = in0;
    J.out[0] = out0;
    J.total_copy[0] = total0;
    J.n[0] = n0;
    J.in[1] = in1;
    J.out[1] = out1;
    J.total_copy[1] = total1;
    J.n[1] = n1;
    scan_jobs(J, 2, s);
}

}  // namespace nair
