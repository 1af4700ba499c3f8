// Vector kernels of restarted GMRES: several dot products of one vector
// against a block of basis vectors, the matching multi-axpy, and the
// normalisation by a device-side norm.  The Arnoldi step orthogonalises with
// classical Gram-Schmidt applied twice, so each pass is one wide reduction
// and one wide update instead of a dot and an axpy per basis vector.
#include <algorithm>

#include "common.h"

namespace nair {
namespace {

constexpr int kDotThreads = 256;
constexpr int kDotPer = 8;                               // elements per thread
constexpr int64_t kDotChunk = kDotThreads * kDotPer;     // elements per workgroup
constexpr int kDotVec = 4;                               // basis vectors per pass
constexpr int kDotWaves = kDotThreads / 64;

// part[i * nblk + blk] = sum over the chunk blk of V_i * w.  Each thread keeps
// its 8 elements of w in registers and streams kDotVec basis vectors per pass.
__global__ __launch_bounds__(kDotThreads) void k_mdot(const double *__restrict__ V, int64_t ld, int nv,
                                                     const double *__restrict__ w, int64_t n,
                                                     double *__restrict__ part, int64_t nblk) {
    __shared__ double red[kDotVec][kDotWaves];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kDotChunk + threadIdx.x;
    double wv[kDotPer];
#pragma unroll
    for (int q = 0; q < kDotPer; ++q) {
        const int64_t idx = base + static_cast<int64_t>(q) * kDotThreads;
        wv[q] = idx < n ? w[idx] : 0.0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i0 = 0; i0 < nv; i0 += kDotVec) {
        double acc[kDotVec];
#pragma unroll
        for (int v = 0; v < kDotVec; ++v) {
            acc[v] = 0.0;
            if (i0 + v < nv) {
                const double *Vi = V + static_cast<int64_t>(i0 + v) * ld;
#pragma unroll
                for (int q = 0; q < kDotPer; ++q) {
                    const int64_t idx = base + static_cast<int64_t>(q) * kDotThreads;
                    if (idx < n) acc[v] = fma(wv[q], Vi[idx], acc[v]);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < kDotVec; ++v)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o, 64);
        __syncthreads();   // the previous pass has read red
        if (lane == 0)
#pragma unroll
            for (int v = 0; v < kDotVec; ++v) red[v][wave] = acc[v];
        __syncthreads();
        if (threadIdx.x < kDotVec && i0 + static_cast<int>(threadIdx.x) < nv) {
            const int v = threadIdx.x;
            double sum = red[v][0];
#pragma unroll
            for (int k = 1; k < kDotWaves; ++k) sum += red[v][k];
            part[static_cast<int64_t>(i0 + v) * nblk + blockIdx.x] = sum;
        }
    }
}

// out[i] = sum_b part[i * nblk + b]: one wave per basis vector, fixed order.
__global__ __launch_bounds__(64) void k_mdot_finish(const double *__restrict__ part, int64_t nblk,
                                                   double *__restrict__ out) {
    const int i = blockIdx.x;
    const double *p = part + static_cast<int64_t>(i) * nblk;
    double sum = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += 64) sum += p[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (threadIdx.x == 0) out[i] = sum;
}

// w_k -= c_i V_i,k for i = 0, 1, ..., nv-1 (one rounding per term).
__global__ __launch_bounds__(256) void k_maxpy(const double *__restrict__ V, int64_t ld, int nv,
                                              const double *__restrict__ c, double *__restrict__ w, int64_t n) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double acc = w[k];
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
        const double v0 = V[static_cast<int64_t>(i) * ld + k];
        const double v1 = V[static_cast<int64_t>(i + 1) * ld + k];
        const double v2 = V[static_cast<int64_t>(i + 2) * ld + k];
        const double v3 = V[static_cast<int64_t>(i + 3) * ld + k];
        acc = fma(-c[i], v0, acc);
        acc = fma(-c[i + 1], v1, acc);
        acc = fma(-c[i + 2], v2, acc);
        acc = fma(-c[i + 3], v3, acc);
    }
    for (; i < nv; ++i) acc = fma(-c[i], V[static_cast<int64_t>(i) * ld + k], acc);
    w[k] = acc;
}

__global__ __launch_bounds__(256) void k_unit(const double *__restrict__ w, const double *__restrict__ ss,
                                             double *__restrict__ v, int64_t n) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    v[k] = w[k] / sqrt(ss[0]);
}

unsigned grid_of(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

}  // namespace

int64_t mdot_parts(int64_t n) { return std::max<int64_t>(1, (n + kDotChunk - 1) / kDotChunk); }

void launch_mdot(const double *V, int64_t ld, int nv, const double *w, int64_t n, double *part, double *out,
                 hipStream_t s) {
    if (nv <= 0) return;
    const int64_t nblk = mdot_parts(n);
    k_mdot<<<static_cast<unsigned>(nblk), kDotThreads, 0, s>>>(V, ld, nv, w, n, part, nblk);
    NAIR_HIP(hipGetLastError());
    k_mdot_finish<<<static_cast<unsigned>(nv), 64, 0, s>>>(part, nblk, out);
    NAIR_HIP(hipGetLastError());
}

void launch_maxpy(const double *V, int64_t ld, int nv, const double *c, double *w, int64_t n, hipStream_t s) {
    if (nv <= 0 || n <= 0) return;
    k_maxpy<<<grid_of(n, 256), 256, 0, s>>>(V, ld, nv, c, w, n);
    NAIR_HIP(hipGetLastError());
}

void launch_unit(const double *w, const double *ss, double *v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_unit<<<grid_of(n, 256), 256, 0, s>>>(w, ss, v, n);
    NAIR_HIP(hipGetLastError());
}

}  // namespace nair
