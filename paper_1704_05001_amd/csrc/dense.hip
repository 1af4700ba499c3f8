// Direct solves on the coarsest level of each system: the dense operator of a
// system's block rows, its inverse by Gauss-Jordan elimination with partial
// pivoting in one 1024-thread workgroup per system (in LDS up to 128 unknowns,
// in global memory beyond, up to a few thousand), and the inverse's transpose
// for the transposed cycle.  A batched hierarchy holds many such systems
// ("segments": a contiguous range of block rows each) on one level.
#include <algorithm>
#include <vector>

#include "common.h"

namespace nair {
namespace {

constexpr int kGJThreads = 1024;

// Segment k = blockIdx.y: block row blk0[k] + blockIdx.x into the dense n x n
// matrix at M + off[k] (n = nbk[k] * bs, columns relative to blk0[k]).
__global__ __launch_bounds__(256) void k_bsr_to_dense(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                     const double *__restrict__ vals, int bs,
                                                     const int *__restrict__ blk0, const int *__restrict__ nbk,
                                                     const int64_t *__restrict__ off, double *__restrict__ M) {
    const int k = blockIdx.y;
    const int i = blockIdx.x;
    if (i >= nbk[k]) return;
    const int b0 = blk0[k];
    const int I = b0 + i;
    const int n = nbk[k] * bs;
    const int bb = bs * bs;
    double *Mk = M + off[k];
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t] - b0;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            const int a = e / bs, b = e - a * bs;
            Mk[static_cast<int64_t>(i * bs + a) * n + J * bs + b] = vals[static_cast<int64_t>(t) * bb + e];
        }
    }
}

__global__ __launch_bounds__(kGJThreads) void k_gauss_jordan(double *__restrict__ M, double *__restrict__ Inv, int n,
                                                            double *__restrict__ colk, int *__restrict__ singular) {
    __shared__ double rv[kGJThreads];
    __shared__ int ri[kGJThreads];
    const int tid = threadIdx.x;
    const int64_t nn = static_cast<int64_t>(n) * n;
    for (int64_t e = tid; e < nn; e += kGJThreads) Inv[e] = (e / n == e % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        double v = -1.0;
        int idx = n;
        for (int i = k + tid; i < n; i += kGJThreads) {
            const double av = fabs(M[static_cast<int64_t>(i) * n + k]);
            if (av > v || (av == v && i < idx)) {
                v = av;
                idx = i;
            }
        }
        rv[tid] = v;
        ri[tid] = idx;
        __syncthreads();
        for (int s = kGJThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                const double ov = rv[tid + s];
                const int oi = ri[tid + s];
                if (ov > rv[tid] || (ov == rv[tid] && oi < ri[tid])) {
                    rv[tid] = ov;
                    ri[tid] = oi;
                }
            }
            __syncthreads();
        }
        const double best = rv[0];
        const int p = ri[0];
        __syncthreads();
        if (!(best > 0.0)) {
            if (tid == 0) *singular = 1;
            return;
        }
        if (p != k) {
            for (int j = tid; j < n; j += kGJThreads) {
                double t = M[static_cast<int64_t>(k) * n + j];
                M[static_cast<int64_t>(k) * n + j] = M[static_cast<int64_t>(p) * n + j];
                M[static_cast<int64_t>(p) * n + j] = t;
                t = Inv[static_cast<int64_t>(k) * n + j];
                Inv[static_cast<int64_t>(k) * n + j] = Inv[static_cast<int64_t>(p) * n + j];
                Inv[static_cast<int64_t>(p) * n + j] = t;
            }
        }
        __syncthreads();
        const double piv = M[static_cast<int64_t>(k) * n + k];
        __syncthreads();
        for (int j = tid; j < n; j += kGJThreads) {
            M[static_cast<int64_t>(k) * n + j] /= piv;
            Inv[static_cast<int64_t>(k) * n + j] /= piv;
        }
        __syncthreads();
        for (int i = tid; i < n; i += kGJThreads) colk[i] = M[static_cast<int64_t>(i) * n + k];
        __syncthreads();
        for (int64_t e = tid; e < nn; e += kGJThreads) {
            const int i = static_cast<int>(e / n);
            if (i == k) continue;
            const int j = static_cast<int>(e - static_cast<int64_t>(i) * n);
            const double f = colk[i];
            if (f == 0.0) continue;
            if (j > k) M[e] -= f * M[static_cast<int64_t>(k) * n + j];
            Inv[e] -= f * Inv[static_cast<int64_t>(k) * n + j];
        }
        __syncthreads();
    }
}

// In-place Gauss-Jordan inversion with partial pivoting, the whole matrix in
// LDS (n <= kLdsOrder): row k is scaled by its pivot with a_kk replaced by 1,
// every other row i eliminates with a_ik replaced by 0; the row exchanges are
// undone as column exchanges in reverse order at the end.
constexpr int kLdsOrder = 128;

// One workgroup per listed segment k = sel[blockIdx.x]: the n x n matrix at
// Min + off[k] (n = nbk[k] * bs) inverted into inv + off[k].
__global__ __launch_bounds__(kGJThreads) void k_gauss_jordan_lds(const double *__restrict__ Mall,
                                                                double *__restrict__ invall,
                                                                const int *__restrict__ sel,
                                                                const int *__restrict__ nbk, int bs,
                                                                const int64_t *__restrict__ off,
                                                                int *__restrict__ singular_all) {
    extern __shared__ double a[];
    const int seg = sel[blockIdx.x];
    const int n = nbk[seg] * bs;
    const double *Min = Mall + off[seg];
    double *inv = invall + off[seg];
    int *singular = singular_all + seg;
    __shared__ double colk[kLdsOrder];
    __shared__ int perm[kLdsOrder];
    __shared__ int piv_row;
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int nn = n * n;
    for (int e = tid; e < nn; e += kGJThreads) a[e] = Min[e];
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            double v = -1.0;
            int idx = n;
            for (int i = k + tid; i < n; i += 64) {
                const double av = fabs(a[i * n + k]);
                if (av > v || (av == v && i < idx)) {
                    v = av;
                    idx = i;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(v, o, 64);
                const int oi = __shfl_xor(idx, o, 64);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (tid == 0) {
                piv_row = idx;
                perm[k] = idx;
                if (!(v > 0.0)) bad = 1;
            }
        }
        __syncthreads();
        if (bad) {
            if (tid == 0) *singular = 1;
            return;
        }
        const int p = piv_row;
        if (p != k)
            for (int j = tid; j < n; j += kGJThreads) {
                const double t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
        __syncthreads();
        const double piv = a[k * n + k];
        __syncthreads();
        for (int j = tid; j < n; j += kGJThreads) a[k * n + j] = ((j == k) ? 1.0 : a[k * n + j]) / piv;
        for (int i = tid; i < n; i += kGJThreads) colk[i] = a[i * n + k];
        __syncthreads();
        for (int e = tid; e < nn; e += kGJThreads) {
            const int i = e / n;
            if (i == k) continue;
            const int j = e - i * n;
            const double f = colk[i];
            a[e] = ((j == k) ? 0.0 : a[e]) - f * a[k * n + j];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k)
            for (int i = tid; i < n; i += kGJThreads) {
                const double t = a[i * n + k];
                a[i * n + k] = a[i * n + p];
                a[i * n + p] = t;
            }
        __syncthreads();
    }
    for (int e = tid; e < nn; e += kGJThreads) inv[e] = a[e];
}

__global__ __launch_bounds__(256) void k_transpose_dense(const double *__restrict__ M, double *__restrict__ MT,
                                                        const int *__restrict__ nbk, int bs,
                                                        const int64_t *__restrict__ off) {
    const int k = blockIdx.y;
    const int n = nbk[k] * bs;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(n) * n) return;
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    MT[off[k] + static_cast<int64_t>(j) * n + i] = M[off[k] + e];
}

}  // namespace

int dense_inverse_segments(const DevBSR &A, int nseg, const int *blk0_h, const int *nbk_h, const int64_t *off_h,
                           double *inv, double *invT, hipStream_t s) {
    if (nseg <= 0) return -1;
    const int bs = A.bs;
    int max_nb = 0;
    for (int k = 0; k < nseg; ++k) max_nb = std::max(max_nb, nbk_h[k]);
    const int64_t last_n = static_cast<int64_t>(nbk_h[nseg - 1]) * bs;
    const int64_t total = off_h[nseg - 1] + last_n * last_n;
    const int64_t max_n = static_cast<int64_t>(max_nb) * bs;
    // dynamic LDS beyond 64 KiB (up to kLdsOrder^2 doubles) needs the attribute;
    // without it every segment takes the global-memory elimination
    static int lds_ok = -1;
    if (lds_ok < 0) {
        lds_ok = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gauss_jordan_lds),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(sizeof(double) * kLdsOrder * kLdsOrder)) == hipSuccess;
        if (!lds_ok) (void)hipGetLastError();
    }
    std::vector<int> sel_lds, sel_big;
    for (int k = 0; k < nseg; ++k)
        (lds_ok && static_cast<int64_t>(nbk_h[k]) * bs <= kLdsOrder ? sel_lds : sel_big).push_back(k);
    DBuf<double> M(static_cast<size_t>(total));
    DBuf<int> blk0(nseg), nbk(nseg), sing(nseg), sel(sel_lds.empty() ? 1 : sel_lds.size());
    DBuf<int64_t> off(nseg);
    NAIR_HIP(hipMemsetAsync(M.get(), 0, sizeof(double) * static_cast<size_t>(total), s));
    NAIR_HIP(hipMemsetAsync(sing.get(), 0, sizeof(int) * nseg, s));
    NAIR_HIP(hipMemcpyAsync(blk0.get(), blk0_h, sizeof(int) * nseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(nbk.get(), nbk_h, sizeof(int) * nseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(off.get(), off_h, sizeof(int64_t) * nseg, hipMemcpyHostToDevice, s));
    if (!sel_lds.empty())
        NAIR_HIP(hipMemcpyAsync(sel.get(), sel_lds.data(), sizeof(int) * sel_lds.size(), hipMemcpyHostToDevice, s));
    k_bsr_to_dense<<<dim3(static_cast<unsigned>(max_nb), static_cast<unsigned>(nseg)), 256, 0, s>>>(
        A.rowptr.get(), A.colidx.get(), A.vals.get(), bs, blk0.get(), nbk.get(), off.get(), M.get());
    NAIR_HIP(hipGetLastError());
    if (!sel_lds.empty()) {
        int lds_n = 0;
        for (int k : sel_lds) lds_n = std::max(lds_n, nbk_h[k] * bs);
        const size_t lds = sizeof(double) * static_cast<size_t>(lds_n) * lds_n;
        k_gauss_jordan_lds<<<static_cast<unsigned>(sel_lds.size()), kGJThreads, lds, s>>>(
            M.get(), inv, sel.get(), nbk.get(), bs, off.get(), sing.get());
        NAIR_HIP(hipGetLastError());
    }
    if (!sel_big.empty()) {
        DBuf<double> colk(static_cast<size_t>(max_n));
        for (int k : sel_big) {
            const int n = nbk_h[k] * bs;
            k_gauss_jordan<<<1, kGJThreads, 0, s>>>(M.get() + off_h[k], inv + off_h[k], n, colk.get(), sing.get() + k);
            NAIR_HIP(hipGetLastError());
        }
    }
    std::vector<int> hs(nseg);
    read_ints(sing.get(), hs.data(), nseg, s);
    for (int k = 0; k < nseg; ++k)
        if (hs[k] != 0) return k;
    k_transpose_dense<<<dim3(grid_for(max_n * max_n, 256), static_cast<unsigned>(nseg)), 256, 0, s>>>(
        inv, invT, nbk.get(), bs, off.get());
    NAIR_HIP(hipGetLastError());
    NAIR_HIP(hipStreamSynchronize(s));   // the host arrays and temporaries end here
    return -1;
}

}  // namespace nair
