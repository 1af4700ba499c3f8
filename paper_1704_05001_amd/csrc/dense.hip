// Coarsest level: dense operator, its inverse by Gauss-Jordan elimination with
// partial pivoting in one 1024-thread workgroup (in LDS up to 128 unknowns,
// in global memory beyond, up to a few thousand), the inverse's transpose for
// the transposed cycle, and the dense matrix-vector product (wave per row).
#include "common.h"

namespace nair {
namespace {

constexpr int kGJThreads = 1024;

__global__ __launch_bounds__(256) void k_bsr_to_dense(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                     const double *__restrict__ vals, int nb, int bs,
                                                     double *__restrict__ M, int n) {
    const int I = blockIdx.x;
    if (I >= nb) return;
    const int bb = bs * bs;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t];
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            const int a = e / bs, b = e - a * bs;
            M[static_cast<int64_t>(I * bs + a) * n + J * bs + b] = vals[static_cast<int64_t>(t) * bb + e];
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

__global__ __launch_bounds__(kGJThreads) void k_gauss_jordan_lds(const double *__restrict__ Min,
                                                                double *__restrict__ inv, int n,
                                                                int *__restrict__ singular) {
    extern __shared__ double a[];
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
                                                        int n) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(n) * n) return;
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    MT[static_cast<int64_t>(j) * n + i] = M[e];
}

}  // namespace

bool dense_inverse_from_bsr(const DevBSR &A, double *inv, double *invT, hipStream_t s) {
    const int n = A.nb * A.bs;
    DBuf<double> M(static_cast<size_t>(n) * n);
    DBuf<int> sing(1);
    NAIR_HIP(hipMemsetAsync(M.get(), 0, sizeof(double) * static_cast<size_t>(n) * n, s));
    NAIR_HIP(hipMemsetAsync(sing.get(), 0, sizeof(int), s));
    k_bsr_to_dense<<<A.nb, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.vals.get(), A.nb, A.bs, M.get(), n);
    NAIR_HIP(hipGetLastError());
    bool done = false;
    if (n <= kLdsOrder) {
        const size_t lds = sizeof(double) * static_cast<size_t>(n) * n;
        static bool attr_set = false;
        if (!attr_set) {
            // allow up to kLdsOrder^2 doubles (128 KiB) of dynamic LDS
            if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_gauss_jordan_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(sizeof(double) * kLdsOrder * kLdsOrder)) != hipSuccess)
                (void)hipGetLastError();
            attr_set = true;
        }
        k_gauss_jordan_lds<<<1, kGJThreads, lds, s>>>(M.get(), inv, n, sing.get());
        done = hipGetLastError() == hipSuccess;
    }
    if (!done) {
        DBuf<double> colk(n);
        k_gauss_jordan<<<1, kGJThreads, 0, s>>>(M.get(), inv, n, colk.get(), sing.get());
        NAIR_HIP(hipGetLastError());
        if (read_int(sing.get(), s) != 0) return false;
    } else if (read_int(sing.get(), s) != 0) {
        return false;
    }
    k_transpose_dense<<<grid_for(static_cast<int64_t>(n) * n, 256), 256, 0, s>>>(inv, invT, n);
    NAIR_HIP(hipGetLastError());
    return true;
}

}  // namespace nair
