// Transposes for the transposed cycle: A^T (blocks transposed), Z^T, and the
// inverse map of the one-point interpolation (rows of P^T).  Entries are placed
// by atomics and then each row is sorted by source index, so the result is
// deterministic.
#include "common.h"

namespace nair {
namespace {

__global__ __launch_bounds__(256) void k_count_cols(const int *__restrict__ colidx, int64_t nnz, int *__restrict__ cnt) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < nnz;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x)
        atomicAdd(&cnt[colidx[t]], 1);
}

__global__ __launch_bounds__(256) void k_transpose_fill(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                       int nrows, const int *__restrict__ trp, int *__restrict__ fill,
                                                       int *__restrict__ tcol, int *__restrict__ tsrc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nrows) return;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t];
        const int o = trp[J] + atomicAdd(&fill[J], 1);
        tcol[o] = I;
        tsrc[o] = t;
    }
}

// Sort each row's (col, src) pairs by col (insertion sort; rows are short).
__global__ __launch_bounds__(256) void k_sort_rows(const int *__restrict__ rp, int nrows, int *__restrict__ col,
                                                  int *__restrict__ src) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nrows) return;
    const int lo = rp[J], hi = rp[J + 1];
    for (int a = lo + 1; a < hi; ++a) {
        const int c = col[a], s = src ? src[a] : 0;
        int b = a - 1;
        while (b >= lo && col[b] > c) {
            col[b + 1] = col[b];
            if (src) src[b + 1] = src[b];
            --b;
        }
        col[b + 1] = c;
        if (src) src[b + 1] = s;
    }
}

// out[t][a][b] = A[src[t]][b][a]
__global__ __launch_bounds__(256) void k_gather_transposed(int64_t n, int bs, const double *__restrict__ A,
                                                          const int *__restrict__ src, double *__restrict__ out) {
    const int bb = bs * bs;
    const int64_t total = n * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bb;
        const int e = static_cast<int>(g - t * bb);
        const int a = e / bs, b = e - a * bs;
        out[g] = A[static_cast<int64_t>(src[t]) * bb + b * bs + a];
    }
}

__global__ __launch_bounds__(256) void k_count_pmap(const int *__restrict__ pmap, int nb, int *__restrict__ cnt) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nb && pmap[I] >= 0) atomicAdd(&cnt[pmap[I]], 1);
}

__global__ __launch_bounds__(256) void k_fill_pmap(const int *__restrict__ pmap, int nb, const int *__restrict__ rp,
                                                  int *__restrict__ fill, int *__restrict__ idx) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb || pmap[I] < 0) return;
    const int j = pmap[I];
    idx[rp[j] + atomicAdd(&fill[j], 1)] = I;
}

unsigned cap_grid(int64_t g) { return static_cast<unsigned>(g > 65536 * 16 ? 65536 * 16 : (g < 1 ? 1 : g)); }

}  // namespace

void bsr_transpose(const DevBSR &A, DevBSR &AT, hipStream_t s) {
    const int nrows_t = A.ncols;
    AT.nb = nrows_t;
    AT.ncols = A.nb;
    AT.bs = A.bs;
    AT.nnzb = A.nnzb;
    AT.rowptr.alloc(static_cast<size_t>(nrows_t) + 1);
    AT.colidx.alloc(A.nnzb);
    AT.vals.alloc(static_cast<size_t>(A.nnzb) * A.bs * A.bs);
    DBuf<int> cnt(nrows_t), fill(nrows_t), src(A.nnzb);
    NAIR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * (nrows_t ? nrows_t : 1), s));
    NAIR_HIP(hipMemsetAsync(fill.get(), 0, sizeof(int) * (nrows_t ? nrows_t : 1), s));
    if (A.nnzb > 0) k_count_cols<<<cap_grid((A.nnzb + 255) / 256), 256, 0, s>>>(A.colidx.get(), A.nnzb, cnt.get());
    scan_exclusive(cnt.get(), AT.rowptr.get(), nrows_t, s);
    if (A.nb > 0)
        k_transpose_fill<<<grid_for(A.nb, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.nb, AT.rowptr.get(),
                                                            fill.get(), AT.colidx.get(), src.get());
    if (nrows_t > 0)
        k_sort_rows<<<grid_for(nrows_t, 256), 256, 0, s>>>(AT.rowptr.get(), nrows_t, AT.colidx.get(), src.get());
    if (A.nnzb > 0)
        k_gather_transposed<<<cap_grid((A.nnzb * A.bs * A.bs + 255) / 256), 256, 0, s>>>(A.nnzb, A.bs, A.vals.get(),
                                                                                         src.get(), AT.vals.get());
    NAIR_HIP(hipGetLastError());
}

void pmap_transpose(const int *pmap, int nb, int nc, DBuf<int> &ptptr, DBuf<int> &ptidx, hipStream_t s) {
    DBuf<int> cnt(nc), fill(nc);
    NAIR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * (nc ? nc : 1), s));
    NAIR_HIP(hipMemsetAsync(fill.get(), 0, sizeof(int) * (nc ? nc : 1), s));
    ptptr.alloc(static_cast<size_t>(nc) + 1);
    k_count_pmap<<<grid_for(nb, 256), 256, 0, s>>>(pmap, nb, cnt.get());
    scan_exclusive(cnt.get(), ptptr.get(), nc, s);
    const int total = read_int(ptptr.get() + nc, s);
    ptidx.alloc(total);
    k_fill_pmap<<<grid_for(nb, 256), 256, 0, s>>>(pmap, nb, ptptr.get(), fill.get(), ptidx.get());
    if (nc > 0) k_sort_rows<<<grid_for(nc, 256), 256, 0, s>>>(ptptr.get(), nc, ptidx.get(), nullptr);
    NAIR_HIP(hipGetLastError());
}

}  // namespace nair
