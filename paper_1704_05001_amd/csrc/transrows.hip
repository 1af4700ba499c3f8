// Transposed row-block copies for the transposed cycle (TransRows, common.h):
// the blocks of selected rows of an operator, listed by block column and
// stored by their nonzero rows.  The pattern is placed by atomics and each
// output row then sorted by source row, so the result is deterministic; the
// values are a RowBlocks copy of the source blocks in that order.
#include <climits>

#include "common.h"

namespace nair {
namespace {

__global__ __launch_bounds__(256) void k_tr_count(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                 int nrows, const int8_t *__restrict__ cf, int keep_cf,
                                                 int *__restrict__ cnt) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nrows || (cf && cf[J] != keep_cf)) return;
    for (int t = rowptr[J]; t < rowptr[J + 1]; ++t) atomicAdd(&cnt[colidx[t]], 1);
}

__global__ __launch_bounds__(256) void k_tr_fill(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                int nrows, const int8_t *__restrict__ cf, int keep_cf,
                                                const int *__restrict__ trp, int *__restrict__ fill,
                                                int *__restrict__ tcol, int *__restrict__ tsrc) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nrows || (cf && cf[J] != keep_cf)) return;
    for (int t = rowptr[J]; t < rowptr[J + 1]; ++t) {
        const int I = colidx[t];
        const int o = trp[I] + atomicAdd(&fill[I], 1);
        tcol[o] = J;
        tsrc[o] = t;
    }
}

// Each output row's (source row, source block) pairs in ascending source row
// (insertion sort: rows are short).
__global__ __launch_bounds__(256) void k_tr_sort(const int *__restrict__ trp, int nrows, int *__restrict__ tcol,
                                                int *__restrict__ tsrc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nrows) return;
    const int lo = trp[I], hi = trp[I + 1];
    for (int a = lo + 1; a < hi; ++a) {
        const int c = tcol[a], sidx = tsrc[a];
        int b = a - 1;
        while (b >= lo && tcol[b] > c) {
            tcol[b + 1] = tcol[b];
            tsrc[b + 1] = tsrc[b];
            --b;
        }
        tcol[b + 1] = c;
        tsrc[b + 1] = sidx;
    }
}

// The flat walk: src of each stored row (one thread per entry) ...
__global__ __launch_bounds__(256) void k_tr_src(const int *__restrict__ colidx, const uint32_t *__restrict__ mask,
                                               const int *__restrict__ off, int64_t nent, int bs,
                                               int *__restrict__ src) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nent) return;
    const int base = colidx[t] * bs;
    int q = off[t] / bs;
    for (uint32_t m = mask[t]; m != 0u; m &= m - 1u) src[q++] = base + __ffs(static_cast<int>(m)) - 1;
}

// ... and each output row's first stored row
__global__ __launch_bounds__(256) void k_tr_qptr(const int *__restrict__ rowptr, const int *__restrict__ off, int nrows,
                                                int bs, int *__restrict__ qptr) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I <= nrows) qptr[I] = off[rowptr[I]] / bs;
}

}  // namespace

bool build_trans_rows(const DevBSR &M, const int8_t *cf, int keep_cf, const uint32_t *mmask, TransRows &T,
                      hipStream_t s) {
    T = TransRows();
    const int bs = M.bs;
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    const int nout = M.ncols;
    if (M.nnzb < 0) fail(NAIR_EDEVICE, "build_trans_rows: block count not known");
    if (bs < 1 || bs > 32 || static_cast<int64_t>(M.nnzb) * bb > INT_MAX) return false;
    T.nrows = nout;
    T.rowptr.alloc(static_cast<size_t>(nout) + 1);
    DBuf<int> cnt(static_cast<size_t>(std::max(nout, 1)));
    NAIR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * static_cast<size_t>(std::max(nout, 1)), s));
    if (M.nb > 0)
        k_tr_count<<<grid_for(M.nb, 256), 256, 0, s>>>(M.rowptr.get(), M.colidx.get(), M.nb, cf, keep_cf, cnt.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), T.rowptr.get(), nout, s);
    const int nent = read_int(T.rowptr.get() + nout, s);
    T.nent = nent;
    T.colidx.alloc(static_cast<size_t>(std::max(nent, 1)));
    DBuf<int> tsrc(static_cast<size_t>(std::max(nent, 1)));
    if (nent > 0) {
        NAIR_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int) * static_cast<size_t>(nout), s));
        k_tr_fill<<<grid_for(M.nb, 256), 256, 0, s>>>(M.rowptr.get(), M.colidx.get(), M.nb, cf, keep_cf,
                                                      T.rowptr.get(), cnt.get(), T.colidx.get(), tsrc.get());
        k_tr_sort<<<grid_for(nout, 256), 256, 0, s>>>(T.rowptr.get(), nout, T.colidx.get(), tsrc.get());
        NAIR_HIP(hipGetLastError());
        // the source blocks' nonzero-row masks: given, or found from the values
        DBuf<uint32_t> own;
        const uint32_t *masks = mmask;
        if (!masks) {
            own.alloc(static_cast<size_t>(M.nnzb));
            launch_block_scan(M.vals.get(), M.nnzb, bs, nullptr, nullptr, nullptr, nullptr, own.get(), nullptr, s);
            masks = own.get();
        }
        RowBlocks R;
        if (!build_row_blocks(M.vals.get(), nent, bs, R, s, tsrc.get(), nullptr, masks)) return false;
        T.mask = std::move(R.mask);
        T.off = std::move(R.off);
        T.vals = std::move(R.vals);
    }
    // the flat walk over stored rows
    T.qptr.alloc(static_cast<size_t>(nout) + 1);
    if (nent > 0) {
        T.nq = read_int(T.off.get() + nent, s) / bs;
        T.src.alloc(static_cast<size_t>(std::max<int64_t>(T.nq, 1)));
        k_tr_src<<<grid_for(nent, 256), 256, 0, s>>>(T.colidx.get(), T.mask.get(), T.off.get(), nent, bs, T.src.get());
        k_tr_qptr<<<grid_for(static_cast<int64_t>(nout) + 1, 256), 256, 0, s>>>(T.rowptr.get(), T.off.get(), nout, bs,
                                                                               T.qptr.get());
        NAIR_HIP(hipGetLastError());
    } else {
        NAIR_HIP(hipMemsetAsync(T.qptr.get(), 0, sizeof(int) * (static_cast<size_t>(nout) + 1), s));
    }
    T.on = true;
    return true;
}

void trans_rows_to_float(TransRows &T, int bs, hipStream_t s) {
    if (!T.on || T.vals32.get() || T.nent == 0) return;
    const int64_t nv = T.nent * bs * bs;
    T.vals32.alloc(static_cast<size_t>(nv));
    launch_to_float(T.vals.get(), T.vals32.get(), nv, s, T.off.get() + T.nent);   // the rows kept: off[nent] entries
}

}  // namespace nair
