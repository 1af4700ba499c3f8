// Sweep copies: the F rows of a level operator (or its transpose) in F-list
// order, each without its diagonal block, with D_F^{-1} in the same order
// (SweepCopy).  A Jacobi F sweep then streams its matrix entries, column
// indices and inverse blocks contiguously instead of picking F rows out from
// between the C rows.  Built once per level and direction: an exact count of
// every row's off-diagonal blocks, a scan, and one wave per row copying its
// column indices, blocks (or face masks and rectangles) and D^{-1} block with
// consecutive lanes on consecutive words.  Nothing is read back to the host.
#include <algorithm>
#include <climits>

#include "common.h"

namespace nair {
namespace {

__global__ __launch_bounds__(256) void k_sweep_count(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                    const int *__restrict__ flist, int nF, int *__restrict__ cnt) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    const int I = flist[f];
    int c = 0;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) c += colidx[t] != I ? 1 : 0;
    cnt[f] = c;
}

// One wave per F row f (I = flist[f]): blocks of A's row I other than the
// diagonal go to positions orp[f] ... in order: their column indices, and
// with FACE the face copy's masks and rc-word rectangles, else the source
// block index (osrc) for the row-compressed copy made next; D_I^{-1} goes to
// position f with the coefficient of input c for output a at c * bb/bs + a
// (dtrans: D_I^{-1} transposed; else as it is, for the sweeps that apply
// D^{-T}).  Nothing is written at or past cap.
template <bool FACE>
__global__ __launch_bounds__(256) void k_sweep_fill(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                   const double *__restrict__ src, const uint64_t *__restrict__ fmeta,
                                                   const double *__restrict__ dinv, const int *__restrict__ flist,
                                                   int nF, int w, int bs, bool dtrans, int64_t cap,
                                                   const int *__restrict__ orp,
                                                   int *__restrict__ ocol, uint64_t *__restrict__ ometa,
                                                   double *__restrict__ ovals, int *__restrict__ osrc,
                                                   double *__restrict__ odinv) {
    const int lane = threadIdx.x & 63;
    const int f = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
    if (f >= nF) return;   // whole waves
    const int bb = bs * bs;
    const int I = flist[f];
    const int lo = rowptr[I], hi = rowptr[I + 1];
    const int o = orp[f];
    // the diagonal block's position (hi if the row has none)
    int dp = hi;
    for (int base = lo; base < hi; base += 64) {
        const int t = base + lane;
        const unsigned long long b = __ballot(t < hi && colidx[t] == I);
        if (b != 0ull) {
            dp = base + __builtin_ctzll(b);
            break;
        }
    }
    const int n = hi - lo;
    for (int k = lane; k < n; k += 64) {
        const int t = lo + k;
        const int64_t d = static_cast<int64_t>(o) + k - (t > dp ? 1 : 0);
        if (t == dp || d >= cap) continue;
        ocol[d] = colidx[t];
        if constexpr (FACE) ometa[d] = fmeta[t];
        else osrc[d] = t;
    }
    if constexpr (FACE) {
        const int64_t total = static_cast<int64_t>(n) * w;
        for (int64_t e = lane; e < total; e += 64) {
            const int k = static_cast<int>(e / w);
            const int64_t q = e - static_cast<int64_t>(k) * w;
            const int t = lo + k;
            const int64_t d = static_cast<int64_t>(o) + k - (t > dp ? 1 : 0);
            if (t == dp || d >= cap) continue;
            ovals[d * w + q] = src[static_cast<int64_t>(t) * w + q];
        }
    }
    const double *Di = dinv + static_cast<int64_t>(I) * bb;
    double *Do = odinv + static_cast<int64_t>(f) * bb;
    // every load of the inverse first (bs <= 32: at most 16 words per lane; words past
    // the block repeat its last, unused), then the stores
    constexpr int kChunks = 16;
    double v[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int e = lane + 64 * i < bb ? lane + 64 * i : bb - 1;
        const int c = e / bs, a = e - c * bs;   // output position: input c, output a
        v[i] = Di[dtrans ? a * bs + c : e];
    }
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int e = lane + 64 * i;
        if (e < bb) Do[e] = v[i];
    }
}

// mask[t] = masks[src[t]] (src null: masks[t]) and size[t] for t < count (past it empty).
__global__ __launch_bounds__(256) void k_rb_take(const uint32_t *__restrict__ masks, int64_t n, int bs,
                                                const int *__restrict__ src, const int *__restrict__ count,
                                                uint32_t *__restrict__ mask, int *__restrict__ size) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t m = t < (count ? *count : n) ? masks[src ? src[t] : t] : 0u;
    mask[t] = m;
    size[t] = __popc(m) * bs;
}

// Block t's nonzero rows, in order, to out[off[t] ...]: one wave per block
// (four per workgroup), lane q of the stored entries taking entry c of the
// block's (q / bs)-th nonzero row, so consecutive lanes read consecutive
// words of a row and write consecutive words of the copy.
__global__ __launch_bounds__(256) void k_rb_fill(const double *__restrict__ vals, int64_t n, int bs,
                                                const int *__restrict__ src, const int *__restrict__ count,
                                                const uint32_t *__restrict__ mask, const int *__restrict__ off,
                                                double *__restrict__ out) {
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    const int lane = threadIdx.x & 63;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= (count ? *count : n)) return;
    const uint32_t m = mask[t];
    const int stored = __popc(m) * bs;
    const double *blk = vals + (src ? src[t] : t) * bb;
    double *o = out + off[t];
    // every load first, then the stores (at most bs * bs <= 1024 entries: 16 per lane)
    constexpr int kChunks = 16;
    double v[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int q = lane + 64 * i;
        v[i] = 0.0;
        if (q < stored) {
            const int k = q / bs, c = q - k * bs;
            uint32_t mm = m;
            for (int j = 0; j < k; ++j) mm &= mm - 1u;   // drop the k lower nonzero rows
            const int a = __ffs(static_cast<int>(mm)) - 1;
            v[i] = blk[a * bs + c];
        }
    }
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int q = lane + 64 * i;
        if (q < stored) o[q] = v[i];
    }
}

}  // namespace

bool build_row_blocks(const double *vals, int64_t n, int bs, RowBlocks &R, hipStream_t s, const int *src,
                      const int *count, const uint32_t *masks) {
    R = RowBlocks();
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    if (n <= 0 || bs < 1 || bs > 32 || n * bb > INT_MAX) return false;
    R.mask.alloc(static_cast<size_t>(n));
    R.off.alloc(static_cast<size_t>(n) + 1);
    R.vals.alloc(static_cast<size_t>(n * bb));   // (the rows kept take less; the total is not read back)
    DBuf<int> size(static_cast<size_t>(n));
    if (masks) {   // the blocks' row masks are known: no pass over their entries
        k_rb_take<<<grid_for(n, 256), 256, 0, s>>>(masks, n, bs, src, count, R.mask.get(), size.get());
        NAIR_HIP(hipGetLastError());
    } else {   // mask[t] and size[t] = nonzero rows * bs of block src[t] (t < count; past it empty)
        launch_block_scan(vals, n, bs, src, count, nullptr, nullptr, R.mask.get(), size.get(), s);
    }
    scan_exclusive(size.get(), R.off.get(), static_cast<int>(n), s);
    k_rb_fill<<<grid_for(n, 4), 256, 0, s>>>(vals, n, bs, src, count, R.mask.get(), R.off.get(), R.vals.get());
    NAIR_HIP(hipGetLastError());
    R.on = true;
    return true;
}

void row_blocks_to_float(RowBlocks &R, int64_t n, int bs, hipStream_t s) {
    if (!R.on || R.vals32.get()) return;
    const int64_t nv = n * bs * bs;
    R.vals32.alloc(static_cast<size_t>(nv));
    launch_to_float(R.vals.get(), R.vals32.get(), nv, s, R.off.get() + n);   // the rows kept: off[n] entries
}

void build_sweep(const DevBSR &A, const FaceCopy &F, const double *dinv, const int *flist, int nF, SweepCopy &S,
                 hipStream_t s, bool trans, const uint32_t *amask) {
    S = SweepCopy();
    if (nF <= 0 || A.nb == 0 || !dinv || !flist) return;
    const int bs = A.bs;
    const int bb = bs * bs;
    const bool face = F.on;
    const int w = face ? F.rc : bb;
    S.nF = nF;
    S.rc = face ? F.rc : 0;
    S.cmax = face ? F.cmax : 0;
    // every row of a level operator holds its diagonal block, so the F rows
    // hold at most nnzb - nF others
    S.cap = std::max<int64_t>(A.nnzb - nF, 1);
    S.rowptr.alloc(static_cast<size_t>(nF) + 1);
    S.colidx.alloc(static_cast<size_t>(S.cap));
    if (face) {
        S.vals.alloc(static_cast<size_t>(S.cap) * w);
        S.meta.alloc(static_cast<size_t>(S.cap));
    }
    S.dinv.alloc(static_cast<size_t>(nF) * bb);
    DBuf<int> cnt(static_cast<size_t>(nF));
    k_sweep_count<<<grid_for(nF, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), flist, nF, cnt.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), S.rowptr.get(), nF, s);
    const unsigned grid = static_cast<unsigned>((nF + 3) / 4);
    if (face) {
        k_sweep_fill<true><<<grid, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), F.vals.get(), F.meta.get(), dinv,
                                                flist, nF, w, bs, !trans, S.cap, S.rowptr.get(), S.colidx.get(),
                                                S.meta.get(), S.vals.get(), nullptr, S.dinv.get());
        NAIR_HIP(hipGetLastError());
    } else {
        DBuf<int> src(static_cast<size_t>(S.cap));
        k_sweep_fill<false><<<grid, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), nullptr, nullptr, dinv, flist, nF,
                                                 w, bs, !trans, S.cap, S.rowptr.get(), S.colidx.get(), nullptr,
                                                 nullptr, src.get(), S.dinv.get());
        NAIR_HIP(hipGetLastError());
        if (!build_row_blocks(A.vals.get(), S.cap, bs, S.rows, s, src.get(), S.rowptr.get() + nF, amask)) return;
    }
    S.on = true;
}

void sweep_to_float(SweepCopy &S, int bs, hipStream_t s) {
    if (!S.on) return;
    if (S.rc > 0) {
        if (S.vals32.get()) return;
        const int64_t nv = S.cap * S.rc;
        S.vals32.alloc(static_cast<size_t>(nv));
        launch_to_float(S.vals.get(), S.vals32.get(), nv, s);
    } else {
        row_blocks_to_float(S.rows, S.cap, bs, s);
    }
}

}  // namespace nair
