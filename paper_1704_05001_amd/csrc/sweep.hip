// Sweep copies: the F rows of a level operator (or its transpose) in F-list
// order, each without its diagonal block, with D_F^{-1} in the same order
// (SweepCopy).  A Jacobi F sweep then streams its matrix entries, column
// indices and inverse blocks contiguously instead of picking F rows out from
// between the C rows.  Built once per level and direction: an exact count of
// every row's off-diagonal blocks, a scan, and one wave per row copying its
// column indices, blocks (or face masks and rectangles) and D^{-1} block with
// consecutive lanes on consecutive words.  Nothing is read back to the host.
#include <algorithm>

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
// diagonal go to positions orp[f] ... in order; w words per block (bs*bs, or
// the face rectangle's rc); nothing is written at or past cap.
template <bool FACE>
__global__ __launch_bounds__(256) void k_sweep_fill(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                   const double *__restrict__ src, const uint64_t *__restrict__ fmeta,
                                                   const double *__restrict__ dinv, const int *__restrict__ flist,
                                                   int nF, int w, int bb, int64_t cap, const int *__restrict__ orp,
                                                   int *__restrict__ ocol, uint64_t *__restrict__ ometa,
                                                   double *__restrict__ ovals, double *__restrict__ odinv) {
    const int lane = threadIdx.x & 63;
    const int f = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
    if (f >= nF) return;   // whole waves
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
    }
    const int64_t total = static_cast<int64_t>(n) * w;
    for (int64_t e = lane; e < total; e += 64) {
        const int k = static_cast<int>(e / w);
        const int64_t q = e - static_cast<int64_t>(k) * w;
        const int t = lo + k;
        const int64_t d = static_cast<int64_t>(o) + k - (t > dp ? 1 : 0);
        if (t == dp || d >= cap) continue;
        ovals[d * w + q] = src[static_cast<int64_t>(t) * w + q];
    }
    const double *Di = dinv + static_cast<int64_t>(I) * bb;
    double *Do = odinv + static_cast<int64_t>(f) * bb;
    for (int e = lane; e < bb; e += 64) Do[e] = Di[e];
}

}  // namespace

void build_sweep(const DevBSR &A, const FaceCopy &F, const double *dinv, const int *flist, int nF, SweepCopy &S,
                 hipStream_t s) {
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
    S.vals.alloc(static_cast<size_t>(S.cap) * w);
    if (face) S.meta.alloc(static_cast<size_t>(S.cap));
    S.dinv.alloc(static_cast<size_t>(nF) * bb);
    DBuf<int> cnt(static_cast<size_t>(nF));
    k_sweep_count<<<grid_for(nF, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), flist, nF, cnt.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), S.rowptr.get(), nF, s);
    const unsigned grid = static_cast<unsigned>((nF + 3) / 4);
    if (face) {
        k_sweep_fill<true><<<grid, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), F.vals.get(), F.meta.get(), dinv,
                                                flist, nF, w, bb, S.cap, S.rowptr.get(), S.colidx.get(),
                                                S.meta.get(), S.vals.get(), S.dinv.get());
    } else {
        k_sweep_fill<false><<<grid, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.vals.get(), nullptr, dinv, flist,
                                                 nF, w, bb, S.cap, S.rowptr.get(), S.colidx.get(), nullptr,
                                                 S.vals.get(), S.dinv.get());
    }
    NAIR_HIP(hipGetLastError());
    S.on = true;
}

void sweep_to_float(SweepCopy &S, int bs, hipStream_t s) {
    if (!S.on || S.vals32.get()) return;
    const int64_t nv = S.cap * (S.rc > 0 ? S.rc : static_cast<int64_t>(bs) * bs);
    S.vals32.alloc(static_cast<size_t>(nv));
    launch_to_float(S.vals.get(), S.vals32.get(), nv, s);
}

}  // namespace nair
