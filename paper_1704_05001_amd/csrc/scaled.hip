// Scalar form: the system scaled by the inverse of its block diagonal
// (section "Blocks, filtering, and parallelization": most of the paper's
// results run scalar nAIR on D^{-1} A).  Builds S = D^{-1} A as a scalar matrix
// and applies D^{-1} (or D^{-T}) to block vectors.
#include "common.h"

#pragma clang fp contract(off)

namespace nair {
namespace {

__global__ __launch_bounds__(256) void k_iota(int *__restrict__ v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = static_cast<int>(i);
}

// Scalar row (I, a) of S: one entry 1 on the diagonal for the block (I, I)
// (the identity, taken exactly) and, for every other stored block, the entries
// of row a of M_t = D_I^{-1} A_t that are not exactly zero, columns ascending.
// fill == false: count them into cnt; fill == true: write them at rowptr.
template <bool FILL>
__global__ __launch_bounds__(256) void k_scaled_rows(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                    const double *__restrict__ M, int nb, int bs,
                                                    int *__restrict__ cnt, const int *__restrict__ srowptr,
                                                    int *__restrict__ scol, double *__restrict__ sval) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    int o = FILL ? srowptr[g] : 0;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t];
        if (J == I) {
            if (FILL) {
                scol[o] = I * bs + a;
                sval[o] = 1.0;
            }
            ++o;
            continue;
        }
        const double *row = M + t * bb + static_cast<int64_t>(a) * bs;
        for (int b = 0; b < bs; ++b) {
            const double v = row[b];
            if (v != 0.0) {
                if (FILL) {
                    scol[o] = J * bs + b;
                    sval[o] = v;
                }
                ++o;
            }
        }
    }
    if (!FILL) cnt[g] = o;
}

// out_I = D_I^{-1} v_I (TRANS: D_I^{-T} v_I) for every block row of a live system.
template <typename VT>
__global__ __launch_bounds__(256) void k_block_diag_apply(const double *__restrict__ dinv, const VT *__restrict__ v,
                                                         double *__restrict__ out, float *__restrict__ out32,
                                                         int nb, int bs, int trans, Gate gate) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
    if (!live(gate, I)) return;
    const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
    const VT *vI = v + static_cast<int64_t>(I) * bs;
    double s = 0.0;
    for (int c = 0; c < bs; ++c) s += (trans ? D[c * bs + a] : D[a * bs + c]) * static_cast<double>(vI[c]);
    out[g] = s;
    if (out32) out32[g] = static_cast<float>(s);
}

}  // namespace

void build_scaled(const DevBSR &A, const double *dinv, DevBSR &S, hipStream_t s) {
    const int nb = A.nb, bs = A.bs;
    const int64_t nnzb = A.nnzb;
    const int64_t n = static_cast<int64_t>(nb) * bs;
    if (n > 2147483647LL) fail(NAIR_EINVAL, "the scaled system has more than 2^31 rows");
    DBuf<int> rowid(nnzb), iota(nnzb);
    DBuf<double> M(static_cast<size_t>(nnzb) * bs * bs);
    launch_rows_of(A.rowptr.get(), nb, rowid.get(), s);
    k_iota<<<grid_for(nnzb, 256), 256, 0, s>>>(iota.get(), nnzb);
    NAIR_HIP(hipGetLastError());
    // M_t = D_I^{-1} A_t (fma chains, c ascending from +0); the diagonal blocks are not used
    launch_block_product(nnzb, bs, dinv, rowid.get(), A.vals.get(), iota.get(), 1.0, M.get(), s);
    S.nb = static_cast<int>(n);
    S.ncols = static_cast<int>(n);
    S.bs = 1;
    S.rowptr.alloc(static_cast<size_t>(n) + 1);
    DBuf<int> cnt(n);
    k_scaled_rows<false><<<grid_for(n, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), M.get(), nb, bs,
                                                          cnt.get(), nullptr, nullptr, nullptr);
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), S.rowptr.get(), static_cast<int>(n), s);
    const int nnz = read_int(S.rowptr.get() + n, s);
    S.nnzb = nnz;
    S.colidx.alloc(nnz);
    S.vals.alloc(nnz);
    k_scaled_rows<true><<<grid_for(n, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), M.get(), nb, bs, nullptr,
                                                         S.rowptr.get(), S.colidx.get(), S.vals.get());
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_block_diag_apply(const double *dinv, const VT *v, double *out, float *out32, int nb, int bs, bool trans,
                             hipStream_t s, Gate gate) {
    if (nb <= 0) return;
    k_block_diag_apply<VT><<<grid_for(static_cast<int64_t>(nb) * bs, 256), 256, 0, s>>>(dinv, v, out, out32, nb, bs,
                                                                                         trans ? 1 : 0, gate);
    NAIR_HIP(hipGetLastError());
}

template void launch_block_diag_apply<double>(const double *, const double *, double *, float *, int, int, bool,
                                              hipStream_t, Gate);
template void launch_block_diag_apply<float>(const double *, const float *, double *, float *, int, int, bool,
                                             hipStream_t, Gate);

}  // namespace nair
