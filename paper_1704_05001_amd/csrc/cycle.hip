// Cycle kernels: block residual r = b - A x with fused squared norm, fused
// block-Jacobi sweep (residual of the block row, then D^-1 or D^-T in LDS),
// restriction r_c = r_C + Z r_F, one-point interpolation, and the transposed
// counterparts (P^T gather, R^T = [Z^T; I] scatter-free update).
#include "common.h"

namespace nair {
namespace {

constexpr int kThreads = 256;

__device__ inline double block_reduce_sum(double v, double *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < static_cast<int>(blockDim.x) / 64; ++k) s += lds[k];
    return s;   // valid in thread 0
}

// r = b - A x, one thread per scalar row; partials[block] = sum of r^2 over the block.
__global__ __launch_bounds__(kThreads) void k_residual(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                      const double *__restrict__ vals, int nb, int bs,
                                                      const double *__restrict__ b, const double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ partials) {
    __shared__ double lds[kThreads / 64];
    const int64_t n = static_cast<int64_t>(nb) * bs;
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    double v = 0.0;
    if (g < n) {
        const int I = static_cast<int>(g / bs);
        const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
        const int bb = bs * bs;
        double acc = 0.0;
        for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            const double *blk = vals + static_cast<int64_t>(t) * bb + a * bs;
            const double *xj = x + static_cast<int64_t>(colidx[t]) * bs;
            for (int c = 0; c < bs; ++c) acc += blk[c] * xj[c];
        }
        const double rv = b[g] - acc;
        r[g] = rv;
        v = rv * rv;
    }
    if (partials) {
        const double s = block_reduce_sum(v, lds);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kThreads) void k_sumsq(const double *__restrict__ v, int64_t n,
                                                   double *__restrict__ partials) {
    __shared__ double lds[kThreads / 64];
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const double x = (g < n) ? v[g] : 0.0;
    const double s = block_reduce_sum(x * x, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_reduce_partials(const double *__restrict__ partials, int npart,
                                                         double *__restrict__ out) {
    __shared__ double lds[1024 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < npart; i += 1024) s += partials[i];
    const double t = block_reduce_sum(s, lds);
    if (threadIdx.x == 0) *out = t;
}

// One Jacobi sweep: e_out_I = e_in_I + D_I^{-1} (r_I - (A e_in)_I) for the listed rows
// (list == nullptr: every row with cf == only_cf; other rows copy e_in).
// floor(256/bs) block rows per workgroup, bs threads per block row.
__global__ __launch_bounds__(kThreads) void k_relax(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                   const double *__restrict__ vals, const double *__restrict__ dinv,
                                                   int dinv_trans, int nb, int bs, const double *__restrict__ r,
                                                   const double *__restrict__ ein, double *__restrict__ eout,
                                                   const int *__restrict__ list, int nlist,
                                                   const int8_t *__restrict__ cf, int only_cf) {
    __shared__ double tb[kThreads];
    const int rows = kThreads / bs;
    const int lr = threadIdx.x / bs;
    const int a = threadIdx.x - lr * bs;
    const int idx = blockIdx.x * rows + lr;
    const int N = list ? nlist : nb;
    int I = -1;
    if (lr < rows && idx < N) I = list ? list[idx] : idx;
    const bool upd = I >= 0 && (list != nullptr || cf[I] == only_cf);
    const int bb = bs * bs;
    if (upd) {
        double acc = 0.0;
        for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            const double *blk = vals + static_cast<int64_t>(t) * bb + a * bs;
            const double *xj = ein + static_cast<int64_t>(colidx[t]) * bs;
            for (int c = 0; c < bs; ++c) acc += blk[c] * xj[c];
        }
        tb[threadIdx.x] = r[static_cast<int64_t>(I) * bs + a] - acc;
    }
    __syncthreads();
    if (I >= 0) {
        const int64_t o = static_cast<int64_t>(I) * bs + a;
        if (upd) {
            const double *D = dinv + static_cast<int64_t>(I) * bb;
            const double *t = tb + lr * bs;
            double d = 0.0;
            if (dinv_trans)
                for (int c = 0; c < bs; ++c) d += D[c * bs + a] * t[c];
            else
                for (int c = 0; c < bs; ++c) d += D[a * bs + c] * t[c];
            eout[o] = ein[o] + d;
        } else {
            eout[o] = ein[o];
        }
    }
}

// rc_i = r_{cpts[i]} + sum_t Z_it r_{col t}
__global__ __launch_bounds__(kThreads) void k_restrict(const int *__restrict__ zrp, const int *__restrict__ zcol,
                                                      const double *__restrict__ zval, int nc, int bs,
                                                      const double *__restrict__ r, const int *__restrict__ cpts,
                                                      double *__restrict__ rc) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nc) * bs) return;
    const int i = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(i) * bs);
    const int bb = bs * bs;
    double acc = 0.0;
    for (int t = zrp[i]; t < zrp[i + 1]; ++t) {
        const double *blk = zval + static_cast<int64_t>(t) * bb + a * bs;
        const double *rj = r + static_cast<int64_t>(zcol[t]) * bs;
        for (int c = 0; c < bs; ++c) acc += blk[c] * rj[c];
    }
    rc[g] = r[static_cast<int64_t>(cpts[i]) * bs + a] + acc;
}

__global__ __launch_bounds__(kThreads) void k_interp(const int *__restrict__ pmap, const double *__restrict__ ec,
                                                    double *__restrict__ e0, double *__restrict__ e1, int nb, int bs) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
    const int p = pmap[I];
    const double v = (p >= 0) ? ec[static_cast<int64_t>(p) * bs + a] : 0.0;
    e0[g] = v;
    e1[g] = v;
}

// sc_j = sum over fine blocks I with pmap(I) = j of s_I
__global__ __launch_bounds__(kThreads) void k_restrict_T(const int *__restrict__ ptptr, const int *__restrict__ ptidx,
                                                        const double *__restrict__ s, double *__restrict__ sc, int nc,
                                                        int bs) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nc) * bs) return;
    const int j = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(j) * bs);
    double acc = 0.0;
    for (int t = ptptr[j]; t < ptptr[j + 1]; ++t) acc += s[static_cast<int64_t>(ptidx[t]) * bs + a];
    sc[g] = acc;
}

// y_I += [I is C] yc_{cidx I} + sum_t (Z^T)_It yc_{col t}
__global__ __launch_bounds__(kThreads) void k_interp_T(const int *__restrict__ ztrp, const int *__restrict__ ztcol,
                                                      const double *__restrict__ ztval, int nb, int bs,
                                                      const int *__restrict__ cidx, const double *__restrict__ yc,
                                                      double *__restrict__ y) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(g / bs);
    const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
    const int bb = bs * bs;
    double acc = 0.0;
    const int ci = cidx[I];
    if (ci >= 0) acc = yc[static_cast<int64_t>(ci) * bs + a];
    for (int t = ztrp[I]; t < ztrp[I + 1]; ++t) {
        const double *blk = ztval + static_cast<int64_t>(t) * bb + a * bs;
        const double *yj = yc + static_cast<int64_t>(ztcol[t]) * bs;
        for (int c = 0; c < bs; ++c) acc += blk[c] * yj[c];
    }
    y[g] += acc;
}

// y0 = y1 = (FC ? [D_C^{-T} g_C ; 0] : 0)
__global__ __launch_bounds__(kThreads) void k_init_T(const double *__restrict__ dinv, const double *__restrict__ g,
                                                    const int8_t *__restrict__ cf, int fc, double *__restrict__ y0,
                                                    double *__restrict__ y1, int nb, int bs) {
    const int64_t gi = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (gi >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(gi / bs);
    const int a = static_cast<int>(gi - static_cast<int64_t>(I) * bs);
    double v = 0.0;
    if (fc && cf[I] == 1) {
        const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
        const double *gI = g + static_cast<int64_t>(I) * bs;
        for (int c = 0; c < bs; ++c) v += D[c * bs + a] * gI[c];
    }
    y0[gi] = v;
    y1[gi] = v;
}

__global__ __launch_bounds__(kThreads) void k_axpy(double *__restrict__ x, const double *__restrict__ e, int64_t n) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g < n) x[g] += e[g];
}

}  // namespace

int residual_partials_count(const DevBSR &A) {
    return static_cast<int>(grid_for(static_cast<int64_t>(A.nb) * A.bs, kThreads));
}

void launch_residual(const DevBSR &A, const double *b, const double *x, double *r, double *partials, int npart,
                     hipStream_t s) {
    const int64_t n = static_cast<int64_t>(A.nb) * A.bs;
    (void)npart;
    k_residual<<<grid_for(n, kThreads), kThreads, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.vals.get(), A.nb, A.bs, b,
                                                         x, r, partials);
    NAIR_HIP(hipGetLastError());
}

void launch_sumsq(const double *v, int64_t n, double *partials, int npart, hipStream_t s) {
    (void)npart;
    k_sumsq<<<grid_for(n, kThreads), kThreads, 0, s>>>(v, n, partials);
    NAIR_HIP(hipGetLastError());
}

void launch_reduce_partials(const double *partials, int npart, double *out, hipStream_t s) {
    k_reduce_partials<<<1, 1024, 0, s>>>(partials, npart, out);
    NAIR_HIP(hipGetLastError());
}

void launch_relax(const DevBSR &A, const double *dinv, bool dinv_trans, const double *r, const double *ein,
                  double *eout, const int *list, int nlist, const int8_t *cf, int only_cf, hipStream_t s) {
    const int rows = kThreads / A.bs;
    const int N = list ? nlist : A.nb;
    if (N <= 0) return;
    k_relax<<<grid_for(N, rows), kThreads, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.vals.get(), dinv,
                                                  dinv_trans ? 1 : 0, A.nb, A.bs, r, ein, eout, list, nlist, cf,
                                                  only_cf);
    NAIR_HIP(hipGetLastError());
}

void launch_restrict(const DevBSR &Z, const double *r, const int *cpts, double *rc, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(Z.nb) * Z.bs;
    if (n <= 0) return;
    k_restrict<<<grid_for(n, kThreads), kThreads, 0, s>>>(Z.rowptr.get(), Z.colidx.get(), Z.vals.get(), Z.nb, Z.bs, r,
                                                         cpts, rc);
    NAIR_HIP(hipGetLastError());
}

void launch_interp(const int *pmap, const double *ec, double *e0, double *e1, int nb, int bs, hipStream_t s) {
    k_interp<<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(pmap, ec, e0, e1, nb, bs);
    NAIR_HIP(hipGetLastError());
}

void launch_restrict_T(const int *ptptr, const int *ptidx, const double *sv, double *sc, int nc, int bs,
                       hipStream_t st) {
    if (nc <= 0) return;
    k_restrict_T<<<grid_for(static_cast<int64_t>(nc) * bs, kThreads), kThreads, 0, st>>>(ptptr, ptidx, sv, sc, nc,
                                                                                          bs);
    NAIR_HIP(hipGetLastError());
}

void launch_interp_T(const DevBSR &ZT, const int *cidx, const double *yc, double *y, hipStream_t s) {
    k_interp_T<<<grid_for(static_cast<int64_t>(ZT.nb) * ZT.bs, kThreads), kThreads, 0, s>>>(
        ZT.rowptr.get(), ZT.colidx.get(), ZT.vals.get(), ZT.nb, ZT.bs, cidx, yc, y);
    NAIR_HIP(hipGetLastError());
}

void launch_init_T(const double *dinv, const double *g, const int8_t *cf, int fc, double *y0, double *y1, int nb,
                   int bs, hipStream_t s) {
    k_init_T<<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(dinv, g, cf, fc, y0, y1, nb, bs);
    NAIR_HIP(hipGetLastError());
}

void launch_axpy(double *x, const double *e, int64_t n, hipStream_t s) {
    k_axpy<<<grid_for(n, kThreads), kThreads, 0, s>>>(x, e, n);
    NAIR_HIP(hipGetLastError());
}

}  // namespace nair
