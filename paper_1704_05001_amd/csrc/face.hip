// Face-compressed copy of a block matrix for the cycle kernels.
//
// In an upwind DG operator the block coupling element I to its upwind
// neighbour J holds the face term: only the rows of I's nodes on the shared
// face and the columns of J's nodes on it are nonzero ((p+1)^2 of the (p+1)^4
// entries with tensor-product nodes on the faces).  The copy keeps, per
// off-diagonal block, the masks of its nonzero rows and columns and the dense
// rectangle they span, and the diagonal blocks whole; the relaxation and
// residual kernels read that instead of whole blocks.  Exact zeros are the
// only entries left out, so the kernels' results do not change.
#include <algorithm>

#include "common.h"

namespace nair {
namespace {

__device__ inline int nth_set_bit(uint32_t m, int k) {
    for (int i = 0; i < k; ++i) m &= m - 1u;
    return __ffs(static_cast<int>(m)) - 1;
}

// Per block row: where its diagonal block sits (its meta cleared: kept whole),
// and the largest nonzero row and column counts of its off-diagonal blocks,
// combined per workgroup before one atomic each.
__global__ __launch_bounds__(256) void k_face_rows(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                  int nb, unsigned long long *__restrict__ meta,
                                                  int *__restrict__ diagpos, int *__restrict__ maxrc) {
    __shared__ int red[2][4];
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    int rmax = 0, cmax = 0;
    if (I < nb) {
        for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            if (colidx[t] == I) {
                diagpos[I] = t;
                meta[t] = 0ull;
            } else {
                const unsigned long long m = meta[t];
                rmax = max(rmax, __popc(static_cast<unsigned>(m)));
                cmax = max(cmax, __popc(static_cast<unsigned>(m >> 32)));
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rmax = max(rmax, __shfl_xor(rmax, o, 64));
        cmax = max(cmax, __shfl_xor(cmax, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = rmax;
        red[1][threadIdx.x >> 6] = cmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(maxrc, max(max(red[0][0], red[0][1]), max(red[0][2], red[0][3])));
        atomicMax(maxrc + 1, max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3])));
    }
}

// out[t][p][q] = block t's entry on its p-th nonzero row and q-th nonzero
// column, zero past its own counts (and for diagonal blocks, meta 0).
__global__ __launch_bounds__(256) void k_face_fill(const double *__restrict__ vals,
                                                  const unsigned long long *__restrict__ meta, int64_t nnzb, int bs,
                                                  int cmax, int rc, double *__restrict__ out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nnzb * rc) return;
    const int64_t t = g / rc;
    const int e = static_cast<int>(g - t * rc);
    const int p = e / cmax, q = e - p * cmax;
    const unsigned long long m = meta[t];
    const uint32_t rm = static_cast<uint32_t>(m), cm = static_cast<uint32_t>(m >> 32);
    double v = 0.0;
    if (p < __popc(rm) && q < __popc(cm))
        v = vals[t * bs * bs + static_cast<int64_t>(nth_set_bit(rm, p)) * bs + nth_set_bit(cm, q)];
    out[g] = v;
}

// dvals[I] = A_II by columns (entry (a, c) at c * bs + a)
__global__ __launch_bounds__(256) void k_face_diag(const double *__restrict__ vals, const int *__restrict__ diagpos,
                                                  int nb, int bs, double *__restrict__ dvals) {
    // one wave per block: read as stored (consecutive lanes, consecutive words)
    // into the wave's LDS tile, written by columns the same way
    __shared__ double tile[4][32 * 32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t I = static_cast<int64_t>(blockIdx.x) * 4 + w;
    if (I >= nb) return;   // whole waves; no workgroup barrier below
    const int bb = bs * bs;
    const double *src = vals + static_cast<int64_t>(diagpos[I]) * bb;
    double *tl = tile[w];
    // every load of the block first (bs <= 32: at most 16 words per lane; words past
    // the block repeat its last, unused), then the tile, then the stores
    constexpr int kChunks = 16;
    double v[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int e = lane + 64 * i;
        v[i] = src[e < bb ? e : bb - 1];
    }
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int e = lane + 64 * i;
        if (e < bb) tl[e] = v[i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double *dst = dvals + I * bb;
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int g = lane + 64 * i;
        if (g < bb) {
            const int c = g / bs, a = g - c * bs;
            dst[g] = tl[a * bs + c];
        }
    }
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

void build_face(const DevBSR &A, FaceCopy &F, hipStream_t s, DBuf<uint64_t> *meta_known) {
    F = FaceCopy();
    const int bs = A.bs;
    if (bs < 2 || bs > 32 || A.nb == 0 || A.nnzb == 0) return;
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    DBuf<uint64_t> meta;
    const bool known = meta_known && meta_known->get();
    if (known)
        meta = std::move(*meta_known);
    else
        meta.alloc(static_cast<size_t>(A.nnzb));
    DBuf<int> diagpos(static_cast<size_t>(A.nb)), maxrc(2);
    NAIR_HIP(hipMemsetAsync(maxrc.get(), 0, sizeof(int) * 2, s));
    NAIR_HIP(hipMemsetAsync(diagpos.get(), 0, sizeof(int) * A.nb, s));   // (every validated row has its diagonal)
    auto *m64 = reinterpret_cast<unsigned long long *>(meta.get());
    // meta[t] = nonzero rows | nonzero columns << 32
    if (!known)
        launch_block_scan(A.vals.get(), A.nnzb, bs, nullptr, nullptr, nullptr, meta.get(), nullptr, nullptr, s);
    k_face_rows<<<blocks_for(A.nb), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), A.nb, m64, diagpos.get(),
                                                  maxrc.get());
    NAIR_HIP(hipGetLastError());
    int rc2[2] = {0, 0};
    read_ints(maxrc.get(), rc2, 2, s);
    const int rmax = rc2[0], cmax = rc2[1];
    if (2 * rmax * cmax > bs * bs) return;   // the rectangles would hold more than half a block
    F.rmax = rmax;
    F.cmax = std::max(cmax, 1);
    F.rc = std::max(rmax * cmax, 1);
    F.meta = std::move(meta);
    F.vals.alloc(static_cast<size_t>(A.nnzb) * F.rc);
    F.dvals.alloc(static_cast<size_t>(A.nb) * bb);
    k_face_fill<<<blocks_for(A.nnzb * F.rc), 256, 0, s>>>(A.vals.get(), m64, A.nnzb, bs, F.cmax, F.rc,
                                                         F.vals.get());
    NAIR_HIP(hipGetLastError());
    k_face_diag<<<static_cast<unsigned>((A.nb + 3) / 4), 256, 0, s>>>(A.vals.get(), diagpos.get(), A.nb, bs,
                                                                     F.dvals.get());
    NAIR_HIP(hipGetLastError());
    F.on = true;
}

void face_to_float(const DevBSR &A, FaceCopy &F, hipStream_t s) {
    if (!F.on || F.vals32.get()) return;
    const int64_t nv = A.nnzb * F.rc, nd = static_cast<int64_t>(A.nb) * A.bs * A.bs;
    F.vals32.alloc(static_cast<size_t>(nv));
    F.dvals32.alloc(static_cast<size_t>(nd));
    launch_to_float(F.vals.get(), F.vals32.get(), nv, s);
    launch_to_float(F.dvals.get(), F.dvals32.get(), nd, s);
}

}  // namespace nair
