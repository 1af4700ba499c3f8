// Row-wise block SpGEMM (Gustavson order) with LDS hash tables for the
// symbolic phase and LDS accumulators for the numeric phase; union-add of
// two block matrices; and the one-point Galerkin merge K = (R A) P with the
// drop filter.
//
// Determinism: every output entry is one fma chain over the inner block
// index K ascending (the order of X's sorted row, with X's implicit identity
// block merged in at its column), c ascending within a block product,
// starting from +0.  Rows are independent; inside a row the K steps are
// separated by barriers, and within a step each output entry has one writer.
#include <algorithm>

#include "common.h"

#pragma clang fp contract(off)

namespace nair {
namespace {

constexpr int kWave = 64;
constexpr int kEmpty = -1;
constexpr int kNumThreads = 256;     // numeric kernels
constexpr int kOutColsLds = 2048;    // output columns kept in LDS (else searched in global memory)
constexpr int kPosLds = 512;         // Y-row positions per chunk
constexpr int kAccBytes = 32768;     // LDS accumulator budget per workgroup

__device__ inline bool hash_insert(int *table, int mask, int key) {
    unsigned slot = (static_cast<unsigned>(key) * 2654435761u) & static_cast<unsigned>(mask);
    while (true) {
        int prev = atomicCAS(&table[slot], kEmpty, key);
        if (prev == kEmpty) return true;
        if (prev == key) return false;
        slot = (slot + 1) & static_cast<unsigned>(mask);
    }
}

__device__ inline int find_pos(const int *arr, int n, int key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (arr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && arr[lo] == key) ? lo : -1;
}

// ------------------------------------------------------------ upper bounds

// ub[i] = sum of the lengths of Y's rows touched by X's row i (plus the identity's row).
__global__ __launch_bounds__(256) void k_row_upper_bound(const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                                        const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                                        int m, int *__restrict__ ub, int small_cap,
                                                        int *__restrict__ big_list, int *__restrict__ big_count,
                                                        int large_cap, int *__restrict__ too_dense) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t s = 0;
    for (int q = xrowptr[i]; q < xrowptr[i + 1]; ++q) s += yrowptr[xcol[q] + 1] - yrowptr[xcol[q]];
    if (xdiag) s += yrowptr[xdiag[i] + 1] - yrowptr[xdiag[i]];
    const int v = s > 0x3fffffff ? 0x3fffffff : static_cast<int>(s);
    ub[i] = v;
    if (v > small_cap) {
        if (v > large_cap) atomicMax(too_dense, v);
        big_list[atomicAdd(big_count, 1)] = i;
    }
}

// ---------------------------------------------------- SpGEMM symbolic phase

// Insert the keys of row i into an LDS hash table shared by `nthr` threads.
__device__ inline int insert_row_keys(int i, const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                      const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                      const int *__restrict__ ycol, int *table, int mask, int tid, int nthr) {
    int added = 0;
    const int q0 = xrowptr[i], q1 = xrowptr[i + 1];
    const int nk = q1 - q0 + (xdiag ? 1 : 0);
    for (int q = 0; q < nk; ++q) {
        const int K = (q < q1 - q0) ? xcol[q0 + q] : xdiag[i];
        for (int u = yrowptr[K] + tid; u < yrowptr[K + 1]; u += nthr) added += hash_insert(table, mask, ycol[u]) ? 1 : 0;
    }
    return added;
}

// Collect the table's keys, rank-sort them and write them to out[0..n).
__device__ inline void emit_sorted(const int *table, int slots, int *list, int *list_n, int *out, int tid, int nthr) {
    for (int s = tid; s < slots; s += nthr) {
        const int k = table[s];
        if (k != kEmpty) list[atomicAdd(list_n, 1)] = k;
    }
    __syncthreads();
    const int n = *list_n;
    for (int a = tid; a < n; a += nthr) {
        const int k = list[a];
        int r = 0;
        for (int b = 0; b < n; ++b) r += (list[b] < k) ? 1 : 0;
        out[r] = k;
    }
}

// Small rows: one wave per row, 4 rows per workgroup; rows with ub > small cap
// are left to the large kernel.  mode 0: count into cnt[i]; mode 1: write sorted
// columns at crowptr[i].
__global__ __launch_bounds__(256) void k_symbolic_small(const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                                       const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                                       const int *__restrict__ ycol, int m,
                                                       const int *__restrict__ ub, int small_cap, int mode,
                                                       int *__restrict__ cnt, const int *__restrict__ crowptr,
                                                       int *__restrict__ ccol) {
    __shared__ int tables[4][kHashSmall];
    __shared__ int lists[4][kHashSmall / 2];
    __shared__ int counts[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *table = tables[w];
    for (int i0 = blockIdx.x * 4; i0 < m; i0 += gridDim.x * 4) {
        const int i = i0 + w;
        const bool active = i < m && ub[i] <= small_cap;
        for (int s = lane; s < kHashSmall; s += kWave) table[s] = kEmpty;
        if (lane == 0) counts[w] = 0;
        __syncthreads();
        int added = 0;
        if (active) added = insert_row_keys(i, xrowptr, xcol, xdiag, yrowptr, ycol, table, kHashSmall - 1, lane, kWave);
        __syncthreads();
        if (mode == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o, kWave);
            if (active && lane == 0) cnt[i] = added;
        } else {
            // emit_sorted synchronises the whole workgroup, so every wave runs it
            int *list = lists[w];
            int *dst = active ? ccol + crowptr[i] : nullptr;
            for (int s = lane; s < kHashSmall; s += kWave) {
                const int k = table[s];
                if (active && k != kEmpty) list[atomicAdd(&counts[w], 1)] = k;
            }
            __syncthreads();
            const int n = active ? counts[w] : 0;
            for (int a = lane; a < n; a += kWave) {
                const int k = list[a];
                int r = 0;
                for (int b = 0; b < n; ++b) r += (list[b] < k) ? 1 : 0;
                dst[r] = k;
            }
        }
        __syncthreads();
    }
}

// Large rows (listed in big_list): one 256-thread workgroup per row, 64 KB hash.
__global__ __launch_bounds__(256) void k_symbolic_large(const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                                       const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                                       const int *__restrict__ ycol, const int *__restrict__ big_list,
                                                       const int *__restrict__ big_count, int large_cap, int mode,
                                                       int *__restrict__ cnt, const int *__restrict__ crowptr,
                                                       int *__restrict__ ccol, const int *__restrict__ ub) {
    extern __shared__ int lds_i[];
    int *table = lds_i;                 // kHashLarge
    int *list = lds_i + kHashLarge;     // kHashLarge / 2
    __shared__ int nadd;
    __shared__ int nlist;
    const int nbig = *big_count;
    for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int i = big_list[b];
        if (ub[i] > large_cap) continue;   // reported as too dense on the host
        for (int s = threadIdx.x; s < kHashLarge; s += blockDim.x) table[s] = kEmpty;
        if (threadIdx.x == 0) {
            nadd = 0;
            nlist = 0;
        }
        __syncthreads();
        int added = insert_row_keys(i, xrowptr, xcol, xdiag, yrowptr, ycol, table, kHashLarge - 1, threadIdx.x,
                                    blockDim.x);
        if (added) atomicAdd(&nadd, added);
        __syncthreads();
        if (mode == 0) {
            if (threadIdx.x == 0) cnt[i] = nadd;
        } else {
            emit_sorted(table, kHashLarge, list, &nlist, ccol + crowptr[i], threadIdx.x, blockDim.x);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------- SpGEMM numeric phase

__global__ __launch_bounds__(kNumThreads) void k_spgemm_numeric(
    const int *__restrict__ xrowptr, const int *__restrict__ xcol, const double *__restrict__ xval,
    const int *__restrict__ xdiag, const int *__restrict__ yrowptr, const int *__restrict__ ycol,
    const double *__restrict__ yval, int m, const int *__restrict__ crowptr, const int *__restrict__ ccol,
    double *__restrict__ cval, int bs, int tile_blocks) {
    extern __shared__ double lds_d[];
    const int bb = bs * bs;
    double *acc = lds_d;                                  // tile_blocks * bb
    double *xblk = acc + static_cast<size_t>(tile_blocks) * bb;   // bb
    int *cols = reinterpret_cast<int *>(xblk + bb);       // kOutColsLds
    int *ypos = cols + kOutColsLds;                       // kPosLds
    const int tid = threadIdx.x;
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const int c0 = crowptr[i];
        const int nout = crowptr[i + 1] - c0;
        const bool cols_in_lds = nout <= kOutColsLds;
        if (cols_in_lds)
            for (int p = tid; p < nout; p += kNumThreads) cols[p] = ccol[c0 + p];
        const int *colsrc = cols_in_lds ? cols : ccol + c0;
        for (int p0 = 0; p0 < nout; p0 += tile_blocks) {
            const int pt = min(tile_blocks, nout - p0);
            for (int e = tid; e < pt * bb; e += kNumThreads) acc[e] = 0.0;
            __syncthreads();
            const int q0 = xrowptr[i], q1 = xrowptr[i + 1];
            int q = q0;
            bool diag_pending = xdiag != nullptr;
            while (q < q1 || diag_pending) {
                const bool take_diag = diag_pending && (q >= q1 || xdiag[i] < xcol[q]);
                const int K = take_diag ? xdiag[i] : xcol[q];
                if (!take_diag)
                    for (int e = tid; e < bb; e += kNumThreads) xblk[e] = xval[static_cast<int64_t>(q) * bb + e];
                const int ylo = yrowptr[K];
                const int yn = yrowptr[K + 1] - ylo;
                for (int u0 = 0; u0 < yn; u0 += kPosLds) {
                    const int un = min(kPosLds, yn - u0);
                    for (int u = tid; u < un; u += kNumThreads) {
                        const int p = find_pos(colsrc, nout, ycol[ylo + u0 + u]);
                        ypos[u] = (p >= p0 && p < p0 + pt) ? p - p0 : -1;
                    }
                    __syncthreads();
                    for (int wi = tid; wi < un * bb; wi += kNumThreads) {
                        const int u = wi / bb;
                        const int lp = ypos[u];
                        if (lp < 0) continue;
                        const int e = wi - u * bb;
                        const double *y = yval + static_cast<int64_t>(ylo + u0 + u) * bb;
                        double s = acc[lp * bb + e];
                        if (take_diag) {
                            s = s + y[e];
                        } else {
                            const int a = e / bs, b = e - a * bs;
                            const double *xr = xblk + a * bs;
                            for (int c = 0; c < bs; ++c) s = __builtin_fma(xr[c], y[c * bs + b], s);
                        }
                        acc[lp * bb + e] = s;
                    }
                    __syncthreads();
                }
                if (take_diag) diag_pending = false;
                else ++q;
            }
            double *dst = cval + static_cast<int64_t>(c0 + p0) * bb;
            for (int e = tid; e < pt * bb; e += kNumThreads) dst[e] = acc[e];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------- union add

__global__ __launch_bounds__(256) void k_add_count(const int *__restrict__ srp, const int *__restrict__ sc,
                                                  const int *__restrict__ wrp, const int *__restrict__ wc, int m,
                                                  int *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int p = srp[i], q = wrp[i];
    const int pe = srp[i + 1], qe = wrp[i + 1];
    int n = 0;
    while (p < pe || q < qe) {
        if (q >= qe || (p < pe && sc[p] < wc[q])) ++p;
        else if (p >= pe || wc[q] < sc[p]) ++q;
        else {
            ++p;
            ++q;
        }
        ++n;
    }
    cnt[i] = n;
}

__global__ __launch_bounds__(256) void k_add_fill(const int *__restrict__ srp, const int *__restrict__ sc,
                                                 const int *__restrict__ wrp, const int *__restrict__ wc, int m,
                                                 const int *__restrict__ orp, int *__restrict__ oc,
                                                 int *__restrict__ srcS, int *__restrict__ srcW) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int p = srp[i], q = wrp[i];
    const int pe = srp[i + 1], qe = wrp[i + 1];
    int o = orp[i];
    while (p < pe || q < qe) {
        if (q >= qe || (p < pe && sc[p] < wc[q])) {
            oc[o] = sc[p];
            srcS[o] = p++;
            srcW[o] = -1;
        } else if (p >= pe || wc[q] < sc[p]) {
            oc[o] = wc[q];
            srcS[o] = -1;
            srcW[o] = q++;
        } else {
            oc[o] = sc[p];
            srcS[o] = p++;
            srcW[o] = q++;
        }
        ++o;
    }
}

__global__ __launch_bounds__(256) void k_add_values(int64_t n, int bb, const double *__restrict__ S,
                                                   const int *__restrict__ srcS, const double *__restrict__ W,
                                                   const int *__restrict__ srcW, double *__restrict__ O) {
    const int64_t total = n * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bb;
        const int e = static_cast<int>(g - t * bb);
        const int a = srcS[t], b = srcW[t];
        double v;
        if (a >= 0 && b >= 0) v = S[static_cast<int64_t>(a) * bb + e] + W[static_cast<int64_t>(b) * bb + e];
        else if (a >= 0) v = S[static_cast<int64_t>(a) * bb + e];
        else v = W[static_cast<int64_t>(b) * bb + e];
        O[g] = v;
    }
}

// ------------------------------------------------- one-point Galerkin merge

// Keys of K's row i: pmap of RA's row columns (>= 0).  Wave per row.
__global__ __launch_bounds__(256) void k_rap_symbolic(const int *__restrict__ rarp, const int *__restrict__ racol,
                                                     const int *__restrict__ pmap, int m, int mode,
                                                     int *__restrict__ cnt, const int *__restrict__ krp,
                                                     int *__restrict__ kcol, int *__restrict__ too_dense) {
    __shared__ int tables[4][kHashSmall];
    __shared__ int lists[4][kHashSmall / 2];
    __shared__ int counts[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *table = tables[w];
    for (int i0 = blockIdx.x * 4; i0 < m; i0 += gridDim.x * 4) {
        const int i = i0 + w;
        const bool active = i < m && (rarp[i + 1] - rarp[i]) <= kHashSmall / 2;
        if (i < m && !active && lane == 0) atomicMax(too_dense, rarp[i + 1] - rarp[i]);
        for (int s = lane; s < kHashSmall; s += kWave) table[s] = kEmpty;
        if (lane == 0) counts[w] = 0;
        __syncthreads();
        int added = 0;
        if (active)
            for (int u = rarp[i] + lane; u < rarp[i + 1]; u += kWave) {
                const int t = pmap[racol[u]];
                if (t >= 0) added += hash_insert(table, kHashSmall - 1, t) ? 1 : 0;
            }
        __syncthreads();
        if (mode == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o, kWave);
            if (active && lane == 0) cnt[i] = added;
        } else {
            int *list = lists[w];
            for (int s = lane; s < kHashSmall; s += kWave) {
                const int k = table[s];
                if (active && k != kEmpty) list[atomicAdd(&counts[w], 1)] = k;
            }
            __syncthreads();
            const int n = active ? counts[w] : 0;
            int *dst = active ? kcol + krp[i] : nullptr;
            for (int a = lane; a < n; a += kWave) {
                const int k = list[a];
                int r = 0;
                for (int b = 0; b < n; ++b) r += (list[b] < k) ? 1 : 0;
                dst[r] = k;
            }
        }
        __syncthreads();
    }
}

// K_{i,p} = sum over RA blocks u (ascending column) with pmap(col u) = kcol[p] of RA_u,
// then block sizes, the diagonal's size and the keep flags of the drop filter.
__global__ __launch_bounds__(kNumThreads) void k_rap_numeric(const int *__restrict__ rarp, const int *__restrict__ racol,
                                                            const double *__restrict__ raval,
                                                            const int *__restrict__ pmap, int m,
                                                            const int *__restrict__ krp, const int *__restrict__ kcol,
                                                            double *__restrict__ kval, int bs, double drop,
                                                            uint8_t *__restrict__ keep, int *__restrict__ kept_cnt) {
    __shared__ int tpos[kHashSmall / 2];
    __shared__ int kc[kHashSmall / 2];
    __shared__ double bn[kHashSmall / 2];
    __shared__ double dnorm;
    __shared__ int nkept;
    const int bb = bs * bs;
    const int tid = threadIdx.x;
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const int r0 = rarp[i], nra = rarp[i + 1] - r0;
        const int k0 = krp[i], nk = krp[i + 1] - k0;
        if (nra > kHashSmall / 2) continue;   // reported by the symbolic phase
        for (int p = tid; p < nk; p += kNumThreads) kc[p] = kcol[k0 + p];
        if (tid == 0) {
            dnorm = 0.0;
            nkept = 0;
        }
        __syncthreads();
        for (int u = tid; u < nra; u += kNumThreads) {
            const int t = pmap[racol[r0 + u]];
            tpos[u] = (t >= 0) ? find_pos(kc, nk, t) : -1;
        }
        __syncthreads();
        for (int w = tid; w < nk * bb; w += kNumThreads) {
            const int p = w / bb;
            const int e = w - p * bb;
            double s = 0.0;
            for (int u = 0; u < nra; ++u)
                if (tpos[u] == p) s = s + raval[static_cast<int64_t>(r0 + u) * bb + e];
            kval[static_cast<int64_t>(k0) * bb + w] = s;
        }
        __syncthreads();
        for (int p = tid; p < nk; p += kNumThreads) {
            const double *blk = kval + static_cast<int64_t>(k0 + p) * bb;
            double mx = 0.0;
            for (int e = 0; e < bb; ++e) mx = fmax(mx, fabs(blk[e]));
            bn[p] = mx;
            if (kc[p] == i) dnorm = mx;
        }
        __syncthreads();
        const double thr = drop * dnorm;
        int mine = 0;
        for (int p = tid; p < nk; p += kNumThreads) {
            const bool kp = (kc[p] == i) || (bn[p] > thr);
            keep[k0 + p] = kp ? 1 : 0;
            mine += kp ? 1 : 0;
        }
        if (mine) atomicAdd(&nkept, mine);
        __syncthreads();
        if (tid == 0) kept_cnt[i] = nkept;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_compact_fill(const int *__restrict__ krp, const int *__restrict__ kcol,
                                                     const uint8_t *__restrict__ keep, int m,
                                                     const int *__restrict__ orp, int *__restrict__ ocol,
                                                     int *__restrict__ osrc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int o = orp[i];
    for (int t = krp[i]; t < krp[i + 1]; ++t)
        if (keep[t]) {
            ocol[o] = kcol[t];
            osrc[o] = t;
            ++o;
        }
}

unsigned cap_grid(int64_t g) { return static_cast<unsigned>(g > 65536 * 16 ? 65536 * 16 : (g < 1 ? 1 : g)); }

}  // namespace

void spgemm(const DevBSR &X, const int *xdiag, const DevBSR &Y, DevBSR &C, hipStream_t s) {
    const int m = X.nb;
    const int bs = X.bs;
    C.nb = m;
    C.ncols = Y.ncols;
    C.bs = bs;
    C.rowptr.alloc(static_cast<size_t>(m) + 1);
    if (m == 0) {
        NAIR_HIP(hipMemsetAsync(C.rowptr.get(), 0, sizeof(int), s));
        C.nnzb = 0;
        C.colidx.alloc(0);
        C.vals.alloc(0);
        return;
    }
    const int small_cap = kHashSmall / 2, large_cap = kHashLarge / 2;
    DBuf<int> ub(m), cnt(m), big_list(m), flags(2);
    NAIR_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int) * 2, s));
    int *big_count = flags.get(), *too_dense = flags.get() + 1;
    k_row_upper_bound<<<grid_for(m, 256), 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), m,
                                                      ub.get(), small_cap, big_list.get(), big_count, large_cap,
                                                      too_dense);
    const unsigned gs = cap_grid((m + 3) / 4);
    const size_t lds_large = sizeof(int) * (kHashLarge + kHashLarge / 2);
    k_symbolic_small<<<gs, 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), Y.colidx.get(), m,
                                        ub.get(), small_cap, 0, cnt.get(), nullptr, nullptr);
    k_symbolic_large<<<256, 256, lds_large, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(),
                                                 Y.colidx.get(), big_list.get(), big_count, large_cap, 0, cnt.get(),
                                                 nullptr, nullptr, ub.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), C.rowptr.get(), m, s);
    int hflags[2];
    read_ints(flags.get(), hflags, 2, s);
    if (hflags[1] > 0)
        fail(NAIR_ENOMEM, "sparse product row has " + std::to_string(hflags[1]) + " candidate blocks (limit " +
                              std::to_string(large_cap) + ")");
    const int nnz = read_int(C.rowptr.get() + m, s);
    C.nnzb = nnz;
    C.colidx.alloc(nnz);
    C.vals.alloc(static_cast<size_t>(nnz) * bs * bs);
    k_symbolic_small<<<gs, 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), Y.colidx.get(), m,
                                        ub.get(), small_cap, 1, nullptr, C.rowptr.get(), C.colidx.get());
    if (hflags[0] > 0)
        k_symbolic_large<<<256, 256, lds_large, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(),
                                                     Y.colidx.get(), big_list.get(), big_count, large_cap, 1, nullptr,
                                                     C.rowptr.get(), C.colidx.get(), ub.get());
    NAIR_HIP(hipGetLastError());
    if (nnz == 0) return;
    const int bb = bs * bs;
    int tile_blocks = kAccBytes / (8 * bb);
    if (tile_blocks < 1) tile_blocks = 1;
    const size_t lds = sizeof(double) * (static_cast<size_t>(tile_blocks) * bb + bb) +
                       sizeof(int) * (kOutColsLds + kPosLds);
    TimerScope ts(TK_SPGEMM_NUM, g_timer_level, s);
    k_spgemm_numeric<<<cap_grid(m), kNumThreads, lds, s>>>(X.rowptr.get(), X.colidx.get(), X.vals.get(), xdiag,
                                                          Y.rowptr.get(), Y.colidx.get(), Y.vals.get(), m,
                                                          C.rowptr.get(), C.colidx.get(), C.vals.get(), bs,
                                                          tile_blocks);
    NAIR_HIP(hipGetLastError());
}

void bsr_add(const DevBSR &S, const DevBSR &W, DevBSR &O, hipStream_t s) {
    const int m = S.nb;
    const int bs = S.bs;
    O.nb = m;
    O.ncols = S.ncols;
    O.bs = bs;
    O.rowptr.alloc(static_cast<size_t>(m) + 1);
    DBuf<int> cnt(m);
    if (m > 0)
        k_add_count<<<grid_for(m, 256), 256, 0, s>>>(S.rowptr.get(), S.colidx.get(), W.rowptr.get(), W.colidx.get(),
                                                     m, cnt.get());
    scan_exclusive(cnt.get(), O.rowptr.get(), m, s);
    const int nnz = read_int(O.rowptr.get() + m, s);
    O.nnzb = nnz;
    O.colidx.alloc(nnz);
    O.vals.alloc(static_cast<size_t>(nnz) * bs * bs);
    if (nnz == 0) return;
    DBuf<int> srcS(nnz), srcW(nnz);
    k_add_fill<<<grid_for(m, 256), 256, 0, s>>>(S.rowptr.get(), S.colidx.get(), W.rowptr.get(), W.colidx.get(), m,
                                                O.rowptr.get(), O.colidx.get(), srcS.get(), srcW.get());
    const int64_t total = static_cast<int64_t>(nnz) * bs * bs;
    k_add_values<<<cap_grid((total + 255) / 256), 256, 0, s>>>(nnz, bs * bs, S.vals.get(), srcS.get(), W.vals.get(),
                                                              srcW.get(), O.vals.get());
    NAIR_HIP(hipGetLastError());
}

void rap_merge_drop(const DevBSR &RA, const int *pmap, int nc, double drop, DevBSR &K, hipStream_t s) {
    const int m = RA.nb;
    const int bs = RA.bs;
    const int bb = bs * bs;
    DBuf<int> cnt(m), krp(static_cast<size_t>(m) + 1), flags(1);
    NAIR_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int), s));
    const unsigned gs = cap_grid((m + 3) / 4);
    k_rap_symbolic<<<gs, 256, 0, s>>>(RA.rowptr.get(), RA.colidx.get(), pmap, m, 0, cnt.get(), nullptr, nullptr,
                                      flags.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive(cnt.get(), krp.get(), m, s);
    const int too_dense = read_int(flags.get(), s);
    if (too_dense > 0)
        fail(NAIR_ENOMEM, "Galerkin row has " + std::to_string(too_dense) + " blocks (limit " +
                              std::to_string(kHashSmall / 2) + ")");
    const int nnz = read_int(krp.get() + m, s);
    DBuf<int> kcol(nnz);
    DBuf<double> kval(static_cast<size_t>(nnz) * bb);
    DBuf<uint8_t> keep(nnz);
    DBuf<int> kept(m);
    k_rap_symbolic<<<gs, 256, 0, s>>>(RA.rowptr.get(), RA.colidx.get(), pmap, m, 1, nullptr, krp.get(), kcol.get(),
                                      flags.get());
    {
        TimerScope ts(TK_RAP, g_timer_level, s);
        k_rap_numeric<<<cap_grid(m), kNumThreads, 0, s>>>(RA.rowptr.get(), RA.colidx.get(), RA.vals.get(), pmap, m,
                                                          krp.get(), kcol.get(), kval.get(), bs, drop, keep.get(),
                                                          kept.get());
    }
    NAIR_HIP(hipGetLastError());
    K.nb = nc;
    K.ncols = nc;
    K.bs = bs;
    K.rowptr.alloc(static_cast<size_t>(nc) + 1);
    scan_exclusive(kept.get(), K.rowptr.get(), m, s);
    const int nk = read_int(K.rowptr.get() + m, s);
    K.nnzb = nk;
    K.colidx.alloc(nk);
    K.vals.alloc(static_cast<size_t>(nk) * bb);
    DBuf<int> src(nk);
    k_compact_fill<<<grid_for(m, 256), 256, 0, s>>>(krp.get(), kcol.get(), keep.get(), m, K.rowptr.get(),
                                                    K.colidx.get(), src.get());
    NAIR_HIP(hipGetLastError());
    launch_block_gather(nk, bs, kval.get(), src.get(), K.vals.get(), s);
}

}  // namespace nair
