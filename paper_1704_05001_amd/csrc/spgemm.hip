// Row-wise block SpGEMM (Gustavson order): LDS hash tables for the symbolic
// phase (a row's products enumerated flat across a wave), per-output-block
// pair lists in the fixed accumulation order, and numeric kernels that walk
// them (FP64 matrix cores for 9x9 and 16x16 blocks, one thread per block row
// otherwise); union-add of two block matrices; and the Galerkin product
// K = R A P with the one-point P and the drop filter.
//
// Determinism: every output entry is one fma chain over the inner block
// index K ascending (the order of X's sorted row, with X's implicit identity
// block merged in at its column), c ascending within a block product,
// starting from +0.  Rows are independent, and each output block's pairs are
// applied in list order by the one wave or thread that owns the block.
#include <algorithm>

#include <climits>

#include "common.h"
#include "mfma_tile.h"

#pragma clang fp contract(off)

namespace nair {
namespace {

constexpr int kWave = 64;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum of x over the wave's 64 lanes by DPP moves (no LDS
// round trips): shifts by 1, 2, 4, 8 within each row of 16 lanes, then each
// row's last lane added into the rows after it.  A lane whose source lies
// outside its row (or a row the step leaves out) receives 0.
template <int CTRL, int ROWS = 0xF>
__device__ inline int dpp_add(int x) {
    return x + __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xF, false);
}
__device__ inline int wave_incl_scan(int x) {
    x = dpp_add<0x111>(x);          // row_shr:1
    x = dpp_add<0x112>(x);          // row_shr:2
    x = dpp_add<0x114>(x);          // row_shr:4
    x = dpp_add<0x118>(x);          // row_shr:8
    x = dpp_add<0x142, 0xA>(x);     // row_bcast:15 into rows 1 and 3
    x = dpp_add<0x143, 0xC>(x);     // row_bcast:31 into rows 2 and 3
    return x;
}

// Sort a wave's n distinct keys list[0 .. n) ascending in place (n <= cap, the
// list's room): up to 64 keys by rank (a key per lane), more by a bitonic
// network over the next power of two, padded with INT_MAX.
__device__ inline void wave_sort(int *list, int n, int cap, int lane) {
    if (n <= kWave) {
        const int k = lane < n ? list[lane] : 0;
        int r = 0;
        if (lane < n)
            for (int b = 0; b < n; ++b) r += (list[b] < k) ? 1 : 0;
        wave_sync();
        if (lane < n) list[r] = k;
        wave_sync();
        return;
    }
    int n2 = kWave;
    while (n2 < n) n2 <<= 1;
    if (n2 > cap) n2 = cap;   // (n <= cap, a power of two)
    for (int a = n + lane; a < n2; a += kWave) list[a] = INT_MAX;
    wave_sync();
    for (int k = 2; k <= n2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int a = lane; a < n2; a += kWave) {
                const int b = a ^ j;
                if (b > a) {
                    const int x = list[a], y = list[b];
                    if ((x > y) == ((a & k) == 0)) {
                        list[a] = y;
                        list[b] = x;
                    }
                }
            }
            wave_sync();
        }
}

constexpr int kEmpty = -1;

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

// blocks t < *count of O (count on the device)
__global__ __launch_bounds__(256) void k_add_values(const int *__restrict__ count, int bb, const double *__restrict__ S,
                                                   const int *__restrict__ srcS, const double *__restrict__ W,
                                                   const int *__restrict__ srcW, double *__restrict__ O) {
    const int64_t total = static_cast<int64_t>(*count) * bb;
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

// The same with one wave per block (blocks of 64 entries or more).
__global__ __launch_bounds__(256) void k_add_values_wave(const int *__restrict__ count, int bb,
                                                        const double *__restrict__ S, const int *__restrict__ srcS,
                                                        const double *__restrict__ W, const int *__restrict__ srcW,
                                                        double *__restrict__ O) {
    const int lane = threadIdx.x & 63;
    const int64_t nblk = *count;
    const int64_t stride = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; t < nblk; t += stride) {
        const int a = srcS[t], b = srcW[t];
        const double *sp = S + static_cast<int64_t>(a < 0 ? 0 : a) * bb;
        const double *wp = W + static_cast<int64_t>(b < 0 ? 0 : b) * bb;
        double *o = O + t * bb;
        for (int e = lane; e < bb; e += 64) {
            double v;
            if (a >= 0 && b >= 0) v = sp[e] + wp[e];
            else if (a >= 0) v = sp[e];
            else v = wp[e];
            o[e] = v;
        }
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
        int slots = kWave;
        if (active)
            while (slots < 2 * (rarp[i + 1] - rarp[i])) slots <<= 1;
        for (int s = lane; s < slots; s += kWave) table[s] = kEmpty;
        if (lane == 0) counts[w] = 0;
        wave_sync();   // (every LDS array here is the wave's own)
        int added = 0;
        if (active)
            for (int u = rarp[i] + lane; u < rarp[i + 1]; u += kWave) {
                const int t = pmap[racol[u]];
                if (t >= 0) added += hash_insert(table, slots - 1, t) ? 1 : 0;
            }
        wave_sync();
        if (mode == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o, kWave);
            if (active && lane == 0) cnt[i] = added;
        } else {
            int *list = lists[w];
            for (int s = lane; s < slots; s += kWave) {
                const int k = table[s];
                if (active && k != kEmpty) list[atomicAdd(&counts[w], 1)] = k;
            }
            wave_sync();
            const int n = active ? counts[w] : 0;
            int *dst = active ? kcol + krp[i] : nullptr;
            wave_sort(list, n, kHashSmall / 2, lane);
            for (int a = lane; a < n; a += kWave) dst[a] = list[a];
        }
        wave_sync();
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

namespace {

// Position of the implicit identity column among X's sorted row [q0, q1).
__device__ inline int identity_slot(const int *__restrict__ xcol, int q0, int q1, int dcol) {
    int lo = q0, hi = q1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (xcol[mid] < dcol) lo = mid + 1;
        else hi = mid;
    }
    return lo - q0;
}

// Exclusive scan of cnt[0..n) in place by the first wave of the workgroup.
__device__ inline void wave0_scan(int *cnt, int n) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < n; base += 64) {
        const int v = (base + lane < n) ? cnt[base + lane] : 0;
        const int x = wave_incl_scan(v);
        if (base + lane < n) cnt[base + lane] = carry + x - v;
        carry += __builtin_amdgcn_readlane(x, 63);
    }
}

// Contribution lists of one output row: for every output block, the (X block,
// Y block) pairs that feed it, in ascending inner index (X's sorted row with the
// identity merged in; the identity is X block -1).  `cols` (LDS) holds the row's
// sorted output columns, `cnt` (LDS) gets per-block counts, then offsets.
__device__ inline void row_pairs(int i, const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                 const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                 const int *__restrict__ ycol, int c0, int nout, int P0, const int *cols, int *cnt,
                                 int *__restrict__ pairptr, int2 *__restrict__ pairs) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int q0 = xrowptr[i], q1 = xrowptr[i + 1];
    const int nx = q1 - q0;
    const int dslot = xdiag ? identity_slot(xcol, q0, q1, xdiag[i]) : -1;
    const int nk = nx + (xdiag ? 1 : 0);
    for (int qq = 0; qq < nk; ++qq) {
        const int K = (qq == dslot) ? xdiag[i] : xcol[q0 + qq - ((dslot >= 0 && qq > dslot) ? 1 : 0)];
        for (int u = yrowptr[K] + tid; u < yrowptr[K + 1]; u += nthr) atomicAdd(&cnt[find_pos(cols, nout, ycol[u])], 1);
    }
    __syncthreads();
    wave0_scan(cnt, nout);
    __syncthreads();
    for (int p = tid; p < nout; p += nthr) pairptr[c0 + p] = P0 + cnt[p];
    __syncthreads();
    for (int qq = 0; qq < nk; ++qq) {
        const bool ident = qq == dslot;
        const int q = ident ? -1 : q0 + qq - ((dslot >= 0 && qq > dslot) ? 1 : 0);
        const int K = ident ? xdiag[i] : xcol[q];
        for (int u = yrowptr[K] + tid; u < yrowptr[K + 1]; u += nthr) {
            const int p = find_pos(cols, nout, ycol[u]);
            const int pos = cnt[p];     // one writer per block within an inner step
            cnt[p] = pos + 1;
            pairs[P0 + pos] = make_int2(q, u);
        }
        __syncthreads();
    }
}

// Rows listed in big_list: one 256-thread workgroup per row.
__global__ __launch_bounds__(256) void k_pairs_large(const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                                    const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                                    const int *__restrict__ ycol, const int *__restrict__ big_list,
                                                    const int *__restrict__ big_count, const int *__restrict__ crowptr,
                                                    const int *__restrict__ ccol, const int *__restrict__ prow,
                                                    int *__restrict__ pairptr, int2 *__restrict__ pairs) {
    __shared__ int cols[kHashLarge / 2];
    __shared__ int cnt[kHashLarge / 2];
    const int nbig = *big_count;
    for (int bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const int i = big_list[bi];
        const int c0 = crowptr[i], nout = crowptr[i + 1] - c0;
        for (int p = threadIdx.x; p < nout; p += blockDim.x) {
            cols[p] = ccol[c0 + p];
            cnt[p] = 0;
        }
        __syncthreads();
        row_pairs(i, xrowptr, xcol, xdiag, yrowptr, ycol, c0, nout, prow[i], cols, cnt, pairptr, pairs);
        __syncthreads();
    }
}

// Intra-wave ordering of LDS traffic (the rows of k_symbolic_flat are per
// wave and take different numbers of steps, so no workgroup barrier fits).
// Up to 64 inner slots of output row i, one per lane: slot base + lane of the
// row's sorted inner indices (X's row with its implicit identity block merged
// in at its column).  A lane holds its slot's X block (-1: the identity), the
// first Y block of the slot's Y row and the row's length, and the number of
// products of the chunk's slots before its own; `total` is the chunk's count.
struct SlotChunk {
    int q, ybeg, len, excl, total;
};

__device__ inline SlotChunk load_slots(int base, int nk, int q0, int dslot, int dcol, const int *__restrict__ xcol,
                                       const int *__restrict__ yrowptr, int lane) {
    SlotChunk c{-1, 0, 0, 0, 0};
    const int qq = base + lane;
    if (qq < nk) {
        const bool ident = qq == dslot;
        c.q = ident ? -1 : q0 + qq - ((dslot >= 0 && qq > dslot) ? 1 : 0);
        const int K = ident ? dcol : xcol[c.q];
        c.ybeg = yrowptr[K];
        c.len = yrowptr[K + 1] - c.ybeg;
    }
    const int x = wave_incl_scan(c.len);
    c.excl = x - c.len;
    c.total = __builtin_amdgcn_readlane(x, 63);
    return c;
}

// Product p < c.total of a chunk: the slot j holding it (the last lane whose
// excl <= p; empty slots share their successor's excl and lie before it) and
// its (X block, Y block) pair.  Every lane of the wave must call it (it reads
// other lanes' registers); p >= c.total gives a pair of no meaning.
__device__ inline int2 locate(const SlotChunk &c, int p) {
    int j = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int e = __shfl(c.excl, j + step, 64);
        if (e <= p) j += step;
    }
    const int q = __shfl(c.q, j, 64);
    const int u = __shfl(c.ybeg, j, 64) + (p - __shfl(c.excl, j, 64));
    return make_int2(q, u);
}

// Rows with ub <= small cap, one wave per row (4 per workgroup): every product
// of the row is enumerated flat across the wave's lanes (a chunk of up to 64
// inner slots at a time), so the row's loads do not queue behind one another
// slot by slot.  mode 0: cnt[i] = the row's distinct output columns.  mode 1:
// the sorted columns at ccol + crowptr[i], and each output block's pair list
// (pairs at prow[i] ..., block t's from pairptr[t]) in ascending inner index:
// products are counted per block, the counts scanned, and then placed in flat
// order 64 at a time, each lane after the lanes before it in the same step
// that feed the same block (a Y row feeds a block at most once).
__global__ __launch_bounds__(256) void k_symbolic_flat(const int *__restrict__ xrowptr, const int *__restrict__ xcol,
                                                      const int *__restrict__ xdiag, const int *__restrict__ yrowptr,
                                                      const int *__restrict__ ycol, int m, const int *__restrict__ ub,
                                                      int small_cap, int mode, int *__restrict__ cnt,
                                                      const int *__restrict__ crowptr, int *__restrict__ ccol,
                                                      const int *__restrict__ prow, int *__restrict__ pairptr,
                                                      int2 *__restrict__ pairs) {
    __shared__ int tables[4][kHashSmall];
    __shared__ int lists[4][kHashSmall / 2];
    __shared__ int counts[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *table = tables[w];
    int *list = lists[w];
    if (mode == 1 && blockIdx.x == 0 && threadIdx.x == 0) pairptr[crowptr[m]] = prow[m];   // end of the last list
    for (int i0 = blockIdx.x * 4; i0 < m; i0 += gridDim.x * 4) {
        const int i = i0 + w;
        const bool active = i < m && ub[i] <= small_cap;
        // table of the next power of two >= 2 ub slots (at least one per lane)
        int slots = kWave;
        if (active)
            while (slots < 2 * ub[i]) slots <<= 1;
        for (int t = lane; t < slots; t += kWave) table[t] = kEmpty;
        if (lane == 0) counts[w] = 0;
        wave_sync();   // (every LDS array here is the wave's own)
        int q0 = 0, nk = 0, dslot = -1, dcol = 0;
        if (active) {
            q0 = xrowptr[i];
            const int q1 = xrowptr[i + 1];
            nk = q1 - q0;
            if (xdiag) {
                dcol = xdiag[i];
                dslot = identity_slot(xcol, q0, q1, dcol);
                ++nk;
            }
        }
        int added = 0;
        for (int base = 0; base < nk; base += kWave) {
            const SlotChunk c = load_slots(base, nk, q0, dslot, dcol, xcol, yrowptr, lane);
            for (int r0 = 0; r0 < c.total; r0 += kWave) {
                const int p = r0 + lane;
                const int2 pr = locate(c, p);
                if (p < c.total) added += hash_insert(table, slots - 1, ycol[pr.y]) ? 1 : 0;
            }
        }
        wave_sync();
        if (mode == 0) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o, kWave);
            if (active && lane == 0) cnt[i] = added;
        } else {
            for (int t = lane; t < slots; t += kWave) {
                const int k = table[t];
                if (active && k != kEmpty) list[atomicAdd(&counts[w], 1)] = k;
            }
            wave_sync();
            const int n = active ? counts[w] : 0;
            // the sorted columns go to ccol and to the table's first n slots
            int *sorted = table;
            int *off = table + kHashSmall / 2;
            const int c0 = active ? crowptr[i] : 0;
            wave_sort(list, n, kHashSmall / 2, lane);
            for (int a = lane; a < n; a += kWave) {
                sorted[a] = list[a];
                ccol[c0 + a] = list[a];
            }
            for (int a = lane; a < n; a += kWave) off[a] = 0;
            wave_sync();
            // products per output block, then their offsets
            for (int base = 0; base < nk; base += kWave) {
                const SlotChunk c = load_slots(base, nk, q0, dslot, dcol, xcol, yrowptr, lane);
                for (int r0 = 0; r0 < c.total; r0 += kWave) {
                    const int p = r0 + lane;
                    const int2 pr = locate(c, p);
                    if (p < c.total) atomicAdd(&off[find_pos(sorted, n, ycol[pr.y])], 1);
                }
            }
            wave_sync();
            int carry = 0;
            for (int base = 0; base < n; base += kWave) {
                const int v = base + lane < n ? off[base + lane] : 0;
                const int x = wave_incl_scan(v);
                if (base + lane < n) off[base + lane] = carry + x - v;
                carry += __builtin_amdgcn_readlane(x, 63);
            }
            wave_sync();
            const int P0 = active ? prow[i] : 0;
            for (int a = lane; a < n; a += kWave) pairptr[c0 + a] = P0 + off[a];
            wave_sync();
            for (int base = 0; base < nk; base += kWave) {
                const SlotChunk c = load_slots(base, nk, q0, dslot, dcol, xcol, yrowptr, lane);
                for (int r0 = 0; r0 < c.total; r0 += kWave) {
                    const int p = r0 + lane;
                    int pos = -1;
                    const int2 pr = locate(c, p);
                    if (p < c.total) pos = find_pos(sorted, n, ycol[pr.y]);
                    int rank = 0;
                    for (int l = 0; l < kWave; ++l) {
                        const int pl = __builtin_amdgcn_readlane(pos, l);   // (l is the same in every lane)
                        rank += (l < lane && pl == pos) ? 1 : 0;
                    }
                    if (pos >= 0) pairs[P0 + off[pos] + rank] = pr;
                    wave_sync();
                    if (pos >= 0) atomicAdd(&off[pos], 1);
                    wave_sync();
                }
            }
        }
        wave_sync();
    }
}

// C[t] entry (a,b) = fma chain over the pairs of block t (ascending inner index)
// and c ascending, from +0; identity pairs add Y's entry plainly.  One thread
// per (output block, block row a) keeps the row's bs accumulators in registers
// and reads contiguous rows of X and Y.
template <int BS>
__global__ __launch_bounds__(256) void k_spgemm_pairs(int64_t nnz, int bs_rt, const int *__restrict__ pairptr,
                                                     const int2 *__restrict__ pairs, const double *__restrict__ X,
                                                     const double *__restrict__ Y, double *__restrict__ C) {
    constexpr int NB = BS > 0 ? BS : kMaxBs;
    const int bs = BS > 0 ? BS : bs_rt;
    const int bb = bs * bs;
    const int64_t total = nnz * bs;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bs;
        const int a = static_cast<int>(g - t * bs);
        double acc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = 0.0;
        for (int k = pairptr[t]; k < pairptr[t + 1]; ++k) {
            const int2 pr = pairs[k];
            const double *y = Y + static_cast<int64_t>(pr.y) * bb;
            if (pr.x < 0) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (BS > 0 || b < bs) acc[b] = acc[b] + y[a * bs + b];
            } else {
                const double *x = X + static_cast<int64_t>(pr.x) * bb + a * bs;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (BS == 0 && c >= bs) break;
                    const double xc = x[c];
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        if (BS > 0 || b < bs) acc[b] = __builtin_fma(xc, y[c * bs + b], acc[b]);
                }
            }
        }
        double *out = C + t * bb + a * bs;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (BS > 0 || b < bs) out[b] = acc[b];
    }
}

// The same sums on the matrix cores (bs 9, 16, 25; mfma_tile.h).  One wave
// holds one output block in 16x16 FP64 accumulator tiles; each pair adds
// ceil(bs/4) 16x16x4 steps per tile over c = 4q .. 4q+3, zero beyond bs.  A
// 16x16x4 FP64 step updates each entry as the fma chain over its four c in
// ascending order, so the sums are the per-thread chains above (padding adds
// exact zeros); identity pairs add Y's entries plainly, in their place in the
// pair order.  The block is written as 0 + the accumulator.
//
// A pair's two blocks are read with consecutive lanes on consecutive words
// (ceil(bs^2/64) loads per lane and block), written to the wave's LDS slot,
// and the fragments taken from there.  The sums are short (a few pairs per
// block), so a wave that started each block from its index would wait on
// three dependent loads per block (the pair range, the pair, the blocks):
// instead each workgroup owns a contiguous range of output blocks, its four
// waves take every fourth block of it, and each wave keeps ahead of itself --
// the pair range two blocks on, the pair indices of the next block, and the
// next pair's blocks (of this block or the next) in registers while the
// current pair's steps run.  Also writes each block's max-abs size and the bit
// mask of its nonzero rows (knorm == nullptr: neither).
// lane src's pair (src the same in every lane: a read of one lane's registers)
__device__ inline int2 shfl_pair(int2 v, int src) {
    return int2{__builtin_amdgcn_readlane(v.x, src), __builtin_amdgcn_readlane(v.y, src)};
}

template <int BS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_pair_sums(
    int64_t nnz, int64_t per_wg, const int *__restrict__ pairptr, const int2 *__restrict__ pairs,
    const double *__restrict__ X, const double *__restrict__ Y, const double *__restrict__ Y2,
    double *__restrict__ K, double *__restrict__ knorm, uint32_t *__restrict__ kmask) {
    constexpr int BB = BS * BS;
    constexpr int NL = (BB + 63) / 64;   // loads per lane and block
    constexpr int NT = MfmaShape<BS>::NT, KQ = MfmaShape<BS>::KQ;
    __shared__ double slot[4][2 * BB];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * per_wg;
    const int64_t hi = lo + per_wg < nnz ? lo + per_wg : nnz;
    int64_t t = lo + w;
    if (t >= hi) return;   // whole waves; no workgroup barrier below
    double *xs = slot[w], *ys = slot[w] + BB;
    double xv[NL], yv[NL];
    auto load = [&](const int2 q) {
        // (a pair's y < 0 names block -y-1 of the second store)
        const double *y = q.y >= 0 ? Y + static_cast<int64_t>(q.y) * BB : Y2 + static_cast<int64_t>(-q.y - 1) * BB;
        // (an identity pair's x is never read: it loads its y block again, so that every
        // load is unconditional -- as are the words past the block, read from its last)
        const double *x = q.x >= 0 ? X + static_cast<int64_t>(q.x) * BB : y;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = lane + 64 * i < BB ? lane + 64 * i : BB - 1;
            yv[i] = y[e];
            xv[i] = x[e];
        }
    };
    auto chunk = [&](int from, int end) { return from + lane < end ? pairs[from + lane] : int2{0, 0}; };
    // this block: pair range and the first 64 pair indices
    int pb = pairptr[t], pe = pairptr[t + 1];
    int2 cp = chunk(pb, pe);
    // the next block: range and pair indices; the one after: range
    int64_t tn = t + 4;
    int npb = 0, npe = 0;
    if (tn < hi) {
        npb = pairptr[tn];
        npe = pairptr[tn + 1];
    }
    int2 ncp = tn < hi ? chunk(npb, npe) : int2{0, 0};
    int64_t tnn = tn + 4;
    int nnpb = 0, nnpe = 0;
    if (tnn < hi) {
        nnpb = pairptr[tnn];
        nnpe = pairptr[tnn + 1];
    }
    bool pend = false;   // xv / yv hold (or are loading) the next pair to run
    for (;;) {
        const int cnt = pe - pb;
        MfmaAcc<BS> acc;
        acc.zero();
        for (int j = 0; j < cnt; ++j) {
            if (j > 0 && (j & 63) == 0) cp = chunk(pb + j, pe);   // (more than 64 pairs: the next 64)
            const int2 pr = shfl_pair(cp, j & 63);
            if (!pend) load(pr);
            // this pair's blocks to LDS (the previous pair's fragment reads were issued before)
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int e = lane + 64 * i;
                if (e < BB) {
                    xs[e] = xv[i];
                    ys[e] = yv[i];
                }
            }
            pend = false;
            // the following pair's blocks load while this pair's steps run
            if (j + 1 < cnt) {
                if (((j + 1) & 63) != 0) {
                    load(shfl_pair(cp, (j + 1) & 63));
                    pend = true;
                }
            } else if (tn < hi && npe > npb) {
                load(shfl_pair(ncp, 0));
                pend = true;
            }
            if (pr.x < 0) {   // identity pair: Y's entries added plainly
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = 16 * ti + kk + 4 * r, jj = 16 * tj + row;
                            if (i < BS && jj < BS) acc.t[ti][tj][r] = acc.t[ti][tj][r] + ys[i * BS + jj];
                        }
            } else {
#pragma unroll
                for (int q = 0; q < KQ; ++q) {
                    const int c = 4 * q + kk;
                    double a[NT], b[NT];
#pragma unroll
                    for (int u = 0; u < NT; ++u) {
                        const int i = 16 * u + row;
                        a[u] = (i < BS && c < BS) ? xs[i * BS + c] : 0.0;
                        b[u] = (i < BS && c < BS) ? ys[c * BS + i] : 0.0;
                    }
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                        for (int tj = 0; tj < NT; ++tj)
                            acc.t[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc.t[ti][tj], 0, 0, 0);
                    // (one step's fragments at a time: the LDS reads are not hoisted past its MFMAs)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        double *out = K + t * BB;
        double m = 0.0;
        uint32_t bits = 0u;
        mfma_for_entries<BS>(acc, row, kk, [&](int i, int jj, double v) {
            const double o = 0.0 + v;
            out[i * BS + jj] = o;
            m = fmax(m, fabs(o));
            if (o != 0.0) bits |= 1u << i;
        });
        if (knorm) {   // (a plain sparse product takes no sizes)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                m = fmax(m, __shfl_xor(m, o, 64));
                bits |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(bits), o, 64));
            }
            if (lane == 0) {
                knorm[t] = m;
                kmask[t] = bits;
            }
        }
        // on to the next block
        t = tn;
        if (t >= hi) break;
        pb = npb;
        pe = npe;
        cp = ncp;
        tn = tnn;
        npb = nnpb;
        npe = nnpe;
        ncp = tn < hi ? chunk(npb, npe) : int2{0, 0};
        tnn = tn + 4;
        if (tnn < hi) {
            nnpb = pairptr[tnn];
            nnpe = pairptr[tnn + 1];
        }
    }
}

// Sums of pair lists for nnz output blocks on the matrix cores (bs 9, 16, 25).
void launch_pair_sums(int bs, int64_t nnz, const int *pairptr, const int2 *pairs, const double *X, const double *Y,
                      const double *Y2, double *K, double *knorm, uint32_t *kmask, hipStream_t s) {
    if (nnz <= 0) return;
    // up to 24,576 workgroups of contiguous ranges: each wave still runs through several
    // blocks with the next ones in flight, and the chains are short enough that the tail
    // balances (at 25 x 25 blocks 12k-36k workgroups all did best, 3,072 1.4% worse)
    const int64_t nwg = std::min<int64_t>((nnz + 3) / 4, 24576);
    const int64_t per_wg = (nnz + nwg - 1) / nwg;
    const int64_t grid = (nnz + per_wg - 1) / per_wg;
    if (bs == 9)
        k_pair_sums<9><<<static_cast<unsigned>(grid), 256, 0, s>>>(nnz, per_wg, pairptr, pairs, X, Y, Y2, K, knorm,
                                                                   kmask);
    else if (bs == 16)
        k_pair_sums<16><<<static_cast<unsigned>(grid), 256, 0, s>>>(nnz, per_wg, pairptr, pairs, X, Y, Y2, K, knorm,
                                                                    kmask);
    else if (bs == 25)
        k_pair_sums<25><<<static_cast<unsigned>(grid), 256, 0, s>>>(nnz, per_wg, pairptr, pairs, X, Y, Y2, K, knorm,
                                                                    kmask);
    else
        fail(NAIR_EDEVICE, "launch_pair_sums: matrix-core block sizes only");
    NAIR_HIP(hipGetLastError());
}

// out[t] = in[src[t]] for t < *count
__global__ __launch_bounds__(256) void k_gather_mask(int64_t n, const uint32_t *__restrict__ in,
                                                    const int *__restrict__ src, const int *__restrict__ count,
                                                    uint32_t *__restrict__ out) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < n && t < *count) out[t] = in[src[t]];
}

// ---------------------------------------------------- Galerkin merge lists

__global__ __launch_bounds__(256) void k_rap_count_contrib(const int *__restrict__ rarp, const int *__restrict__ racol,
                                                          const int *__restrict__ pmap, int m, int *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int c = 0;
    for (int u = rarp[i]; u < rarp[i + 1]; ++u) c += (pmap[racol[u]] >= 0) ? 1 : 0;
    cnt[i] = c;
}

// For K's row i: the RA blocks of row i merged into each K block, in ascending
// RA column.  One 64-thread workgroup per row (rows have <= 1024 RA blocks).
__global__ __launch_bounds__(64) void k_rap_contrib(const int *__restrict__ rarp, const int *__restrict__ racol,
                                                   const int *__restrict__ pmap, int m, const int *__restrict__ krp,
                                                   const int *__restrict__ kcol, const int *__restrict__ crow,
                                                   int *__restrict__ kptr, int *__restrict__ klist) {
    __shared__ int kc[kHashSmall / 2];
    __shared__ int off[kHashSmall / 2];
    const int lane = threadIdx.x;
    if (blockIdx.x == 0 && lane == 0) kptr[krp[m]] = crow[m];   // the end of the last block's list
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const int r0 = rarp[i], nra = rarp[i + 1] - r0;
        const int k0 = krp[i], nk = krp[i + 1] - k0;
        const int R0 = crow[i];
        for (int p = lane; p < nk; p += 64) {
            kc[p] = kcol[k0 + p];
            off[p] = 0;
        }
        __syncthreads();
        for (int u = lane; u < nra; u += 64) {
            const int t = pmap[racol[r0 + u]];
            if (t >= 0) atomicAdd(&off[find_pos(kc, nk, t)], 1);
        }
        __syncthreads();
        wave0_scan(off, nk);
        __syncthreads();
        for (int p = lane; p < nk; p += 64) kptr[k0 + p] = R0 + off[p];
        __syncthreads();
        for (int u0 = 0; u0 < nra; u0 += 64) {
            const int u = u0 + lane;
            int p = -1;
            if (u < nra) {
                const int t = pmap[racol[r0 + u]];
                if (t >= 0) p = find_pos(kc, nk, t);
            }
            int rank = 0;
            for (int l = 0; l < 64; ++l) {
                const int pl = __builtin_amdgcn_readlane(p, l);   // (l is the same in every lane)
                rank += (l < lane && pl == p) ? 1 : 0;
            }
            if (p >= 0) klist[R0 + off[p] + rank] = r0 + u;
            __syncthreads();
            if (p >= 0) atomicAdd(&off[p], 1);
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(256) void k_rap_values(int64_t nnz, int bb, const int *__restrict__ kptr,
                                                   const int *__restrict__ klist, const double *__restrict__ RA,
                                                   double *__restrict__ K) {
    const int64_t total = nnz * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bb;
        const int e = static_cast<int>(g - t * bb);
        double s = 0.0;
        for (int k = kptr[t]; k < kptr[t + 1]; ++k) s = s + RA[static_cast<int64_t>(klist[k]) * bb + e];
        K[g] = s;
    }
}

// The same with one wave per block (blocks of 64 entries or more).
__global__ __launch_bounds__(256) void k_rap_values_wave(int64_t nnz, int bb, const int *__restrict__ kptr,
                                                        const int *__restrict__ klist, const double *__restrict__ RA,
                                                        double *__restrict__ K) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; t < nnz; t += stride) {
        const int k0 = kptr[t], k1 = kptr[t + 1];
        for (int e = lane; e < bb; e += 64) {
            double v = 0.0;
            for (int k = k0; k < k1; ++k) v = v + RA[static_cast<int64_t>(klist[k]) * bb + e];
            K[t * bb + e] = v;
        }
    }
}

// A P blocks with one contributor are that A block itself; the others (flag 1)
// are summed into a second store.  ymap[t]: the A block, or -(merged index)-1.
__global__ __launch_bounds__(256) void k_ap_flags(int64_t nnz, const int *__restrict__ kptr, int *__restrict__ flag) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < nnz) flag[t] = (kptr[t + 1] - kptr[t] > 1) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_ap_map(int64_t nnz, const int *__restrict__ kptr,
                                               const int *__restrict__ klist, const int *__restrict__ midx,
                                               int *__restrict__ ymap, int *__restrict__ mblk) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    if (kptr[t + 1] - kptr[t] > 1) {
        ymap[t] = -midx[t] - 1;
        mblk[midx[t]] = static_cast<int>(t);
    } else {
        ymap[t] = klist[kptr[t]];
    }
}

// merged block q = sum of A P block mblk[q]'s contributors, one wave per block
// (NCH: 64-word chunks that cover a block, at most 16 for bs <= 32)
template <int NCH>
__global__ __launch_bounds__(256) void k_ap_merged(int nm, int bb, const int *__restrict__ mblk,
                                                  const int *__restrict__ kptr, const int *__restrict__ klist,
                                                  const double *__restrict__ A, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t q = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; q < nm; q += stride) {
        const int t = mblk[q];
        const int k0 = kptr[t], k1 = kptr[t + 1];
        // contributors outermost, two at a time: their entries load together (one wait
        // per two contributors, not per entry); every entry still sums its contributors
        // in order.  (Words past a block repeat its last, unused.)
        constexpr int kChunks = NCH;
        double v[kChunks];
#pragma unroll
        for (int i = 0; i < kChunks; ++i) v[i] = 0.0;
        int k = k0;
        for (; k + 1 < k1; k += 2) {
            const double *a0 = A + static_cast<int64_t>(klist[k]) * bb;
            const double *a1 = A + static_cast<int64_t>(klist[k + 1]) * bb;
            double u0[kChunks], u1[kChunks];
#pragma unroll
            for (int i = 0; i < kChunks; ++i) {
                const int e = lane + 64 * i < bb ? lane + 64 * i : bb - 1;
                u0[i] = a0[e];
                u1[i] = a1[e];
            }
#pragma unroll
            for (int i = 0; i < kChunks; ++i) v[i] = (v[i] + u0[i]) + u1[i];
        }
        if (k < k1) {
            const double *a = A + static_cast<int64_t>(klist[k]) * bb;
#pragma unroll
            for (int i = 0; i < kChunks; ++i) {
                const int e = lane + 64 * i;
                if (e < bb) v[i] = v[i] + a[e];
            }
        }
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const int e = lane + 64 * i;
            if (e < bb) out[q * bb + e] = v[i];
        }
    }
}

// pairs[k].x = xmap[pairs[k].x] where x >= 0 (identity pairs keep x < 0)
__global__ __launch_bounds__(256) void k_remap_x(int64_t n, const int *__restrict__ xmap, int2 *__restrict__ pairs) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = pairs[k].x;
    if (x >= 0) pairs[k].x = xmap[x];
}

__global__ __launch_bounds__(256) void k_remap_y(int64_t n, const int *__restrict__ ymap, int2 *__restrict__ pairs) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n) pairs[p].y = ymap[pairs[p].y];
}

// Drop filter: keep the diagonal and blocks with size > drop * size(diagonal).
// One wave per row, its lanes over the row's blocks.
__global__ __launch_bounds__(256) void k_drop_mark(const int *__restrict__ krp, const int *__restrict__ kcol,
                                                  const double *__restrict__ knorm, int m, double drop,
                                                  uint8_t *__restrict__ keep, int *__restrict__ kept,
                                                  int *__restrict__ margin) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + static_cast<int>(threadIdx.x >> 6);
    if (i >= m) return;   // whole waves
    const int lo = krp[i], hi = krp[i + 1];
    double dn = 0.0;   // the diagonal block's size (0 if the row has none)
    for (int base = lo; base < hi; base += 64) {
        const int t = base + lane;
        const bool isd = t < hi && kcol[t] == i;
        const double v = isd ? knorm[t] : 0.0;
        const unsigned long long b = __ballot(isd);
        if (b != 0ull) {
            dn = __shfl(v, static_cast<int>(__builtin_ctzll(b)), 64);
            break;
        }
    }
    const double thr = drop * dn;
    int c = 0, nties = 0;
    for (int t = lo + lane; t < hi; t += 64) {
        const bool diag = kcol[t] == i;
        const double kn = knorm[t];
        const bool k = diag || (kn > thr);
        keep[t] = k ? 1 : 0;
        c += k ? 1 : 0;
        // audit: the two sides of the drop test within 1e-12 relative
        if (!diag && fabs(kn - thr) <= 1e-12 * fmax(fabs(kn), fabs(thr))) ++nties;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        nties += __shfl_xor(nties, o, 64);
    }
    if (lane == 0) {
        kept[i] = c;
        if (nties) atomicAdd(margin + 3, nties);
    }
}


}  // namespace

#define NAIR_BS_DISPATCH(bs, KERNEL, ...)            \
    switch (bs) {                                    \
        case 2: KERNEL<2> __VA_ARGS__; break;        \
        case 3: KERNEL<3> __VA_ARGS__; break;        \
        case 4: KERNEL<4> __VA_ARGS__; break;        \
        case 6: KERNEL<6> __VA_ARGS__; break;        \
        case 9: KERNEL<9> __VA_ARGS__; break;        \
        case 10: KERNEL<10> __VA_ARGS__; break;      \
        case 16: KERNEL<16> __VA_ARGS__; break;      \
        case 25: KERNEL<25> __VA_ARGS__; break;      \
        default: KERNEL<0> __VA_ARGS__; break;       \
    }

namespace {

// The pair lists of a product's blocks (pairs[pairptr[t]] ... for block t).
struct Pairs {
    DBuf<int> pairptr;
    DBuf<int2> pairs;
    int64_t n = 0;   // pairs
};

// C's pattern (rowptr, colidx, nnzb) and the pair lists of its blocks; C.vals
// is left unallocated.
void spgemm_structure(const DevBSR &X, const int *xdiag, const DevBSR &Y, DevBSR &C, Pairs &P, hipStream_t s) {
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
        return;
    }
    const int small_cap = kHashSmall / 2, large_cap = kHashLarge / 2;
    // flags: big-row count, too-dense row, then the scans' totals (nnz, pairs), read in one copy
    DBuf<int> ub(m), cnt(m), big_list(m), flags(4), prow(static_cast<size_t>(m) + 1);
    NAIR_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int) * 2, s));
    int *big_count = flags.get(), *too_dense = flags.get() + 1;
    k_row_upper_bound<<<grid_for(m, 256), 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), m,
                                                      ub.get(), small_cap, big_list.get(), big_count, large_cap,
                                                      too_dense);
    const unsigned gs = cap_grid((m + 3) / 4);
    const size_t lds_large = sizeof(int) * (kHashLarge + kHashLarge / 2);
    k_symbolic_flat<<<gs, 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), Y.colidx.get(), m,
                                       ub.get(), small_cap, 0, cnt.get(), nullptr, nullptr, nullptr, nullptr, nullptr);
    {
        TimerScope ts(TK_SPGEMM_SYM, g_timer_level, s);
        k_symbolic_large<<<256, 256, lds_large, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(),
                                                     Y.colidx.get(), big_list.get(), big_count, large_cap, 0,
                                                     cnt.get(), nullptr, nullptr, ub.get());
    }
    NAIR_HIP(hipGetLastError());
    scan_exclusive2(cnt.get(), C.rowptr.get(), m, flags.get() + 2, ub.get(), prow.get(), m, flags.get() + 3, s);
    int hflags[4] = {0, 0, 0, 0};
    read_ints(flags.get(), hflags, 4, s);
    const int nnz = hflags[2], npairs = hflags[3];
    if (hflags[1] > 0)
        fail(NAIR_ENOMEM, "sparse product row has " + std::to_string(hflags[1]) + " candidate blocks (limit " +
                              std::to_string(large_cap) + ")");
    C.nnzb = nnz;
    C.colidx.alloc(nnz);
    if (nnz == 0) return;
    P.pairptr.alloc(static_cast<size_t>(nnz) + 1);
    P.pairs.alloc(npairs);
    P.n = npairs;
    k_symbolic_flat<<<gs, 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), Y.colidx.get(), m,
                                       ub.get(), small_cap, 1, nullptr, C.rowptr.get(), C.colidx.get(), prow.get(),
                                       P.pairptr.get(), P.pairs.get());
    if (hflags[0] > 0)
        k_symbolic_large<<<256, 256, lds_large, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(),
                                                     Y.colidx.get(), big_list.get(), big_count, large_cap, 1, nullptr,
                                                     C.rowptr.get(), C.colidx.get(), ub.get());
    if (hflags[0] > 0)
        k_pairs_large<<<256, 256, 0, s>>>(X.rowptr.get(), X.colidx.get(), xdiag, Y.rowptr.get(), Y.colidx.get(),
                                          big_list.get(), big_count, C.rowptr.get(), C.colidx.get(), prow.get(),
                                          P.pairptr.get(), P.pairs.get());
    NAIR_HIP(hipGetLastError());
}

// C's values from its pair lists (C.vals allocated by the caller).
void spgemm_values(const double *xvals, const DevBSR &Y, const Pairs &P, DevBSR &C, hipStream_t s) {
    const int64_t nnz = C.nnzb;
    const int bs = C.bs;
    if (nnz == 0) return;
    const int64_t total = nnz * bs;
    const unsigned grid = cap_grid((total + 255) / 256);
    TimerScope ts(TK_SPGEMM_NUM, g_timer_level, s);
    if (use_matrix_cores(bs)) {
        launch_pair_sums(bs, nnz, P.pairptr.get(), P.pairs.get(), xvals, Y.vals.get(), nullptr, C.vals.get(), nullptr,
                         nullptr, s);
    } else {
        NAIR_BS_DISPATCH(bs, k_spgemm_pairs, <<<grid, 256, 0, s>>>(nnz, bs, P.pairptr.get(), P.pairs.get(), xvals,
                                                                   Y.vals.get(), C.vals.get()));
    }
    NAIR_HIP(hipGetLastError());
}

}  // namespace

void spgemm(const DevBSR &X, const int *xdiag, const DevBSR &Y, DevBSR &C, hipStream_t s, const double *xvals,
            const int *xmap) {
    Pairs P;
    spgemm_structure(X, xdiag, Y, C, P, s);
    if (xmap && P.n > 0) {   // X's block x is block xmap[x] of xvals
        k_remap_x<<<grid_for(P.n, 256), 256, 0, s>>>(P.n, xmap, P.pairs.get());
        NAIR_HIP(hipGetLastError());
    }
    C.vals.alloc(static_cast<size_t>(C.nnzb) * C.bs * C.bs);
    spgemm_values(xmap ? xvals : X.vals.get(), Y, P, C, s);
}

void bsr_add(const DevBSR &S, const DevBSR &W, DevBSR &O, hipStream_t s, DBuf<int> *srcS_out, DBuf<int> *srcW_out) {
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
    // the union has at most the two counts together; the exact count stays on the device
    const int64_t cap = S.bound() + W.bound();
    O.nnzb = -1;
    O.cap = cap;
    O.colidx.alloc(static_cast<size_t>(cap));
    const bool pattern_only = srcS_out && srcW_out;
    if (!pattern_only) O.vals.alloc(static_cast<size_t>(cap) * bs * bs);
    if (cap == 0 || m == 0) return;
    DBuf<int> srcS(static_cast<size_t>(cap)), srcW(static_cast<size_t>(cap));
    k_add_fill<<<grid_for(m, 256), 256, 0, s>>>(S.rowptr.get(), S.colidx.get(), W.rowptr.get(), W.colidx.get(), m,
                                                O.rowptr.get(), O.colidx.get(), srcS.get(), srcW.get());
    if (pattern_only) {
        NAIR_HIP(hipGetLastError());
        *srcS_out = std::move(srcS);
        *srcW_out = std::move(srcW);
        return;
    }
    const int64_t total = cap * bs * bs;
    if (bs * bs >= 64)
        k_add_values_wave<<<cap_grid((cap + 3) / 4), 256, 0, s>>>(O.rowptr.get() + m, bs * bs, S.vals.get(),
                                                                   srcS.get(), W.vals.get(), srcW.get(), O.vals.get());
    else
        k_add_values<<<cap_grid((total + 255) / 256), 256, 0, s>>>(O.rowptr.get() + m, bs * bs, S.vals.get(),
                                                                  srcS.get(), W.vals.get(), srcW.get(), O.vals.get());
    NAIR_HIP(hipGetLastError());
}

namespace {

// AP = A P for one-point P: A's columns merged through pmap, each AP block the
// sum of its A blocks in ascending column (from +0).  Z's block count comes
// back with the same read when it is still on the device.  With `ymap`, only
// the blocks with several contributors are summed (into `merged`); ymap[t]
// names block t's values: A's block, or -(merged index)-1 (a lone block is
// its A block, up to the sign of a zero entry).
void merge_columns(const DevBSR &A, const int *pmap, int nc, DevBSR &Z, DevBSR &AP, hipStream_t s,
                   DBuf<int> *ymap = nullptr, DBuf<double> *merged = nullptr) {
    const int m = A.nb, bs = A.bs, bb = bs * bs;
    AP.nb = m;
    AP.ncols = nc;
    AP.bs = bs;
    DBuf<int> cnt(m), ccnt(m), crow(static_cast<size_t>(m) + 1), flags(3);
    AP.rowptr.alloc(static_cast<size_t>(m) + 1);
    NAIR_HIP(hipMemsetAsync(flags.get(), 0, sizeof(int), s));
    const unsigned gs = cap_grid((m + 3) / 4);
    k_rap_symbolic<<<gs, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), pmap, m, 0, cnt.get(), nullptr, nullptr,
                                      flags.get());
    k_rap_count_contrib<<<grid_for(m, 256), 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), pmap, m, ccnt.get());
    NAIR_HIP(hipGetLastError());
    scan_exclusive2(cnt.get(), AP.rowptr.get(), m, flags.get() + 1, ccnt.get(), crow.get(), m, flags.get() + 2, s);
    int hflags[3] = {0, 0, 0};
    int zcount = 0;
    const bool zdev = Z.nnzb < 0;
    read_device({{flags.get(), hflags, sizeof(int) * 3},
                 {zdev ? Z.rowptr.get() + Z.nb : nullptr, &zcount, zdev ? sizeof(int) : 0}},
                s);
    if (zdev) Z.nnzb = zcount;
    if (hflags[0] > 0)
        fail(NAIR_ENOMEM, "operator row has " + std::to_string(hflags[0]) + " blocks (limit " +
                              std::to_string(kHashSmall / 2) + ")");
    const int nnz = hflags[1], ncontrib = hflags[2];
    AP.nnzb = nnz;
    AP.colidx.alloc(static_cast<size_t>(nnz));
    if (!ymap) AP.vals.alloc(static_cast<size_t>(nnz) * bb);
    if (nnz == 0) return;
    DBuf<int> kptr(static_cast<size_t>(nnz) + 1), klist(static_cast<size_t>(ncontrib));
    k_rap_symbolic<<<gs, 256, 0, s>>>(A.rowptr.get(), A.colidx.get(), pmap, m, 1, nullptr, AP.rowptr.get(),
                                      AP.colidx.get(), flags.get());
    k_rap_contrib<<<cap_grid(m), 64, 0, s>>>(A.rowptr.get(), A.colidx.get(), pmap, m, AP.rowptr.get(),
                                             AP.colidx.get(), crow.get(), kptr.get(), klist.get());
    if (ymap) {
        DBuf<int> flag(static_cast<size_t>(nnz)), midx(static_cast<size_t>(nnz) + 1);
        k_ap_flags<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, kptr.get(), flag.get());
        scan_exclusive(flag.get(), midx.get(), nnz, s);
        const int nm = read_int(midx.get() + nnz, s);
        ymap->alloc(static_cast<size_t>(nnz));
        merged->alloc(static_cast<size_t>(std::max(nm, 1)) * bb);
        DBuf<int> mblk(static_cast<size_t>(std::max(nm, 1)));
        k_ap_map<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, kptr.get(), klist.get(), midx.get(), ymap->get(), mblk.get());
        if (nm > 0) {
            // the instance for blocks of at most 64, 128, 256 or 640 entries, else 16 chunks
            void (*kern)(int, int, const int *, const int *, const int *, const double *, double *) = k_ap_merged<16>;
            switch ((bb + 63) / 64) {
                case 1: kern = k_ap_merged<1>; break;
                case 2: kern = k_ap_merged<2>; break;
                case 4: kern = k_ap_merged<4>; break;
                case 10: kern = k_ap_merged<10>; break;
                default: break;
            }
            kern<<<cap_grid((static_cast<int64_t>(nm) + 3) / 4), 256, 0, s>>>(nm, bb, mblk.get(), kptr.get(),
                                                                             klist.get(), A.vals.get(), merged->get());
        }
        NAIR_HIP(hipGetLastError());
        return;
    }
    if (bb >= 64)
        k_rap_values_wave<<<cap_grid((static_cast<int64_t>(nnz) + 3) / 4), 256, 0, s>>>(nnz, bb, kptr.get(),
                                                                                      klist.get(), A.vals.get(),
                                                                                      AP.vals.get());
    else
        k_rap_values<<<cap_grid((static_cast<int64_t>(nnz) * bb + 255) / 256), 256, 0, s>>>(
            nnz, bb, kptr.get(), klist.get(), A.vals.get(), AP.vals.get());
    NAIR_HIP(hipGetLastError());
}

}  // namespace

void galerkin(DevBSR &Z, const int *cpts, const DevBSR &A, const int *pmap, int nc, double drop, DevBSR &K,
              int *margin, DBuf<double> &knext, DBuf<uint32_t> &kmask, hipStream_t s) {
    // A P first (P is one unit block per row: a merge of A's columns), then
    // K = R (A P) with R = [Z I]: its pattern and pair lists, and each block's
    // sum on the matrix cores (with its size and row mask) or by pairs
    const int bs = A.bs;
    const int bb = bs * bs;
    const bool fused = use_matrix_cores(bs);
    DevBSR AP;
    DBuf<int> ymap;
    DBuf<double> merged;
    merge_columns(A, pmap, nc, Z, AP, s, fused ? &ymap : nullptr, fused ? &merged : nullptr);
    DevBSR RK;
    Pairs P;
    spgemm_structure(Z, cpts, AP, RK, P, s);
    if (fused && P.n > 0) {   // the pairs name A's block or a merged block
        k_remap_y<<<grid_for(P.n, 256), 256, 0, s>>>(P.n, ymap.get(), P.pairs.get());
        NAIR_HIP(hipGetLastError());
    }
    const int m = nc;
    const int nnz = static_cast<int>(RK.nnzb);
    DBuf<double> kval, knorm(static_cast<size_t>(nnz));
    DBuf<uint32_t> kbits(fused ? nnz : 0);
    DBuf<uint8_t> keep(static_cast<size_t>(nnz));
    DBuf<int> kept(static_cast<size_t>(m));
    if (fused) {
        kval.alloc(static_cast<size_t>(nnz) * bb);
        if (nnz > 0) {
            TimerScope ts(TK_RAP, g_timer_level, s);
            launch_pair_sums(bs, nnz, P.pairptr.get(), P.pairs.get(), Z.vals.get(), A.vals.get(), merged.get(),
                             kval.get(), knorm.get(), kbits.get(), s);
        }
    } else {
        RK.vals.alloc(static_cast<size_t>(nnz) * bb);
        {
            TimerScope ts(TK_RAP, g_timer_level, s);
            spgemm_values(Z.vals.get(), AP, P, RK, s);
        }
        kval = std::move(RK.vals);
        launch_block_maxabs(kval.get(), nnz, bs, knorm.get(), s);
    }
    const int *krp = RK.rowptr.get();
    const int *kcol = RK.colidx.get();
    k_drop_mark<<<static_cast<unsigned>(std::max((m + 3) / 4, 1)), 256, 0, s>>>(krp, kcol, knorm.get(), m, drop,
                                                                               keep.get(), kept.get(), margin);
    NAIR_HIP(hipGetLastError());
    K.nb = nc;
    K.ncols = nc;
    K.bs = bs;
    K.rowptr.alloc(static_cast<size_t>(nc) + 1);
    scan_exclusive(kept.get(), K.rowptr.get(), m, s);
    // the kept count stays on the device (the next level reads it back with its first read)
    K.nnzb = -1;
    K.cap = nnz;
    K.colidx.alloc(static_cast<size_t>(nnz));
    K.vals.alloc(static_cast<size_t>(nnz) * bb);
    knext.alloc(static_cast<size_t>(nnz));
    const int *nk = K.rowptr.get() + m;
    DBuf<int> src(static_cast<size_t>(nnz));
    k_compact_fill<<<grid_for(m, 256), 256, 0, s>>>(krp, kcol, keep.get(), m, K.rowptr.get(), K.colidx.get(),
                                                    src.get());
    NAIR_HIP(hipGetLastError());
    launch_block_gather(nnz, bs, kval.get(), src.get(), K.vals.get(), s, nk);
    launch_block_gather(nnz, 1, knorm.get(), src.get(), knext.get(), s, nk);   // a block's size is its max-abs entry
    if (fused && nnz > 0) {
        kmask.alloc(static_cast<size_t>(nnz));
        k_gather_mask<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, kbits.get(), src.get(), nk, kmask.get());
        NAIR_HIP(hipGetLastError());
    }
}

}  // namespace nair
