// Setup-phase kernels: block sizes, block-diagonal inverses, strength, C/F
// splitting, one-point interpolation and the block products of the Neumann
// restriction.  Values that feed later comparisons are computed in one fixed
// order (fma chains, c ascending), with no implicit contraction.
#include "common.h"
#include "mfma_tile.h"

#pragma clang fp contract(off)

namespace nair {
namespace {

constexpr int kWave = 64;

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// ----------------------------------------------------------- block sizes

// One pass over n blocks that gives, per block, its max-abs entry (entries that
// are NaN are ignored, as fmax ignores them), the mask of its nonzero rows and
// the mask of its nonzero columns.  L lanes share a block (L: the power of two
// >= bs*bs, at most 64), so a block's entries are read as consecutive words;
// the lanes' partial results meet by shuffles (max and or are exact, so the
// order is free).  Block t is vals[src[t]] when src is given; with count,
// blocks at or past *count are empty (zero results).  Outputs may be null;
// copy (no src, no count) receives the blocks as they are read.
__global__ __launch_bounds__(256) void k_block_scan(const double *__restrict__ vals, int64_t n, int bs, int L,
                                                   const int *__restrict__ src, const int *__restrict__ count,
                                                   double *__restrict__ maxabs, unsigned long long *__restrict__ meta,
                                                   uint32_t *__restrict__ rmask, int *__restrict__ rsize,
                                                   double *__restrict__ copy) {
    const int per = 256 / L;
    const int sub = static_cast<int>(threadIdx.x) & (L - 1);
    const int64_t t = static_cast<int64_t>(blockIdx.x) * per + static_cast<int>(threadIdx.x) / L;
    const int bb = bs * bs;
    const int64_t nn = count ? min(static_cast<int64_t>(*count), n) : n;
    double m = 0.0;
    uint32_t rm = 0u, cm = 0u;
    if (t < nn && L == kWave) {
        // a wave per block (more than 32 entries; bs <= 32, so at most 16 words per lane):
        // every load first, then the copy and the sizes -- one memory wait per block
        // instead of one per word
        constexpr int kChunks = 16;
        const double *blk = vals + (src ? static_cast<int64_t>(src[t]) : t) * bb;
        double v[kChunks];
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const int e = sub + kWave * i;
            v[i] = blk[e < bb ? e : bb - 1];   // (words past the block repeat its last, unused)
        }
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const int e = sub + kWave * i;
            if (e < bb) {
                const double x = v[i];
                if (copy) copy[t * bb + e] = x;
                if (x != 0.0) {
                    const int r = e / bs;
                    rm |= 1u << r;
                    cm |= 1u << (e - r * bs);
                }
                m = fmax(m, fabs(x));
            }
        }
    } else if (t < nn) {
        const double *blk = vals + (src ? static_cast<int64_t>(src[t]) : t) * bb;
        for (int e = sub; e < bb; e += L) {
            const double x = blk[e];
            if (copy) copy[t * bb + e] = x;
            if (x != 0.0) {
                const int r = e / bs;
                rm |= 1u << r;
                cm |= 1u << (e - r * bs);
            }
            m = fmax(m, fabs(x));
        }
    }
    for (int o = L >> 1; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o, kWave));
        rm |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(rm), o, kWave));
        cm |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(cm), o, kWave));
    }
    if (sub == 0 && t < n) {
        if (maxabs) maxabs[t] = m;
        if (meta) meta[t] = (static_cast<unsigned long long>(cm) << 32) | rm;
        if (rmask) rmask[t] = rm;
        if (rsize) rsize[t] = __popc(rm) * bs;
    }
}

// -------------------------------------------------- diagonal block inverse

// Lane-to-lane moves within groups of a half wave for the pivot search: DPP
// for the quad and row patterns, a swizzle for the two 16-lane rows.
template <int CTRL>
__device__ inline int dpp_move(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = dpp_move<CTRL>(static_cast<int>(u)), hi = dpp_move<CTRL>(static_cast<int>(u >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
constexpr int kSwizzleXor16 = 0x401F;   // bit mode: lane i of 32 reads lane i ^ 16
__device__ inline int swz16(int v) { return __builtin_amdgcn_ds_swizzle(v, kSwizzleXor16); }
__device__ inline double swz16(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = swz16(static_cast<int>(u)), hi = swz16(static_cast<int>(u >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// The same LU recipe with each block on a half wave and its rows in registers
// (bs 16 and 25).  Lane r holds row r of the block for the whole factorisation
// and tracks the position `pos` that row has in the pivoted order, so a row
// exchange is two position updates instead of moving the rows.  Step k: the
// first position >= k of largest |a_.k| wins (the largest value, then the
// smallest position among the lanes that hold it, each a reduction over the
// half by DPP and one swizzle), its lane and the lane at position k
// trade positions, the pivot row -- final from here on -- is written once to
// row k of the half's LDS factor slot, and every lane at a later position
// forms its multiplier and updates its row from that LDS row.  Lane j then
// keeps column j of the inverse in registers through the forward and back
// substitution, reading the factors from LDS (every lane of the half the same
// word), and writes row i of the inverse with consecutive lanes on
// consecutive words.  The operations and their order are those of
// k_block_inverse: the same bits.
template <int BS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_block_inverse_rows(const int *__restrict__ rowptr,
                                                           const int *__restrict__ colidx,
                                                           const double *__restrict__ vals, int nb,
                                                           const int8_t *__restrict__ skip, double *__restrict__ dinv,
                                                           int *__restrict__ singular_min) {
    static_assert(BS >= 2 && BS <= 32, "a block row per lane of a half wave");
    constexpr int BB = BS * BS;
    constexpr int kNone = (64 << 5) | 31;     // key of a lane that is no candidate
    __shared__ double slot[8][BB];
    __shared__ int8_t pslot[8][32];   // (bytes: four workgroups' slots fit one CU's LDS)
    const int h = threadIdx.x >> 5;           // half wave: one block
    const int r = threadIdx.x & 31;           // its row
    const int I = blockIdx.x * 8 + h;
    const bool on = I < nb && !(skip && skip[I]);
    // the diagonal block's position in row I
    int dpos = -1;
    if (on)
        for (int t = rowptr[I] + r; t < rowptr[I + 1]; t += 32)
            if (colidx[t] == I) dpos = t;
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) dpos = max(dpos, __shfl_xor(dpos, o, kWave));
    bool live = on && dpos >= 0;
    if (on && dpos < 0 && r == 0) atomicMin(singular_min, I);   // validated before; never taken for valid input
    double a[BS];
    {
        const double *src = vals + static_cast<int64_t>(live ? dpos : 0) * BB + (r < BS ? r : 0) * BS;
#pragma unroll
        for (int c = 0; c < BS; ++c) a[c] = (live && r < BS) ? src[c] : 0.0;
    }
    double *fac = slot[h];
    int8_t *pm = pslot[h];
    int pos = r;   // lanes r >= BS keep positions >= BS: never candidates, never updated
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        // the largest candidate |a_.k| over the half, then the smallest key (position)
        // among the lanes that hold it: the first position of the largest, as before
        const bool cand = pos >= k && pos < BS;
        const double own = cand ? fabs(a[k]) : -1.0;
        double v = own;
        v = fmax(v, dpp_move<0xB1>(v));     // quad_perm 1,0,3,2
        v = fmax(v, dpp_move<0x4E>(v));     // quad_perm 2,3,0,1
        v = fmax(v, dpp_move<0x141>(v));    // row_half_mirror
        v = fmax(v, dpp_move<0x140>(v));    // row_mirror
        v = fmax(v, swz16(v));
        int key = (cand && own == v) ? (pos << 5) | r : kNone;
        key = min(key, dpp_move<0xB1>(key));
        key = min(key, dpp_move<0x4E>(key));
        key = min(key, dpp_move<0x141>(key));
        key = min(key, dpp_move<0x140>(key));
        key = min(key, swz16(key));
        if (live && !(v > 0.0)) {
            if (r == 0) atomicMin(singular_min, I);
            live = false;
        }
        // exchange positions k and wpos (the pivot row's lane p moves to k)
        const int wpos = key >> 5, p = key & 31;
        if (pos == k)
            pos = wpos;
        else if (r == p)
            pos = k;
        if (pos == k) {
#pragma unroll
            for (int c = 0; c < BS; ++c) fac[k * BS + c] = a[c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (pos > k && pos < BS) {
            a[k] = a[k] / fac[k * BS + k];
#pragma unroll
            for (int j = k + 1; j < BS; ++j) a[j] = __builtin_fma(-a[k], fac[k * BS + j], a[j]);
        }
    }
    if (r < BS && pos < BS) pm[pos] = static_cast<int8_t>(r);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (!live || r >= BS) return;
    const int j = r;
    double y[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        double sacc = (pm[i] == j) ? 1.0 : 0.0;
#pragma unroll
        for (int mm = 0; mm < i; ++mm) sacc = __builtin_fma(-fac[i * BS + mm], y[mm], sacc);
        y[i] = sacc;
    }
#pragma unroll
    for (int i = BS - 1; i >= 0; --i) {
        double sacc = y[i];
#pragma unroll
        for (int mm = i + 1; mm < BS; ++mm) sacc = __builtin_fma(-fac[i * BS + mm], y[mm], sacc);
        y[i] = sacc / fac[i * BS + i];
    }
    double *dst = dinv + static_cast<int64_t>(I) * BB;
#pragma unroll
    for (int i = 0; i < BS; ++i) dst[i * BS + j] = y[i];
}

// One wave per block row.  LU with partial pivoting (first row of largest
// |a_ik|, whole-row exchange), multipliers by division, trailing update
// a_ij = fma(-a_ik, a_kj, a_ij); then column j of the inverse by forward
// substitution of P e_j (fma, m ascending) and back substitution (fma over
// m > i ascending, one division by u_ii).  LDS: a[bs*bs], y[bs*bs], perm[bs].
__global__ __launch_bounds__(64) void k_block_inverse(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                     const double *__restrict__ vals, int nb, int bs,
                                                     const int8_t *__restrict__ skip, double *__restrict__ dinv,
                                                     int *__restrict__ singular_min) {
    extern __shared__ double lds[];
    const int bb = bs * bs;
    double *a = lds;
    double *y = lds + bb;
    int *perm = reinterpret_cast<int *>(y + bb);
    __shared__ int dpos;
    const int lane = threadIdx.x;
    for (int I = blockIdx.x; I < nb; I += gridDim.x) {
        if (skip && skip[I]) continue;   // uniform over the workgroup
        if (lane == 0) dpos = -1;
        __syncthreads();
        for (int t = rowptr[I] + lane; t < rowptr[I + 1]; t += kWave)
            if (colidx[t] == I) dpos = t;
        __syncthreads();
        if (dpos < 0) {   // validated before; never taken for valid input
            if (lane == 0) atomicMin(singular_min, I);
            __syncthreads();
            continue;
        }
        const double *src = vals + static_cast<int64_t>(dpos) * bb;
        for (int e = lane; e < bb; e += kWave) a[e] = src[e];
        for (int i = lane; i < bs; i += kWave) perm[i] = i;
        __syncthreads();
        bool singular = false;
        for (int k = 0; k < bs; ++k) {
            double v = -1.0;
            int idx = bs;
            for (int i = k + lane; i < bs; i += kWave) {
                double av = fabs(a[i * bs + k]);
                if (av > v || (av == v && i < idx)) {
                    v = av;
                    idx = i;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                double ov = __shfl_xor(v, o, kWave);
                int oi = __shfl_xor(idx, o, kWave);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (!(v > 0.0)) {
                singular = true;
                break;
            }
            if (idx != k) {
                for (int j = lane; j < bs; j += kWave) {
                    double tmp = a[k * bs + j];
                    a[k * bs + j] = a[idx * bs + j];
                    a[idx * bs + j] = tmp;
                }
                if (lane == 0) {
                    int tp = perm[k];
                    perm[k] = perm[idx];
                    perm[idx] = tp;
                }
            }
            __syncthreads();
            const double piv = a[k * bs + k];
            for (int i = k + 1 + lane; i < bs; i += kWave) a[i * bs + k] = a[i * bs + k] / piv;
            __syncthreads();
            const int m = bs - k - 1;
            for (int e = lane; e < m * m; e += kWave) {
                const int i = k + 1 + e / m;
                const int j = k + 1 + e % m;
                a[i * bs + j] = __builtin_fma(-a[i * bs + k], a[k * bs + j], a[i * bs + j]);
            }
            __syncthreads();
        }
        if (singular) {
            if (lane == 0) atomicMin(singular_min, I);
            __syncthreads();
            continue;
        }
        for (int j = lane; j < bs; j += kWave) {
            for (int i = 0; i < bs; ++i) y[i * bs + j] = (perm[i] == j) ? 1.0 : 0.0;
            for (int i = 0; i < bs; ++i) {
                double s = y[i * bs + j];
                for (int mm = 0; mm < i; ++mm) s = __builtin_fma(-a[i * bs + mm], y[mm * bs + j], s);
                y[i * bs + j] = s;
            }
            for (int i = bs - 1; i >= 0; --i) {
                double s = y[i * bs + j];
                for (int mm = i + 1; mm < bs; ++mm) s = __builtin_fma(-a[i * bs + mm], y[mm * bs + j], s);
                y[i * bs + j] = s / a[i * bs + i];
            }
        }
        __syncthreads();
        double *dst = dinv + static_cast<int64_t>(I) * bb;
        for (int e = lane; e < bb; e += kWave) dst[e] = y[e];
        __syncthreads();
    }
}

// The same recipe with one thread per block row and the block in registers
// (small blocks, every index known at compile time; the pivot row exchange is
// a predicated swap with each candidate row).  Many small blocks then run at
// memory speed instead of one latency-bound wave each.
template <int BS>
__global__ __launch_bounds__(64) void k_block_inverse_thread(const int *__restrict__ rowptr,
                                                            const int *__restrict__ colidx,
                                                            const double *__restrict__ vals, int nb,
                                                            const int8_t *__restrict__ skip,
                                                            double *__restrict__ dinv, int *__restrict__ singular_min) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb || (skip && skip[I])) return;
    int dpos = -1;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t)
        if (colidx[t] == I) dpos = t;
    if (dpos < 0) {   // validated before; never taken for valid input
        atomicMin(singular_min, I);
        return;
    }
    double a[BS][BS];
    int perm[BS];
    const double *src = vals + static_cast<int64_t>(dpos) * BS * BS;
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        perm[i] = i;
#pragma unroll
        for (int j = 0; j < BS; ++j) a[i][j] = src[i * BS + j];
    }
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        // pivot: the first row i >= k of largest |a_ik|
        double v = -1.0;
        int idx = BS;
#pragma unroll
        for (int i = k; i < BS; ++i) {
            const double av = fabs(a[i][k]);
            if (av > v) {
                v = av;
                idx = i;
            }
        }
        if (!(v > 0.0)) {
            atomicMin(singular_min, I);
            return;
        }
#pragma unroll
        for (int r = k + 1; r < BS; ++r)
            if (idx == r) {
#pragma unroll
                for (int j = 0; j < BS; ++j) {
                    const double tmp = a[k][j];
                    a[k][j] = a[r][j];
                    a[r][j] = tmp;
                }
                const int tp = perm[k];
                perm[k] = perm[r];
                perm[r] = tp;
            }
        const double piv = a[k][k];
#pragma unroll
        for (int i = k + 1; i < BS; ++i) a[i][k] = a[i][k] / piv;
#pragma unroll
        for (int i = k + 1; i < BS; ++i)
#pragma unroll
            for (int j = k + 1; j < BS; ++j) a[i][j] = __builtin_fma(-a[i][k], a[k][j], a[i][j]);
    }
    double *dst = dinv + static_cast<int64_t>(I) * BS * BS;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        double y[BS];
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            double sacc = (perm[i] == j) ? 1.0 : 0.0;
#pragma unroll
            for (int mm = 0; mm < i; ++mm) sacc = __builtin_fma(-a[i][mm], y[mm], sacc);
            y[i] = sacc;
        }
#pragma unroll
        for (int i = BS - 1; i >= 0; --i) {
            double sacc = y[i];
#pragma unroll
            for (int mm = i + 1; mm < BS; ++mm) sacc = __builtin_fma(-a[i][mm], y[mm], sacc);
            y[i] = sacc / a[i][i];
        }
#pragma unroll
        for (int i = 0; i < BS; ++i) dst[i * BS + j] = y[i];
    }
}

// -------------------------------------------------------------- strength

// Row I: m = largest off-diagonal block size; block J != I is theta-strong
// when size >= theta*m (m > 0), phi-strong likewise; lambda_J counts the rows
// depending theta-strongly on J.
// The two sides of a comparison are within 1e-12 of each other, relative to
// the larger (both zero counts as a tie): the decision-margin audit.
__device__ inline bool near_tie(double a, double b) { return fabs(a - b) <= 1e-12 * fmax(fabs(a), fabs(b)); }

__global__ __launch_bounds__(256) void k_strength(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                 const double *__restrict__ bnorm, int nb, double theta, double phi,
                                                 uint8_t *__restrict__ mask, int *__restrict__ lambda,
                                                 int *__restrict__ margin) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    const int lo = rowptr[I], hi = rowptr[I + 1];
    double m = 0.0;
    for (int t = lo; t < hi; ++t)
        if (colidx[t] != I && bnorm[t] > m) m = bnorm[t];
    const double tt = theta * m, tp = phi * m;
    for (int t = lo; t < hi; ++t) {
        const int J = colidx[t];
        uint8_t mk = 0;
        if (J != I && m > 0.0) {
            if (bnorm[t] >= tt) mk |= 1;
            if (bnorm[t] >= tp) mk |= 2;
            if (near_tie(bnorm[t], tt)) atomicAdd(margin, 1);
            if (near_tie(bnorm[t], tp)) atomicAdd(margin + 1, 1);
        }
        mask[t] = mk;
        if (mk & 1) atomicAdd(&lambda[J], 1);
    }
}

// stidx[stptr[J] ...]: rows that depend theta-strongly on J (any order)
__global__ __launch_bounds__(256) void k_strong_transpose(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                         const uint8_t *__restrict__ mask, int nb,
                                                         const int *__restrict__ stptr, int *__restrict__ fill,
                                                         int *__restrict__ stidx) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t)
        if (mask[t] & 1) {
            const int J = colidx[t];
            const int pos = atomicAdd(&fill[J], 1);
            stidx[stptr[J] + pos] = I;
        }
}

// ------------------------------------------------------------ splitting

// kD: a block of a system that is solved directly on this level (batched
// hierarchies); it takes no part in the splitting.
constexpr int8_t kUnd = -1, kF = 0, kC = 1, kD = 2;

// splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014).
__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// key (lambda, hash, index) of I beats J's
__device__ inline bool key_beats(int lamI, uint64_t hI, int I, int lamJ, uint64_t hJ, int J) {
    if (lamI != lamJ) return lamI > lamJ;
    if (hI != hJ) return hI > hJ;
    return I > J;
}

__global__ __launch_bounds__(256) void k_pmis_init(const int *__restrict__ lambda, const int8_t *__restrict__ direct,
                                                  int nb, int8_t *__restrict__ state, int *__restrict__ dround,
                                                  int *__restrict__ undecided0) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    dround[I] = 0;
    if (direct && direct[I]) {
        state[I] = kD;
        return;
    }
    const bool und = lambda[I] != 0;
    state[I] = und ? kUnd : kF;
    if (und) atomicAdd(undecided0, 1);
}

// New C: undecided blocks whose key beats every undecided neighbour in S u S^T.
// The hash takes the block's index within its own system (I - lbase[I]; lbase
// == nullptr: one system), so a batched hierarchy splits every system exactly
// as it would alone; neighbours always share the system.
__global__ __launch_bounds__(256) void k_pmis_select(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                    const uint8_t *__restrict__ mask, const int *__restrict__ stptr,
                                                    const int *__restrict__ stidx, const int *__restrict__ lambda,
                                                    const int *__restrict__ lbase, int nb, uint64_t seed, int level,
                                                    const int8_t *__restrict__ state, int8_t *__restrict__ newc,
                                                    const int *__restrict__ prev) {
    if (*prev == 0) return;   // nothing was left undecided: the round has nothing to do
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    if (state[I] != kUnd) {
        newc[I] = 0;
        return;
    }
    const uint64_t salt = seed ^ (static_cast<uint64_t>(level) << 40);
    const int base = lbase ? lbase[I] : 0;
    const int lamI = lambda[I];
    const uint64_t hI = splitmix64(salt ^ static_cast<uint64_t>(I - base));
    bool is_max = true;
    for (int t = rowptr[I]; t < rowptr[I + 1] && is_max; ++t) {
        if (!(mask[t] & 1)) continue;
        const int J = colidx[t];
        if (state[J] == kUnd &&
            !key_beats(lamI, hI, I, lambda[J], splitmix64(salt ^ static_cast<uint64_t>(J - base)), J))
            is_max = false;
    }
    for (int t = stptr[I]; t < stptr[I + 1] && is_max; ++t) {
        const int J = stidx[t];
        if (state[J] == kUnd &&
            !key_beats(lamI, hI, I, lambda[J], splitmix64(salt ^ static_cast<uint64_t>(J - base)), J))
            is_max = false;
    }
    newc[I] = is_max ? 1 : 0;
}

// New C blocks become C; undecided blocks depending strongly on a new C become F.
__global__ __launch_bounds__(256) void k_pmis_update(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                    const uint8_t *__restrict__ mask, int nb, int round,
                                                    int8_t *__restrict__ state, const int8_t *__restrict__ newc,
                                                    int *__restrict__ dround, int *__restrict__ undecided) {
    if (undecided[-1] == 0) return;   // as k_pmis_select: the splitting has finished
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    if (state[I] != kUnd) return;
    if (newc[I]) {
        state[I] = kC;
        dround[I] = round;
        return;
    }
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t)
        if ((mask[t] & 1) && newc[colidx[t]]) {
            state[I] = kF;
            dround[I] = round;
            return;
        }
    atomicAdd(undecided, 1);
}

__global__ __launch_bounds__(256) void k_cf_flags(const int8_t *__restrict__ state, int nb, int8_t want,
                                                 int *__restrict__ flags) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nb) flags[I] = (state[I] == want) ? 1 : 0;
}

// cscan[I] = number of C blocks before I; fscan[I] = number of F blocks before
// I (fscan == nullptr: every non-C block is F).
__global__ __launch_bounds__(256) void k_cf_index(const int8_t *__restrict__ cf, const int *__restrict__ cscan,
                                                 const int *__restrict__ fscan, int nb, int *__restrict__ cidx,
                                                 int *__restrict__ cpts, int *__restrict__ flist) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    const int c = cscan[I];
    if (cf[I] == kC) {
        cidx[I] = c;
        cpts[c] = I;
    } else {
        cidx[I] = -1;
        if (cf[I] == kF) flist[fscan ? fscan[I] : I - c] = I;
    }
}

// Per block: first block of its system (lbase) and whether the system is
// solved directly on this level (direct); seg holds nsys + 1 block offsets.
__global__ __launch_bounds__(256) void k_seg_info(const int *__restrict__ seg, const int8_t *__restrict__ mode,
                                                 int nsys, int nb, int *__restrict__ lbase,
                                                 int8_t *__restrict__ direct, int *__restrict__ bsys) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    int lo = 0, hi = nsys;   // the largest s < nsys with seg[s] <= I (skips empty systems)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= I) lo = mid;
        else hi = mid;
    }
    if (lbase) lbase[I] = seg[lo];
    if (direct) direct[I] = mode[lo] == 2 ? 1 : 0;
    if (bsys) bsys[I] = lo;
}

// Blocks of systems switched to a direct solve after their splitting stalled.
__global__ __launch_bounds__(256) void k_mark_direct(const int8_t *__restrict__ direct, int nb,
                                                    int8_t *__restrict__ state) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < nb && direct[I]) state[I] = kD;
}

struct FillJobs {
    int *p[4];
    int64_t n[4];
    int v[4];
    int k;
};

__global__ __launch_bounds__(256) void k_fill_ints(FillJobs J) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int j = 0; j < J.k; ++j)
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < J.n[j]; i += stride)
            J.p[j][i] = J.v[j];
}

// out[i] = v[idx[i]] for i < n
__global__ __launch_bounds__(256) void k_gather_int(const int *__restrict__ v, const int *__restrict__ idx, int n,
                                                   int *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v[idx[i]];
}

// ------------------------------------------------------ one-point interpolation

// F block: coarse index of its largest (nonzero) stored C block, lowest column on ties.
__global__ __launch_bounds__(256) void k_one_point(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                  const double *__restrict__ bnorm, const int8_t *__restrict__ cf,
                                                  const int *__restrict__ cidx, int nb, int *__restrict__ pmap,
                                                  int *__restrict__ margin) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    if (cf[I] == kC) {
        pmap[I] = cidx[I];
        return;
    }
    int best = -1;
    double bestn = 0.0;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t];
        if (J != I && cf[J] == kC && bnorm[t] > bestn) {
            bestn = bnorm[t];
            best = J;
        }
    }
    pmap[I] = (best >= 0) ? cidx[best] : -1;
    if (best >= 0)   // audit: another candidate within 1e-12 of the chosen one's size
        for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            const int J = colidx[t];
            if (J != I && J != best && cf[J] == kC && bnorm[t] > 0.0 && near_tie(bnorm[t], bestn)) {
                atomicAdd(margin + 2, 1);
                break;
            }
        }
}

// ----------------------------------------------- Neumann operands (patterns)

__global__ __launch_bounds__(256) void k_count_T(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                const uint8_t *__restrict__ mask, const int8_t *__restrict__ cf,
                                                int nb, int *__restrict__ cnt) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    int c = 0;
    if (cf[I] == kF)
        for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            const int J = colidx[t];
            c += (J != I && cf[J] == kF && (mask[t] & 2)) ? 1 : 0;
        }
    cnt[I] = c;
}

__global__ __launch_bounds__(256) void k_fill_T(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                               const uint8_t *__restrict__ mask, const int8_t *__restrict__ cf, int nb,
                                               const int *__restrict__ trowptr, int *__restrict__ tcol,
                                               int *__restrict__ trow, int *__restrict__ tsrc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb || cf[I] != kF) return;
    int o = trowptr[I];
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) {
        const int J = colidx[t];
        if (J != I && cf[J] == kF && (mask[t] & 2)) {
            tcol[o] = J;
            trow[o] = I;
            tsrc[o] = t;
            ++o;
        }
    }
}

__global__ __launch_bounds__(256) void k_count_Acf(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                  const int8_t *__restrict__ cf, const int *__restrict__ cpts, int nc,
                                                  int *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int I = cpts[i];
    int c = 0;
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t) c += (cf[colidx[t]] == kF) ? 1 : 0;
    cnt[i] = c;
}

__global__ __launch_bounds__(256) void k_fill_Acf(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                 const int8_t *__restrict__ cf, const int *__restrict__ cpts, int nc,
                                                 const int *__restrict__ wrowptr, int *__restrict__ wcol,
                                                 int *__restrict__ wsrc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int I = cpts[i];
    int o = wrowptr[i];
    for (int t = rowptr[I]; t < rowptr[I + 1]; ++t)
        if (cf[colidx[t]] == kF) {
            wcol[o] = colidx[t];
            wsrc[o] = t;
            ++o;
        }
}

// out[t] = sign * (X[xi[t]] Y[yi[t]]): entry (a,b) = fma chain over c ascending
// from +0.  One thread per (block, row a) with the row's accumulators in
// registers; xi == nullptr means xi[t] = t.
template <int BS>
__global__ __launch_bounds__(256) void k_block_product(int64_t n, int bs_rt, const double *__restrict__ X,
                                                      const int *__restrict__ xi, const double *__restrict__ Y,
                                                      const int *__restrict__ yi, double sign,
                                                      double *__restrict__ out, const int *__restrict__ count) {
    constexpr int NB = BS > 0 ? BS : kMaxBs;
    const int bs = BS > 0 ? BS : bs_rt;
    const int bb = bs * bs;
    const int64_t total = (count ? *count : n) * bs;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bs;
        const int a = static_cast<int>(g - t * bs);
        const double *x = X + static_cast<int64_t>(xi ? xi[t] : t) * bb + a * bs;
        const double *y = Y + static_cast<int64_t>(yi[t]) * bb;
        double acc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (BS == 0 && c >= bs) break;
            const double xc = x[c];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (BS > 0 || b < bs) acc[b] = __builtin_fma(xc, y[c * bs + b], acc[b]);
        }
        double *o = out + t * bb + a * bs;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (BS > 0 || b < bs) o[b] = sign * acc[b];
    }
}

// The same on the FP64 matrix cores (bs 9, 16, 25; mfma_tile.h): one wave per
// block, the product in 16x16 accumulator tiles built by ceil(bs/4) 16x16x4
// steps per tile, each the ascending fma chain over its four inner indices,
// from +0; then the sign.  Bit-identical to the chain above (up to the sign of
// a zero, see mfma_tile.h).  Also the mask of the block's nonzero rows.
template <int BS>
__global__ __launch_bounds__(256) void k_block_product_mfma(int64_t n, const double *__restrict__ X,
                                                           const int *__restrict__ xi, const double *__restrict__ Y,
                                                           const int *__restrict__ yi, double sign,
                                                           double *__restrict__ out, const int *__restrict__ count,
                                                           uint32_t *__restrict__ rmask) {
    // both blocks read with consecutive lanes on consecutive words into the
    // wave's LDS slot, the matrix-core fragments taken from there
    constexpr int bb = BS * BS;
    constexpr int NL = (bb + 63) / 64;   // loads per lane and block
    constexpr int NT = MfmaShape<BS>::NT, KQ = MfmaShape<BS>::KQ;
    __shared__ double slot[4][2 * bb];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + w;
    if (t >= (count ? *count : n)) return;   // whole waves; no workgroup barrier below
    double *xs = slot[w], *ys = slot[w] + bb;
    const double *x = X + static_cast<int64_t>(xi ? xi[t] : t) * bb;
    const double *y = Y + static_cast<int64_t>(yi[t]) * bb;
    double xv[NL], yv[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int e = lane + 64 * i;
        xv[i] = e < bb ? x[e] : 0.0;
        yv[i] = e < bb ? y[e] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int e = lane + 64 * i;
        if (e < bb) {
            xs[e] = xv[i];
            ys[e] = yv[i];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    MfmaAcc<BS> acc;
    acc.zero();
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
    }
    double *o = out + t * bb;
    uint32_t bits = 0u;   // this lane's nonzero rows, then the block's
    mfma_for_entries<BS>(acc, row, kk, [&](int i, int j, double v) {
        const double wv = sign * v;
        o[i * BS + j] = wv;
        if (wv != 0.0) bits |= 1u << i;
    });
    if (rmask) {
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) bits |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(bits), o2, 64));
        if (lane == 0) rmask[t] = bits;
    }
}

// The same product with X the blocks of a sum that is never stored: block t
// of X is the sum, in term order, of the present terms' blocks, added entry by
// entry as repeated bsr_add adds them, so the results equal storing the sum
// first.  (Presence is per block: the branches are uniform over the wave.)
template <int BS>
__global__ __launch_bounds__(256) void k_sum_product_mfma(int64_t n, const SumTerms terms,
                                                         const double *__restrict__ Y, const int *__restrict__ yi,
                                                         double sign, double *__restrict__ out,
                                                         const int *__restrict__ count, uint32_t *__restrict__ rmask) {
    constexpr int bb = BS * BS;
    constexpr int NL = (bb + 63) / 64;   // loads per lane and block
    constexpr int NT = MfmaShape<BS>::NT, KQ = MfmaShape<BS>::KQ;
    __shared__ double slot[4][2 * bb];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kk = lane >> 4;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + w;
    if (t >= (count ? *count : n)) return;   // whole waves; no workgroup barrier below
    double *xs = slot[w], *ys = slot[w] + bb;
    // every term's block index at once (lane k: term k), and D^-1's block
    const int msrc = lane < terms.n ? terms.map[lane][t] : -1;
    const double *y = Y + static_cast<int64_t>(yi[t]) * bb;
    double yv[NL], sv[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int e = lane + 64 * i;
        yv[i] = e < bb ? y[e] : 0.0;
        sv[i] = 0.0;
    }
    // the sum's block, entry by entry in term order (consecutive lanes on consecutive words)
    bool first = true;
    for (int k = 0; k < terms.n; ++k) {
        const int src = __shfl(msrc, k, 64);
        if (src < 0) continue;
        const double *x = terms.vals[k] + static_cast<int64_t>(src) * bb;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = lane + 64 * i;
            if (e < bb) {
                const double v = x[e];
                sv[i] = first ? v : sv[i] + v;
            }
        }
        first = false;
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int e = lane + 64 * i;
        if (e < bb) {
            xs[e] = sv[i];
            ys[e] = yv[i];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    MfmaAcc<BS> acc;
    acc.zero();
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
    }
    double *o = out + t * bb;
    uint32_t bits = 0u;
    mfma_for_entries<BS>(acc, row, kk, [&](int i, int j, double v) {
        const double wv = sign * v;
        o[i * BS + j] = wv;
        if (wv != 0.0) bits |= 1u << i;
    });
    if (rmask) {
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) bits |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(bits), o2, 64));
        if (lane == 0) rmask[t] = bits;
    }
}

__global__ __launch_bounds__(256) void k_map_through(int64_t n, const int *__restrict__ count, int *__restrict__ map,
                                                    const int *__restrict__ through) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n || (count && t >= *count)) return;
    const int v = map[t];
    map[t] = v >= 0 ? through[v] : -1;
}

// maps[i][t] = srcS[t] >= 0 ? old[i][srcS[t]] : -1 for every term i
struct MapsIO {
    const int *old[kMaxSumTerms] = {};
    int *out[kMaxSumTerms] = {};
    int n = 0;
};
__global__ __launch_bounds__(256) void k_compose_maps(int64_t cap, const int *__restrict__ count,
                                                     const int *__restrict__ srcS, const MapsIO io) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= cap || t >= *count) return;
    const int a = srcS[t];
    for (int i = 0; i < io.n; ++i) io.out[i][t] = a >= 0 ? io.old[i][a] : -1;
}

__global__ __launch_bounds__(256) void k_block_gather(int64_t n, int bb, const double *__restrict__ Y,
                                                     const int *__restrict__ src, double *__restrict__ out,
                                                     const int *__restrict__ count) {
    const int64_t total = (count ? *count : n) * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bb;
        const int e = static_cast<int>(g - t * bb);
        out[g] = Y[static_cast<int64_t>(src[t]) * bb + e];
    }
}

// The same with one wave per block (blocks of 64 entries or more): the block
// index and its source are read once per block and the entries need no division.
// Each wave takes two blocks per round and issues every load of both before the
// stores (NCH: the 64-word chunks that cover a block, at most 16 for bs <= 32;
// words past a block repeat its last, unused).
template <int NCH>
__global__ __launch_bounds__(256) void k_block_gather_wave(int64_t n, int bb, const double *__restrict__ Y,
                                                          const int *__restrict__ src, double *__restrict__ out,
                                                          const int *__restrict__ count) {
    const int lane = threadIdx.x & 63;
    const int64_t nblk = count ? *count : n;
    const int64_t stride = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t t = ((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6) * 2; t < nblk;
         t += 2 * stride) {
        const bool two = t + 1 < nblk;
        const double *y0 = Y + static_cast<int64_t>(src[t]) * bb;
        const double *y1 = two ? Y + static_cast<int64_t>(src[t + 1]) * bb : y0;
        double v0[NCH], v1[NCH];
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int e = lane + 64 * i < bb ? lane + 64 * i : bb - 1;
            v0[i] = y0[e];
            v1[i] = y1[e];
        }
        double *o = out + t * bb;
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int e = lane + 64 * i;
            if (e < bb) {
                o[e] = v0[i];
                if (two) o[bb + e] = v1[i];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_rows_of(const int *__restrict__ rowptr, int nrows, int *__restrict__ rowid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int t = rowptr[i]; t < rowptr[i + 1]; ++t) rowid[t] = i;
}

unsigned cap_grid(int64_t g) { return static_cast<unsigned>(g > 65536 * 16 ? 65536 * 16 : (g < 1 ? 1 : g)); }

}  // namespace

void launch_block_scan(const double *vals, int64_t n, int bs, const int *src, const int *count, double *maxabs,
                       uint64_t *meta, uint32_t *rmask, int *rsize, hipStream_t s, double *copy) {
    if (n <= 0) return;
    if (bs < 1 || bs > 32) fail(NAIR_EINVAL, "block scan: bs must be in 1..32");
    if (copy && (src || count)) fail(NAIR_EDEVICE, "block scan: a copy only of blocks in place");
    int L = 1;
    while (L < bs * bs && L < kWave) L <<= 1;
    const int per = 256 / L;
    k_block_scan<<<grid_for(n, per), 256, 0, s>>>(vals, n, bs, L, src, count, maxabs,
                                                  reinterpret_cast<unsigned long long *>(meta), rmask, rsize, copy);
    NAIR_HIP(hipGetLastError());
}

void launch_block_maxabs(const double *vals, int64_t nnzb, int bs, double *out, hipStream_t s) {
    launch_block_scan(vals, nnzb, bs, nullptr, nullptr, out, nullptr, nullptr, nullptr, s);
}

void launch_block_inverse(const int *rowptr, const int *colidx, const double *vals, int nb, int bs,
                          const int8_t *skip, double *dinv, int *singular_min, hipStream_t s) {
    if (nb <= 0) return;
    const unsigned grid = static_cast<unsigned>((nb + 63) / 64);
    if (bs == 9) {
        k_block_inverse_thread<9><<<grid, 64, 0, s>>>(rowptr, colidx, vals, nb, skip, dinv, singular_min);
    } else if (bs == 4) {
        k_block_inverse_thread<4><<<grid, 64, 0, s>>>(rowptr, colidx, vals, nb, skip, dinv, singular_min);
    } else if (bs == 16 || bs == 25) {
        const unsigned hgrid = static_cast<unsigned>((nb + 7) / 8);   // eight half waves (blocks) per workgroup
        if (bs == 16)
            k_block_inverse_rows<16><<<hgrid, 256, 0, s>>>(rowptr, colidx, vals, nb, skip, dinv, singular_min);
        else
            k_block_inverse_rows<25><<<hgrid, 256, 0, s>>>(rowptr, colidx, vals, nb, skip, dinv, singular_min);
    } else {
        const size_t lds = sizeof(double) * 2 * bs * bs + sizeof(int) * bs;
        k_block_inverse<<<cap_grid(nb), 64, lds, s>>>(rowptr, colidx, vals, nb, bs, skip, dinv, singular_min);
    }
    NAIR_HIP(hipGetLastError());
}

void launch_strength(const int *rowptr, const int *colidx, const double *bnorm, int nb, double theta, double phi,
                     uint8_t *mask, int *lambda, int *margin, hipStream_t s) {
    k_strength<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, bnorm, nb, theta, phi, mask, lambda, margin);
    NAIR_HIP(hipGetLastError());
}

void launch_strong_transpose(const int *rowptr, const int *colidx, const uint8_t *mask, int nb, const int *stptr,
                             int *fill, int *stidx, hipStream_t s) {
    k_strong_transpose<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, mask, nb, stptr, fill, stidx);
    NAIR_HIP(hipGetLastError());
}

void launch_pmis_init(const int *lambda, const int8_t *direct, int nb, int8_t *state, int *dround, int *undecided0,
                      hipStream_t s) {
    k_pmis_init<<<grid_for(nb, 256), 256, 0, s>>>(lambda, direct, nb, state, dround, undecided0);
    NAIR_HIP(hipGetLastError());
}

void launch_pmis_round(const int *rowptr, const int *colidx, const uint8_t *mask, const int *stptr, const int *stidx,
                       const int *lambda, const int *lbase, int nb, uint64_t seed, int level, int round,
                       int8_t *state, int8_t *newc, int *dround, int *undecided, hipStream_t s) {
    k_pmis_select<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, mask, stptr, stidx, lambda, lbase, nb, seed,
                                                    level, state, newc, undecided - 1);
    k_pmis_update<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, mask, nb, round, state, newc, dround,
                                                    undecided);
    NAIR_HIP(hipGetLastError());
}

void launch_cf_flags(const int8_t *state, int nb, int want, int *flags, hipStream_t s) {
    k_cf_flags<<<grid_for(nb, 256), 256, 0, s>>>(state, nb, static_cast<int8_t>(want), flags);
    NAIR_HIP(hipGetLastError());
}

void launch_cf_index(const int8_t *cf, const int *cscan, const int *fscan, int nb, int *cidx, int *cpts, int *flist,
                     hipStream_t s) {
    k_cf_index<<<grid_for(nb, 256), 256, 0, s>>>(cf, cscan, fscan, nb, cidx, cpts, flist);
    NAIR_HIP(hipGetLastError());
}

void launch_seg_info(const int *seg, const int8_t *mode, int nsys, int nb, int *lbase, int8_t *direct, int *bsys,
                     hipStream_t s) {
    if (nb <= 0) return;
    k_seg_info<<<grid_for(nb, 256), 256, 0, s>>>(seg, mode, nsys, nb, lbase, direct, bsys);
    NAIR_HIP(hipGetLastError());
}

void launch_mark_direct(const int8_t *direct, int nb, int8_t *state, hipStream_t s) {
    if (nb <= 0) return;
    k_mark_direct<<<grid_for(nb, 256), 256, 0, s>>>(direct, nb, state);
    NAIR_HIP(hipGetLastError());
}

void launch_fill_ints(std::initializer_list<FillInts> jobs, hipStream_t s) {
    FillJobs J{};
    int64_t most = 0;
    for (const FillInts &f : jobs) {
        if (J.k == 4) fail(NAIR_EDEVICE, "launch_fill_ints: more than four arrays");
        if (f.n <= 0) continue;
        J.p[J.k] = f.p;
        J.n[J.k] = f.n;
        J.v[J.k] = f.v;
        most = std::max(most, f.n);
        ++J.k;
    }
    if (J.k == 0) return;
    k_fill_ints<<<cap_grid((most + 255) / 256), 256, 0, s>>>(J);
    NAIR_HIP(hipGetLastError());
}

void launch_gather_int(const int *v, const int *idx, int n, int *out, hipStream_t s) {
    if (n <= 0) return;
    k_gather_int<<<grid_for(n, 256), 256, 0, s>>>(v, idx, n, out);
    NAIR_HIP(hipGetLastError());
}

void launch_one_point(const int *rowptr, const int *colidx, const double *bnorm, const int8_t *cf, const int *cidx,
                      int nb, int *pmap, int *margin, hipStream_t s) {
    k_one_point<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, bnorm, cf, cidx, nb, pmap, margin);
    NAIR_HIP(hipGetLastError());
}

void launch_count_T(const int *rowptr, const int *colidx, const uint8_t *mask, const int8_t *cf, int nb, int *cnt,
                    hipStream_t s) {
    k_count_T<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, mask, cf, nb, cnt);
    NAIR_HIP(hipGetLastError());
}

void launch_fill_T(const int *rowptr, const int *colidx, const uint8_t *mask, const int8_t *cf, int nb,
                   const int *trowptr, int *tcol, int *trow, int *tsrc, hipStream_t s) {
    k_fill_T<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, mask, cf, nb, trowptr, tcol, trow, tsrc);
    NAIR_HIP(hipGetLastError());
}

void launch_count_Acf(const int *rowptr, const int *colidx, const int8_t *cf, const int *cpts, int nc, int *cnt,
                      hipStream_t s) {
    if (nc <= 0) return;
    k_count_Acf<<<grid_for(nc, 256), 256, 0, s>>>(rowptr, colidx, cf, cpts, nc, cnt);
    NAIR_HIP(hipGetLastError());
}

void launch_fill_Acf(const int *rowptr, const int *colidx, const int8_t *cf, const int *cpts, int nc,
                     const int *wrowptr, int *wcol, int *wsrc, hipStream_t s) {
    if (nc <= 0) return;
    k_fill_Acf<<<grid_for(nc, 256), 256, 0, s>>>(rowptr, colidx, cf, cpts, nc, wrowptr, wcol, wsrc);
    NAIR_HIP(hipGetLastError());
}

void launch_block_product(int64_t n, int bs, const double *X, const int *xi, const double *Y, const int *yi,
                          double sign, double *out, hipStream_t s, const int *count, uint32_t *rmask) {
    if (n <= 0) return;
    if (use_matrix_cores(bs)) {
        const unsigned mgrid = static_cast<unsigned>((n + 3) / 4);   // four waves (blocks) per workgroup
        if (bs == 9) k_block_product_mfma<9><<<mgrid, 256, 0, s>>>(n, X, xi, Y, yi, sign, out, count, rmask);
        else if (bs == 16) k_block_product_mfma<16><<<mgrid, 256, 0, s>>>(n, X, xi, Y, yi, sign, out, count, rmask);
        else k_block_product_mfma<25><<<mgrid, 256, 0, s>>>(n, X, xi, Y, yi, sign, out, count, rmask);
        NAIR_HIP(hipGetLastError());
        return;
    }
    if (rmask) fail(NAIR_EDEVICE, "launch_block_product: row masks only from the matrix-core products");
    const unsigned grid = cap_grid((n * bs + 255) / 256);
    switch (bs) {
        case 4: k_block_product<4><<<grid, 256, 0, s>>>(n, bs, X, xi, Y, yi, sign, out, count); break;
        case 9: k_block_product<9><<<grid, 256, 0, s>>>(n, bs, X, xi, Y, yi, sign, out, count); break;
        case 16: k_block_product<16><<<grid, 256, 0, s>>>(n, bs, X, xi, Y, yi, sign, out, count); break;
        case 25: k_block_product<25><<<grid, 256, 0, s>>>(n, bs, X, xi, Y, yi, sign, out, count); break;
        default: k_block_product<0><<<grid, 256, 0, s>>>(n, bs, X, xi, Y, yi, sign, out, count); break;
    }
    NAIR_HIP(hipGetLastError());
}

void launch_sum_product(int64_t n, int bs, const SumTerms &terms, const double *Y, const int *yi, double sign,
                        double *out, hipStream_t s, const int *count, uint32_t *rmask) {
    if (n <= 0) return;
    if (!use_matrix_cores(bs)) fail(NAIR_EDEVICE, "launch_sum_product: matrix-core block sizes only");
    if (terms.n < 1 || terms.n > kMaxSumTerms) fail(NAIR_EDEVICE, "launch_sum_product: 1 to 17 terms");
    for (int i = 0; i < terms.n; ++i)
        if (!terms.map[i]) fail(NAIR_EDEVICE, "launch_sum_product: a term without its map");
    const unsigned mgrid = static_cast<unsigned>((n + 3) / 4);   // four waves (blocks) per workgroup
    if (bs == 9)
        k_sum_product_mfma<9><<<mgrid, 256, 0, s>>>(n, terms, Y, yi, sign, out, count, rmask);
    else if (bs == 16)
        k_sum_product_mfma<16><<<mgrid, 256, 0, s>>>(n, terms, Y, yi, sign, out, count, rmask);
    else
        k_sum_product_mfma<25><<<mgrid, 256, 0, s>>>(n, terms, Y, yi, sign, out, count, rmask);
    NAIR_HIP(hipGetLastError());
}

void launch_map_through(int64_t n, const int *count, int *map, const int *through, hipStream_t s) {
    if (n <= 0) return;
    k_map_through<<<grid_for(n, 256), 256, 0, s>>>(n, count, map, through);
    NAIR_HIP(hipGetLastError());
}

void compose_term_maps(int64_t cap, const int *count, const int *srcS, std::vector<DBuf<int>> &maps,
                       hipStream_t s) {
    if (static_cast<int>(maps.size()) + 1 > kMaxSumTerms) fail(NAIR_EDEVICE, "compose_term_maps: too many terms");
    std::vector<DBuf<int>> out(maps.size());
    MapsIO io;
    io.n = static_cast<int>(maps.size());
    for (int i = 0; i < io.n; ++i) {
        out[i].alloc(static_cast<size_t>(std::max<int64_t>(cap, 1)));
        io.old[i] = maps[i].get();
        io.out[i] = out[i].get();
    }
    if (cap > 0) {
        k_compose_maps<<<grid_for(cap, 256), 256, 0, s>>>(cap, count, srcS, io);
        NAIR_HIP(hipGetLastError());
    }
    maps = std::move(out);
}

void launch_block_gather(int64_t n, int bs, const double *Y, const int *src, double *out, hipStream_t s,
                         const int *count) {
    if (n <= 0) return;
    if (bs * bs >= 64) {
        // the instance for blocks of at most 128, 256 or 640 entries, else 16 chunks
        const int bb = bs * bs;
        void (*kern)(int64_t, int, const double *, const int *, double *, const int *) = k_block_gather_wave<16>;
        switch ((bb + 63) / 64) {
            case 2: kern = k_block_gather_wave<2>; break;
            case 4: kern = k_block_gather_wave<4>; break;
            case 10: kern = k_block_gather_wave<10>; break;
            default: break;
        }
        kern<<<cap_grid((n + 7) / 8), 256, 0, s>>>(n, bb, Y, src, out, count);
    } else {
        k_block_gather<<<cap_grid((n * bs * bs + 255) / 256), 256, 0, s>>>(n, bs * bs, Y, src, out, count);
    }
    NAIR_HIP(hipGetLastError());
}

void launch_rows_of(const int *rowptr, int nrows, int *rowid, hipStream_t s) {
    if (nrows <= 0) return;
    k_rows_of<<<grid_for(nrows, 256), 256, 0, s>>>(rowptr, nrows, rowid);
    NAIR_HIP(hipGetLastError());
}

}  // namespace nair

namespace nair {
namespace {

// bad |= 1: rowptr not monotone/out of range; 2: column out of range;
// 4: columns not strictly increasing; 8: missing diagonal block; 16: a block
// couples two systems (seg: nsys + 1 block offsets, or nullptr for one system).
__global__ __launch_bounds__(256) void k_validate(const int *__restrict__ rowptr, const int *__restrict__ colidx, int nb,
                                                 int64_t nnzb, const int *__restrict__ seg, int nsys,
                                                 int *__restrict__ bad) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nb) return;
    const int lo = rowptr[I], hi = rowptr[I + 1];
    if ((I == 0 && lo != 0) || lo < 0 || hi < lo || hi > nnzb) {
        atomicOr(bad, 1);
        return;
    }
    int s_lo = 0, s_hi = nb;   // block range of I's system
    if (seg) {
        int a = 0, b = nsys;
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (seg[mid] <= I) a = mid;
            else b = mid;
        }
        s_lo = seg[a];
        s_hi = seg[a + 1];
    }
    bool diag = false;
    for (int t = lo; t < hi; ++t) {
        const int J = colidx[t];
        if (J < 0 || J >= nb) {
            atomicOr(bad, 2);
            return;
        }
        if (J < s_lo || J >= s_hi) atomicOr(bad, 16);
        if (t > lo && J <= colidx[t - 1]) atomicOr(bad, 4);
        if (J == I) diag = true;
    }
    if (!diag) atomicOr(bad, 8);
}

}  // namespace

void launch_validate(const int *rowptr, const int *colidx, int nb, int64_t nnzb, const int *seg, int nsys, int *bad,
                     hipStream_t s) {
    k_validate<<<grid_for(nb, 256), 256, 0, s>>>(rowptr, colidx, nb, nnzb, seg, nsys, bad);
    NAIR_HIP(hipGetLastError());
}

}  // namespace nair
