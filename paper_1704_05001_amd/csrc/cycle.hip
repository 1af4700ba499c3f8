// Cycle kernels: block residual r = b - A x with fused squared norm, fused
// block-Jacobi sweep (residual of the block row, then D^-1 or D^-T from LDS),
// restriction r_c = r_C + Z r_F, one-point interpolation, and the transposed
// counterparts (P^T gather, R^T = [Z^T; I] update).
//
// Mapping: a workgroup of 256 threads holds floor(256 / (G*bs)) block rows;
// each block row gets G groups of bs lanes, lane (g, a) accumulating scalar row
// a over the row's blocks g, g+G, ...; the G partial sums meet in LDS.  G is
// picked per level from the average row length, so short rows (the fine level)
// waste no lanes and long rows (coarse levels) are not serial.  The block size
// is a template parameter for the common sizes, so a block row's loads issue
// together; other sizes use the runtime-bs instance (bs <= 32).
//
// Precision: matrices (MT) and cycle vectors (VT) are double, or float for the
// FP32-stored hierarchy; accumulation and the block-diagonal inverses are
// always double.
#include <string>

#include "common.h"

namespace nair {
namespace {

constexpr int kThreads = 256;

template <int BS>
struct Bs {
    __device__ static constexpr int get(int) { return BS; }
};
template <>
struct Bs<0> {
    __device__ static int get(int bs) { return bs; }
};

// Where a row product reads the block vector of column J.
template <typename VT>
struct PlainSrc {
    const VT *x;
    int bs;
    static constexpr bool kMaySkip = false;
    __device__ const VT *row(int j) const { return x + static_cast<int64_t>(j) * bs; }
};
// x = P e_c read through the one-point map: block J is e_c's block pmap[J], or
// zero (skipped: its products would add zeros) when pmap[J] < 0.
template <typename VT>
struct PmapSrc {
    const VT *ec;
    const int *pmap;
    int bs;
    static constexpr bool kMaySkip = true;
    __device__ const VT *row(int j) const {
        const int p = pmap[j];
        return p >= 0 ? ec + static_cast<int64_t>(p) * bs : nullptr;
    }
};
// One block row's product with x_J: sum over c of blk[c] x_J[c], the even and
// the odd c summed apart and then added.  Every row product below adds these
// per-block sums in block order, whichever lanes form them, so the kernels that
// read a level's blocks whole, face-compressed, by their nonzero rows or one
// lane per stored row agree bit for bit (at one lane group per row).
template <int BS, typename MT, typename VT>
__device__ inline double block_row_dot(const MT *__restrict__ blk, const VT *__restrict__ xj, int bs) {
    double p0 = 0.0, p1 = 0.0;
    if constexpr (BS > 0) {
#pragma unroll
        for (int c = 0; c < BS; c += 2) {
            p0 += static_cast<double>(blk[c]) * static_cast<double>(xj[c]);
            if (c + 1 < BS) p1 += static_cast<double>(blk[c + 1]) * static_cast<double>(xj[c + 1]);
        }
    } else {
        for (int c = 0; c < bs; c += 2) {
            p0 += static_cast<double>(blk[c]) * static_cast<double>(xj[c]);
            if (c + 1 < bs) p1 += static_cast<double>(blk[c + 1]) * static_cast<double>(xj[c + 1]);
        }
    }
    return p0 + p1;
}

// sum over blocks t = lo+g, lo+g+G, ... < hi of (block t row a) . x[col t];
// with SKIP, the block in column `skip` (the row's diagonal block) is left out.
template <int BS, typename MT, typename VT, typename SRC, bool SKIP = false>
__device__ inline double row_part_src(const int *__restrict__ colidx, const MT *__restrict__ vals, int lo, int hi,
                                      int g, int G, int a, int bs_rt, const SRC &src, int skip = -1) {
    const int bs = Bs<BS>::get(bs_rt);
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    double acc = 0.0;
    for (int t = lo + g; t < hi; t += G) {
        const MT *blk = vals + t * bb + a * bs;
        const int J = colidx[t];
        if constexpr (SKIP) {
            if (J == skip) continue;
        }
        const VT *xj = src.row(J);
        if constexpr (SRC::kMaySkip) {
            if (xj == nullptr) continue;
        }
        acc += block_row_dot<BS>(blk, xj, bs);
    }
    return acc;
}

template <int BS, typename MT, typename VT, bool SKIP = false>
__device__ inline double row_part(const int *__restrict__ colidx, const MT *__restrict__ vals, int lo, int hi, int g,
                                  int G, int a, int bs_rt, const VT *__restrict__ x, int skip = -1) {
    return row_part_src<BS, MT, VT, PlainSrc<VT>, SKIP>(colidx, vals, lo, hi, g, G, a, bs_rt,
                                                        PlainSrc<VT>{x, Bs<BS>::get(bs_rt)}, skip);
}

// The same row product over a face-compressed copy: the diagonal block whole
// (from dvals; left out with SKIP), an off-diagonal block only when row a is
// one of its nonzero rows, and then only over its nonzero columns.  The
// entries left out are exact zeros and every product kept goes to the
// accumulator row_part gives it (column parity), in the same order, so for
// finite x the result equals row_part's bit for bit.
// The diagonal block's part of row_part_face (column-major dvals), for a
// caller that loads it before the row's other blocks.
template <int BS, typename MT, typename VT>
__device__ inline double face_diag_dot(const FaceView<MT> &F, int I, int a, int bs_rt, const VT *__restrict__ x) {
    const int bs = Bs<BS>::get(bs_rt);
    const MT *blk = F.dvals + static_cast<int64_t>(I) * bs * bs + a;
    const VT *xj = x + static_cast<int64_t>(I) * bs;
    double p0 = 0.0, p1 = 0.0;
    if constexpr (BS > 0) {
#pragma unroll
        for (int c = 0; c < BS; c += 2) {
            p0 += static_cast<double>(blk[c * BS]) * static_cast<double>(xj[c]);
            if (c + 1 < BS) p1 += static_cast<double>(blk[(c + 1) * BS]) * static_cast<double>(xj[c + 1]);
        }
    } else {
        for (int c = 0; c < bs; c += 2) {
            p0 += static_cast<double>(blk[c * bs]) * static_cast<double>(xj[c]);
            if (c + 1 < bs) p1 += static_cast<double>(blk[(c + 1) * bs]) * static_cast<double>(xj[c + 1]);
        }
    }
    return p0 + p1;
}

// (PRE: the diagonal block's part is given as `pre`, added at its place in block
// order; NODIAG: the blocks hold no diagonal block, as in a sweep copy)
constexpr int kFaceUnroll = 8;   // face rectangles up to this many columns take the unrolled row

template <int BS, typename MT, typename VT, bool SKIP = false, bool PRE = false, bool NODIAG = false>
__device__ inline double row_part_face(const int *__restrict__ colidx, const FaceView<MT> &F, int lo, int hi, int g,
                                       int G, int a, int I, int bs_rt, const VT *__restrict__ x, double pre = 0.0) {
    const int bs = Bs<BS>::get(bs_rt);
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    double acc = 0.0;
    int t = lo + g;
    if (t >= hi) return acc;
    // the next block's column and masks load while this block's values and x do
    int J = colidx[t];
    uint64_t m = F.meta[t];
    for (;; t += G) {
        const int tn = t + G;
        int Jn = 0;
        uint64_t mn = 0;
        if (tn < hi) {
            Jn = colidx[tn];
            mn = F.meta[tn];
        }
        const VT *xj = x + static_cast<int64_t>(J) * bs;
        if (!NODIAG && J == I) {
            if constexpr (SKIP) {
                if (tn >= hi) break;
                J = Jn;
                m = mn;
                continue;
            }
            if constexpr (PRE) acc += pre;
            else acc += face_diag_dot<BS, MT, VT>(F, I, a, bs, x);
        } else {
            const uint32_t rm = static_cast<uint32_t>(m);
            if ((rm >> a) & 1u) {
                const uint32_t cm = static_cast<uint32_t>(m >> 32);
                const MT *row = F.vals + static_cast<int64_t>(t) * F.rc + __popc(rm & ((1u << a) - 1u)) * F.cmax;
                double p0 = 0.0, p1 = 0.0;
                if (__popc(cm) <= kFaceUnroll) {
                    // the row's columns first, then all its loads, then the sums: one
                    // memory wait per block instead of one per entry (same order)
                    int cs[kFaceUnroll];
                    uint32_t mm = cm;
#pragma unroll
                    for (int q = 0; q < kFaceUnroll; ++q) {
                        cs[q] = mm ? __ffs(static_cast<int>(mm)) - 1 : -1;
                        mm &= mm - 1u;
                    }
                    double rv[kFaceUnroll], xv[kFaceUnroll];
#pragma unroll
                    for (int q = 0; q < kFaceUnroll; ++q) {
                        rv[q] = cs[q] >= 0 ? static_cast<double>(row[q]) : 0.0;
                        xv[q] = cs[q] >= 0 ? static_cast<double>(xj[cs[q]]) : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < kFaceUnroll; ++q) {
                        if (cs[q] < 0) break;
                        if (cs[q] & 1) p1 += rv[q] * xv[q];
                        else p0 += rv[q] * xv[q];
                    }
                } else {
                    int q = 0;
                    for (uint32_t mm = cm; mm != 0u; mm &= mm - 1u, ++q) {
                        const int c = __ffs(static_cast<int>(mm)) - 1;
                        if (c & 1) p1 += static_cast<double>(row[q]) * static_cast<double>(xj[c]);
                        else p0 += static_cast<double>(row[q]) * static_cast<double>(xj[c]);
                    }
                }
                acc += p0 + p1;
            }
        }
        if (tn >= hi) break;
        J = Jn;
        m = mn;
    }
    return acc;
}

// The same row product over blocks kept by their nonzero rows (RowBlockView):
// block t's row a, when nonzero, is bs entries at vals[off[t] + rank(a) * bs],
// summed exactly as row_part sums it; a zero row's products are exact zeros
// and are left out, so for finite x the result equals row_part's bit for bit.
template <int BS, typename MT, typename VT>
__device__ inline double row_part_rows(const int *__restrict__ colidx, const RowBlockView<MT> &R, int lo, int hi,
                                       int g, int G, int a, int bs_rt, const VT *__restrict__ x) {
    const int bs = Bs<BS>::get(bs_rt);
    const uint32_t below = (1u << a) - 1u;
    double acc = 0.0;
    int t = lo + g;
    if (t >= hi) return acc;
    // the next block's column, mask and offset load while this block's row and x do
    int J = colidx[t];
    uint32_t m = R.mask[t];
    int o = R.off[t];
    for (;;) {
        const int tn = t + G;
        int Jn = 0, on = 0;
        uint32_t mn = 0u;
        if (tn < hi) {
            Jn = colidx[tn];
            mn = R.mask[tn];
            on = R.off[tn];
        }
        if ((m >> a) & 1u) acc += block_row_dot<BS>(R.vals + o + __popc(m & below) * bs, x + static_cast<int64_t>(J) * bs, bs);
        if (tn >= hi) break;
        t = tn;
        J = Jn;
        m = mn;
        o = on;
    }
    return acc;
}

// The same row product read transposed from a TransRows copy: output row I
// owns the stored rows q = qptr[I] + g, + G, ... < qptr[I+1], row q being
// M_JI[c][.] of some source block, to be multiplied by x at src[q] = J bs + c;
// lane a adds M_JI[c][a] x_J[c] (with SKIP, rows with J == skip are left out).
// Four rows per step load together; the sums alternate between two
// accumulators in walk order.
template <int BS, typename MT, typename VT, bool SKIP = false>
__device__ inline double row_part_tr(const TransRowsView<MT> &T, int I, int g, int G, int a, int bs_rt,
                                     const VT *__restrict__ x, int skip = -1) {
    const int bs = Bs<BS>::get(bs_rt);
    const int hi = T.qptr[I + 1];
    double acc0 = 0.0, acc1 = 0.0;
    int q = T.qptr[I] + g;
    for (; q + 3 * G < hi; q += 4 * G) {
        int s[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s[u] = T.src[q + u * G];
            v[u] = static_cast<double>(T.vals[static_cast<int64_t>(q + u * G) * bs + a]);
        }
        if constexpr (SKIP) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (s[u] / bs == skip) continue;
                if (u & 1) acc1 += v[u] * static_cast<double>(x[s[u]]);
                else acc0 += v[u] * static_cast<double>(x[s[u]]);
            }
        } else {
            const double x0 = static_cast<double>(x[s[0]]), x1 = static_cast<double>(x[s[1]]);
            const double x2 = static_cast<double>(x[s[2]]), x3 = static_cast<double>(x[s[3]]);
            acc0 += v[0] * x0;
            acc1 += v[1] * x1;
            acc0 += v[2] * x2;
            acc1 += v[3] * x3;
        }
    }
    for (int u = 0; q < hi; q += G, ++u) {
        const int s = T.src[q];
        const double v = static_cast<double>(T.vals[static_cast<int64_t>(q) * bs + a]);
        if constexpr (SKIP) {
            if (s / bs == skip) continue;
        }
        if (u & 1) acc1 += v * static_cast<double>(x[s]);
        else acc0 += v * static_cast<double>(x[s]);
    }
    return acc0 + acc1;
}

// Row I's product with x (SKIP: without its diagonal block).
template <int BS, bool FACE, typename MT, typename VT, bool SKIP = false>
__device__ inline double row_product(const int *__restrict__ colidx, const MT *__restrict__ vals,
                                     const FaceView<MT> &F, int lo, int hi, int g, int G, int a, int I, int bs_rt,
                                     const VT *__restrict__ x) {
    if constexpr (FACE) return row_part_face<BS, MT, VT, SKIP>(colidx, F, lo, hi, g, G, a, I, bs_rt, x);
    else return row_part<BS, MT, VT, SKIP>(colidx, vals, lo, hi, g, G, a, bs_rt, x, I);
}

// D_I^{-1} t (TRANS: D_I^{-T} t) for scalar row a, with t in LDS.
template <int BS, bool TRANS>
__device__ inline double apply_dinv(const double *__restrict__ D, const double *t, int a, int bs) {
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int c = 0; c < (BS > 0 ? BS : kMaxBs); c += 2) {
        if (BS == 0 && c >= bs) break;
        if (TRANS) {
            d0 += D[c * bs + a] * t[c];
            if (c + 1 < bs) d1 += D[(c + 1) * bs + a] * t[c + 1];
        } else {
            d0 += D[a * bs + c] * t[c];
            if (c + 1 < bs) d1 += D[a * bs + c + 1] * t[c + 1];
        }
    }
    return d0 + d1;
}

// This lane's row of a D^{-1} block (column for D^{-T}): in registers for small
// blocks (up to 25 with WIDE: the face-compressed sweep, whose row product is
// short), loaded before the row product so its latency overlaps it; apply()
// gives apply_dinv's sums either way.
template <int BS, bool TRANS, bool WIDE = false>
struct DinvRow {
    static constexpr bool kPre = BS > 0 && (BS <= 16 || (WIDE && BS <= 25));
    double d[kPre ? BS : 1];
    __device__ void load(const double *D, int a) {
        if constexpr (kPre) {
#pragma unroll
            for (int c = 0; c < BS; ++c) d[c] = TRANS ? D[c * BS + a] : D[a * BS + c];
        }
    }
    __device__ double apply(const double *D, const double *t, int a, int bs) const {
        if constexpr (kPre) {
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int c = 0; c < BS; c += 2) {
                d0 += d[c] * t[c];
                if (c + 1 < BS) d1 += d[c + 1] * t[c + 1];
            }
            return d0 + d1;
        } else {
            return apply_dinv<BS, TRANS>(D, t, a, bs);
        }
    }
};

struct Lane {
    int lr, g, a;   // local row, group, scalar row in block
    bool valid;     // lr < rows per workgroup
};

__device__ inline Lane lane_of(int G, int bs) {
    Lane L;
    const int per_row = G * bs;
    L.lr = threadIdx.x / per_row;
    const int rem = threadIdx.x - L.lr * per_row;
    L.g = rem / bs;
    L.a = rem - L.g * bs;
    L.valid = L.lr < kThreads / per_row;
    return L;
}

// Sum the G partials of (lr, a) into the g == 0 lane (returns the total there).
__device__ inline double reduce_groups(double v, const Lane &L, int G, int bs, double *part) {
    if (G == 1) return v;
    part[threadIdx.x] = v;
    __syncthreads();
    double s = v;
    if (L.valid && L.g == 0)
        for (int g = 1; g < G; ++g) s += part[threadIdx.x + g * bs];
    return s;
}

__device__ inline double block_reduce_sum(double v, double *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < static_cast<int>(blockDim.x) / 64; ++k) s += lds[k];
    return s;   // valid in thread 0
}

// r = b - A x (b == nullptr: r = A x); r_lo (if given) receives r rounded to float.
template <int BS, typename MT, typename VT, bool FACE = false>
__global__ __launch_bounds__(kThreads) void k_residual(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                      const MT *__restrict__ vals, int nb, int bs_rt, int G,
                                                      const VT *__restrict__ b, const VT *__restrict__ x,
                                                      VT *__restrict__ r, float *__restrict__ r_lo, Gate gate,
                                                      FaceView<MT> face) {
    __shared__ double part[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int I = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const bool act = L.valid && I < nb && live(gate, I);
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    const double bv = (act && L.g == 0 && b) ? static_cast<double>(b[o]) : 0.0;   // loads during the product
    double acc = 0.0;
    if constexpr (FACE) {
        if (act && G == 1) {   // the diagonal block (most of the row's bytes) loads first, at a known place
            const double pd = face_diag_dot<BS, MT, VT>(face, I, L.a, bs, x);
            acc = row_part_face<BS, MT, VT, false, true>(colidx, face, rowptr[I], rowptr[I + 1], 0, 1, L.a, I, bs, x,
                                                         pd);
        } else if (act) {
            acc = row_part_face<BS, MT, VT>(colidx, face, rowptr[I], rowptr[I + 1], L.g, G, L.a, I, bs, x);
        }
    } else {
        acc = act ? row_product<BS, FACE>(colidx, vals, face, rowptr[I], rowptr[I + 1], L.g, G, L.a, I, bs, x) : 0.0;
    }
    acc = reduce_groups(acc, L, G, bs, part);
    if (act && L.g == 0) {
        const double rv = b ? bv - acc : acc;
        r[o] = static_cast<VT>(rv);
        if (r_lo) r_lo[o] = static_cast<float>(rv);
    }
}

// One Jacobi sweep over the listed rows (list == nullptr: rows with cf == only_cf;
// the other rows copy e_in): e_out_I = D_I^{-1} (r_I - sum_{J != I} A_IJ e_in_J),
// or with D_I^{-T} (TRANS: the sweeps of the transposed cycle, with A^T's
// rows).  D_I is the diagonal block A_II, so this is e_in_I + D_I^{-1} (r_I -
// (A e_in)_I) without the diagonal block's product and its cancellation: the
// sweep reads neither A_II nor e_in_I (the two agree up to rounding).
template <int BS, typename MT, typename VT, bool TRANS, bool FACE>
__device__ inline void relax_rows(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                  const MT *__restrict__ vals, const double *__restrict__ dinv, int nb, int bs_rt,
                                  int G, const VT *__restrict__ r, const VT *__restrict__ ein, VT *__restrict__ eout,
                                  const int *__restrict__ list, int nlist, const int8_t *__restrict__ cf, int only_cf,
                                  Gate gate, const FaceView<MT> &face) {
    __shared__ double part[kThreads];
    __shared__ double tb[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int idx = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const int N = list ? nlist : nb;
    int I = -1;
    if (L.valid && idx < N) I = list ? list[idx] : idx;
    if (I >= 0 && !live(gate, I)) I = -1;   // a stopped system: nothing to do
    const bool upd = I >= 0 && (list != nullptr || cf[I] == only_cf);
    // loads that do not depend on the row product go out first: this lane's
    // row of D_I^{-1} and r (e_in for rows that only copy it)
    DinvRow<BS, TRANS> dr;
    const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    double rv = 0.0, ev = 0.0;
    if (I >= 0 && L.g == 0) {
        if (!upd) {
            ev = static_cast<double>(ein[o]);
        } else {
            rv = static_cast<double>(r[o]);
            dr.load(D, L.a);
        }
    }
    double acc = upd ? row_product<BS, FACE, MT, VT, true>(colidx, vals, face, rowptr[I], rowptr[I + 1], L.g, G, L.a,
                                                          I, bs, ein)
                     : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    if (upd && L.g == 0) tb[L.lr * bs + L.a] = rv - acc;
    __syncthreads();
    if (I >= 0 && L.g == 0) {
        if (upd) eout[o] = static_cast<VT>(dr.apply(D, tb + L.lr * bs, L.a, bs));
        else eout[o] = static_cast<VT>(ev);
    }
}

// The same sweep over the F list from a sweep copy: row f of the copy is F row
// I = flist[f] without its diagonal block (face rectangles, or blocks by their
// nonzero rows), D_I^{-1} sits at position f.  The
// copy keeps each row's blocks in order, so with one lane group per row the
// sums are relax_rows' bit for bit (with G > 1 the blocks are dealt to the
// groups from the row's start, which moves the diagonal's gap).
template <int BS, typename MT, typename VT, bool TRANS, bool FACE>
__device__ inline void sweep_rows(const SweepView<MT> &S, const int *__restrict__ flist, int nF, int bs_rt, int G,
                                  const VT *__restrict__ r, const VT *__restrict__ ein, VT *__restrict__ eout,
                                  Gate gate) {
    __shared__ double part[kThreads];
    __shared__ double tb[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int f = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    int I = -1;
    if (L.valid && f < nF) I = flist[f];
    if (I >= 0 && !live(gate, I)) I = -1;
    // the copy's inverse block holds the coefficient of input c for output a at
    // c * bs + a in both directions (D^{-1} transposed, or D^{-1} for D^{-T})
    DinvRow<BS, true, FACE> dr;
    const double *D = S.dinv + static_cast<int64_t>(f) * bs * bs;
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    double rv = 0.0;
    if (I >= 0 && L.g == 0) {
        rv = static_cast<double>(r[o]);
        dr.load(D, L.a);
    }
    double acc = 0.0;
    if (I >= 0) {
        const int lo = S.rowptr[f], hi = S.rowptr[f + 1];
        if constexpr (FACE)
            acc = row_part_face<BS, MT, VT, false, false, true>(
                S.colidx, FaceView<MT>{S.meta, S.vals, nullptr, S.cmax, S.rc}, lo, hi, L.g, G, L.a, -1, bs, ein);
        else
            acc = row_part_rows<BS, MT, VT>(S.colidx, S.rows, lo, hi, L.g, G, L.a, bs, ein);
    }
    acc = reduce_groups(acc, L, G, bs, part);
    if (I >= 0 && L.g == 0) tb[L.lr * bs + L.a] = rv - acc;
    __syncthreads();
    if (I >= 0 && L.g == 0) eout[o] = static_cast<VT>(dr.apply(D, tb + L.lr * bs, L.a, bs));
}

template <int BS, typename MT, typename VT, bool FACE = false>
__global__ __launch_bounds__(kThreads) void k_sweep(SweepView<MT> S, const int *__restrict__ flist, int nF,
                                                   int bs_rt, int G, const VT *__restrict__ r,
                                                   const VT *__restrict__ ein, VT *__restrict__ eout, Gate gate) {
    sweep_rows<BS, MT, VT, false, FACE>(S, flist, nF, bs_rt, G, r, ein, eout, gate);
}

template <int BS, typename MT, typename VT, bool FACE = false>
__global__ __launch_bounds__(kThreads) void k_sweep_T(SweepView<MT> S, const int *__restrict__ flist, int nF,
                                                     int bs_rt, int G, const VT *__restrict__ r,
                                                     const VT *__restrict__ ein, VT *__restrict__ eout, Gate gate) {
    sweep_rows<BS, MT, VT, true, FACE>(S, flist, nF, bs_rt, G, r, ein, eout, gate);
}

// The first transposed F sweep from a zero guess (F relaxation only): e1_F =
// D_F^{-T} r_F; every other row is zero in e0 and e1.  No matrix entries are
// read: the sweep's product with A^T is a product with zero.
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_relax_T_first(const double *__restrict__ dinv,
                                                           const VT *__restrict__ r, const int8_t *__restrict__ cf,
                                                           VT *__restrict__ e0, VT *__restrict__ e1, int nb, int bs,
                                                           Gate gate) {
    const int64_t gi = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (gi >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(gi / bs);
    const int a = static_cast<int>(gi - static_cast<int64_t>(I) * bs);
    if (!live(gate, I)) return;
    if (cf[I] == 0) {
        const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
        const VT *rI = r + static_cast<int64_t>(I) * bs;
        double d0 = 0.0, d1 = 0.0;
        for (int c = 0; c < bs; c += 2) {
            d0 += D[c * bs + a] * static_cast<double>(rI[c]);
            if (c + 1 < bs) d1 += D[(c + 1) * bs + a] * static_cast<double>(rI[c + 1]);
        }
        e1[gi] = static_cast<VT>(d0 + d1);
    } else {
        e0[gi] = VT(0);
        e1[gi] = VT(0);
    }
}

template <int BS, typename MT, typename VT, bool FACE = false>
__global__ __launch_bounds__(kThreads) void k_relax(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                   const MT *__restrict__ vals, const double *__restrict__ dinv,
                                                   int nb, int bs_rt, int G, const VT *__restrict__ r,
                                                   const VT *__restrict__ ein, VT *__restrict__ eout,
                                                   const int *__restrict__ list, int nlist,
                                                   const int8_t *__restrict__ cf, int only_cf, Gate gate,
                                                   FaceView<MT> face) {
    relax_rows<BS, MT, VT, false, FACE>(rowptr, colidx, vals, dinv, nb, bs_rt, G, r, ein, eout, list, nlist, cf,
                                        only_cf, gate, face);
}

template <int BS, typename MT, typename VT, bool FACE = false>
__global__ __launch_bounds__(kThreads) void k_relax_T(const int *__restrict__ rowptr, const int *__restrict__ colidx,
                                                     const MT *__restrict__ vals, const double *__restrict__ dinv,
                                                     int nb, int bs_rt, int G, const VT *__restrict__ r,
                                                     const VT *__restrict__ ein, VT *__restrict__ eout,
                                                     const int *__restrict__ list, int nlist,
                                                     const int8_t *__restrict__ cf, int only_cf, Gate gate,
                                                     FaceView<MT> face) {
    relax_rows<BS, MT, VT, true, FACE>(rowptr, colidx, vals, dinv, nb, bs_rt, G, r, ein, eout, list, nlist, cf,
                                       only_cf, gate, face);
}

// The interpolation e = P e_c and the first F sweep in one launch (small
// levels, where launches cost more than their work): e0 = P e_c on every row;
// e1 = D^{-1}(r - sum_{J != I} A_IJ e0_J) on F rows, e1 = e0 on C rows --
// what the two kernels leave, computed in the same order.
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_relax_interp(const int *__restrict__ rowptr,
                                                          const int *__restrict__ colidx, const MT *__restrict__ vals,
                                                          const double *__restrict__ dinv, int nb, int bs_rt, int G,
                                                          const VT *__restrict__ r, const int *__restrict__ pmap,
                                                          const VT *__restrict__ ec, const int8_t *__restrict__ cf,
                                                          VT *__restrict__ e0, VT *__restrict__ e1, Gate gate) {
    __shared__ double part[kThreads];
    __shared__ double tb[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    int I = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    if (!L.valid || I >= nb || !live(gate, I)) I = -1;
    const bool upd = I >= 0 && cf[I] == 0;
    const PmapSrc<VT> src{ec, pmap, bs};
    double acc = upd ? row_part_src<BS, MT, VT, PmapSrc<VT>, true>(colidx, vals, rowptr[I], rowptr[I + 1], L.g, G,
                                                                   L.a, bs, src, I)
                     : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    VT v = VT(0);
    if (I >= 0 && L.g == 0) {
        const int p = pmap[I];
        v = p >= 0 ? ec[static_cast<int64_t>(p) * bs + L.a] : VT(0);
        if (upd) tb[L.lr * bs + L.a] = static_cast<double>(r[o]) - acc;
    }
    __syncthreads();
    if (I >= 0 && L.g == 0) {
        e0[o] = v;
        if (upd) {
            const double d = apply_dinv<BS, false>(dinv + static_cast<int64_t>(I) * bs * bs, tb + L.lr * bs, L.a, bs);
            e1[o] = static_cast<VT>(d);
        } else {
            e1[o] = v;
        }
    }
}

// rc_i = r_{cpts[i]} + sum_t Z_it r_{col t} (RB: Z's blocks by their nonzero rows)
template <int BS, typename MT, typename VT, bool RB = false>
__global__ __launch_bounds__(kThreads) void k_restrict(const int *__restrict__ zrp, const int *__restrict__ zcol,
                                                      const MT *__restrict__ zval, int nc, int bs_rt, int G,
                                                      const VT *__restrict__ r, const int *__restrict__ cpts,
                                                      VT *__restrict__ rc, Gate gate, RowBlockView<MT> zr) {
    __shared__ double part[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int i = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const bool act = L.valid && i < nc && live(gate, i);
    // r_C loads while the row product runs
    double rv = 0.0;
    if (act && L.g == 0) rv = static_cast<double>(r[static_cast<int64_t>(cpts[i]) * bs + L.a]);
    double acc = 0.0;
    if (act) {
        if constexpr (RB) acc = row_part_rows<BS, MT, VT>(zcol, zr, zrp[i], zrp[i + 1], L.g, G, L.a, bs, r);
        else acc = row_part<BS>(zcol, zval, zrp[i], zrp[i + 1], L.g, G, L.a, bs, r);
    }
    acc = reduce_groups(acc, L, G, bs, part);
    if (act && L.g == 0) rc[static_cast<int64_t>(i) * bs + L.a] = static_cast<VT>(rv + acc);
}

// The same restriction with one lane per stored row of Z (block sizes >= 8,
// where a block row's lanes would mostly wait: a Z block has a few nonzero
// rows, a face's worth).  The R coarse rows of a workgroup own the stored rows
// [q0, q1) of their blocks, contiguous and in block order (RB: Z's blocks by
// their nonzero rows, row k of block t at q = off[t] / bs + k; else all bs
// rows of block t at q = t bs + a).  In passes of up to kCrCap stored rows:
// (1) each block's lane writes the block's column against its stored rows in
// LDS; (2) each lane forms one stored row's product with r_J (split by column
// parity as the row products are); (3) output lane (i, a) adds the products of
// row i's blocks that store row a, in block order, to its total.
constexpr int kCrCap = 1024;
constexpr int kCrBlk = 512;   // blocks of a workgroup whose row masks and first rows are staged in LDS

template <int BS, typename MT, typename VT, bool RB>
__global__ __launch_bounds__(kThreads) void k_restrict_cr(const int *__restrict__ zrp, const int *__restrict__ zcol,
                                                         const MT *__restrict__ zval, int nc, int bs_rt, int R,
                                                         const VT *__restrict__ r, const int *__restrict__ cpts,
                                                         VT *__restrict__ rc, Gate gate, RowBlockView<MT> zr) {
    __shared__ double dot[kCrCap];
    __shared__ int qcol[kCrCap];
    __shared__ uint32_t bmask[kCrBlk];
    __shared__ int bq[kCrBlk + 1];
    __shared__ int rowb[2 * kThreads / 8 + 1];
    const int bs = Bs<BS>::get(bs_rt);
    const int i0 = blockIdx.x * R;
    if (i0 >= nc) return;   // (the whole workgroup)
    const int i1 = min(nc, i0 + R);
    // a workgroup whose rows all belong to stopped systems does nothing
    if (gate.active && !__syncthreads_or(static_cast<int>(threadIdx.x) < i1 - i0 && live(gate, i0 + threadIdx.x)))
        return;
    const int t0 = zrp[i0], t1 = zrp[i1];
    const MT *vals = RB ? zr.vals : zval;
    auto first_row_g = [&](int t) { return RB ? zr.off[t] / bs : t * bs; };
    // the rows' block ranges and (when few enough) the blocks' masks and first stored rows, in LDS
    const bool staged = t1 - t0 <= kCrBlk;
    for (int k = threadIdx.x; k <= i1 - i0; k += kThreads) rowb[k] = zrp[i0 + k];
    if (staged)
        for (int t = t0 + static_cast<int>(threadIdx.x); t <= t1; t += kThreads) {
            bq[t - t0] = first_row_g(t);
            if (RB && t < t1) bmask[t - t0] = zr.mask[t];
        }
    const int nout = (i1 - i0) * bs;   // <= 2 kThreads (host)
    // r_C loads while the products run
    double rv[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * kThreads;
        if (k < nout) {
            const int i = i0 + k / bs, a = k - (k / bs) * bs;
            rv[j] = static_cast<double>(r[static_cast<int64_t>(cpts[i]) * bs + a]);
        }
    }
    __syncthreads();
    auto first_row = [&](int t) { return staged ? bq[t - t0] : first_row_g(t); };
    const int q0 = first_row(t0), q1 = first_row(t1);
    double acc[2] = {0.0, 0.0};
    for (int qc = q0; qc < q1; qc += kCrCap) {
        const int qe = min(q1, qc + kCrCap);
        for (int t = t0 + static_cast<int>(threadIdx.x); t < t1; t += kThreads) {
            const int lo = max(first_row(t), qc), hi = min(first_row(t + 1), qe);
            if (lo < hi) {
                const int J = zcol[t];
                for (int q = lo; q < hi; ++q) qcol[q - qc] = J;
            }
        }
        __syncthreads();
        for (int q = qc + static_cast<int>(threadIdx.x); q < qe; q += kThreads)
            dot[q - qc] = block_row_dot<BS>(vals + static_cast<int64_t>(q) * bs, r + static_cast<int64_t>(qcol[q - qc]) * bs,
                                            bs);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = static_cast<int>(threadIdx.x) + j * kThreads;
            if (k < nout) {
                const int il = k / bs, a = k - (k / bs) * bs;
                const int hi = rowb[il + 1];
                for (int t = rowb[il]; t < hi; ++t) {
                    int q;
                    if constexpr (RB) {
                        const uint32_t m = staged ? bmask[t - t0] : zr.mask[t];
                        if (!((m >> a) & 1u)) continue;
                        q = first_row(t) + __popc(m & ((1u << a) - 1u));
                    } else {
                        q = t * bs + a;
                    }
                    if (q >= qc && q < qe) acc[j] += dot[q - qc];
                }
            }
        }
        if (qe < q1) __syncthreads();   // the next pass rewrites the LDS rows
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * kThreads;
        if (k < nout) {
            const int i = i0 + k / bs, a = k - (k / bs) * bs;
            if (live(gate, i)) rc[static_cast<int64_t>(i) * bs + a] = static_cast<VT>(rv[j] + acc[j]);
        }
    }
}

// The F sweep from a sweep copy stored by nonzero rows, one lane per stored
// row (block sizes >= 8 on the larger levels), as k_restrict_cr forms Z r: the
// R F rows f0 .. of a workgroup own the stored rows of their blocks; per pass
// each lane forms one stored row's product with e_in, and output lane (f, a)
// adds those of row f's blocks that store row a, in block order (the sums
// sweep_rows forms at one lane group).  Then t = r_I - sum goes to LDS and
// e_out_I = D^{-1} t (or D^{-T} t: the copy's inverse block holds the
// coefficient of input c for output a at c bs + a either way).
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_sweep_cr(SweepView<MT> S, const int *__restrict__ flist, int nF,
                                                      int bs_rt, int R, const VT *__restrict__ r,
                                                      const VT *__restrict__ ein, VT *__restrict__ eout, Gate gate) {
    __shared__ double dot[kCrCap];
    __shared__ int qcol[kCrCap];
    __shared__ double tb[2 * kThreads];
    __shared__ uint32_t bmask[kCrBlk];
    __shared__ int bq[kCrBlk + 1];
    __shared__ int rowb[2 * kThreads / 8 + 1];
    const int bs = Bs<BS>::get(bs_rt);
    const int f0 = blockIdx.x * R;
    if (f0 >= nF) return;   // (the whole workgroup)
    const int f1 = min(nF, f0 + R);
    // a workgroup whose rows all belong to stopped systems does nothing
    if (gate.active &&
        !__syncthreads_or(static_cast<int>(threadIdx.x) < f1 - f0 && live(gate, flist[f0 + threadIdx.x])))
        return;
    const int t0 = S.rowptr[f0], t1 = S.rowptr[f1];
    const RowBlockView<MT> &RB = S.rows;
    // the rows' block ranges and (when few enough) the blocks' masks and first stored rows, in LDS
    const bool staged = t1 - t0 <= kCrBlk;
    for (int k = threadIdx.x; k <= f1 - f0; k += kThreads) rowb[k] = S.rowptr[f0 + k];
    if (staged)
        for (int t = t0 + static_cast<int>(threadIdx.x); t <= t1; t += kThreads) {
            bq[t - t0] = RB.off[t] / bs;
            if (t < t1) bmask[t - t0] = RB.mask[t];
        }
    const int nout = (f1 - f0) * bs;   // <= 2 kThreads (host)
    // r_I loads while the products run
    double rv[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * kThreads;
        if (k < nout) rv[j] = static_cast<double>(r[static_cast<int64_t>(flist[f0 + k / bs]) * bs + (k - (k / bs) * bs)]);
    }
    __syncthreads();
    auto first_row = [&](int t) { return staged ? bq[t - t0] : RB.off[t] / bs; };
    const int q0 = first_row(t0), q1 = first_row(t1);
    double acc[2] = {0.0, 0.0};
    for (int qc = q0; qc < q1; qc += kCrCap) {
        const int qe = min(q1, qc + kCrCap);
        for (int t = t0 + static_cast<int>(threadIdx.x); t < t1; t += kThreads) {
            const int lo = max(first_row(t), qc), hi = min(first_row(t + 1), qe);
            if (lo < hi) {
                const int J = S.colidx[t];
                for (int q = lo; q < hi; ++q) qcol[q - qc] = J;
            }
        }
        __syncthreads();
        for (int q = qc + static_cast<int>(threadIdx.x); q < qe; q += kThreads)
            dot[q - qc] = block_row_dot<BS>(RB.vals + static_cast<int64_t>(q) * bs,
                                            ein + static_cast<int64_t>(qcol[q - qc]) * bs, bs);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = static_cast<int>(threadIdx.x) + j * kThreads;
            if (k < nout) {
                const int fl = k / bs, a = k - (k / bs) * bs;
                const int hi = rowb[fl + 1];
                for (int t = rowb[fl]; t < hi; ++t) {
                    const uint32_t m = staged ? bmask[t - t0] : RB.mask[t];
                    if (!((m >> a) & 1u)) continue;
                    const int q = first_row(t) + __popc(m & ((1u << a) - 1u));
                    if (q >= qc && q < qe) acc[j] += dot[q - qc];
                }
            }
        }
        if (qe < q1) __syncthreads();   // the next pass rewrites the LDS rows
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * kThreads;
        if (k < nout) tb[k] = rv[j] - acc[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = static_cast<int>(threadIdx.x) + j * kThreads;
        if (k < nout) {
            const int fl = k / bs, a = k - fl * bs;
            const int I = flist[f0 + fl];
            if (live(gate, I)) {
                const double *D = S.dinv + static_cast<int64_t>(f0 + fl) * bs * bs + a;
                const double *t = tb + fl * bs;
                double d0 = 0.0, d1 = 0.0;
                if constexpr (BS > 0) {
#pragma unroll
                    for (int c = 0; c < BS; c += 2) {
                        d0 += D[c * BS] * t[c];
                        if (c + 1 < BS) d1 += D[(c + 1) * BS] * t[c + 1];
                    }
                } else {
                    for (int c = 0; c < bs; c += 2) {
                        d0 += D[c * bs] * t[c];
                        if (c + 1 < bs) d1 += D[(c + 1) * bs] * t[c + 1];
                    }
                }
                eout[static_cast<int64_t>(I) * bs + a] = static_cast<VT>(d0 + d1);
            }
        }
    }
}

// y_I += [I is C] yc_{cidx I} + sum_t (Z^T)_It yc_{col t}
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_interp_T(const int *__restrict__ ztrp, const int *__restrict__ ztcol,
                                                      const MT *__restrict__ ztval, int nb, int bs_rt, int G,
                                                      const int *__restrict__ cidx, const VT *__restrict__ yc,
                                                      VT *__restrict__ y, Gate gate) {
    __shared__ double part[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int I = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const bool act = L.valid && I < nb && live(gate, I);
    // y_I and the C term load while the row product runs
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    double yv = 0.0, cv = 0.0;
    int ci = -1;
    if (act && L.g == 0) {
        yv = static_cast<double>(y[o]);
        ci = cidx[I];
        if (ci >= 0) cv = static_cast<double>(yc[static_cast<int64_t>(ci) * bs + L.a]);
    }
    double acc = act ? row_part<BS>(ztcol, ztval, ztrp[I], ztrp[I + 1], L.g, G, L.a, bs, yc) : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    if (act && L.g == 0) {
        if (ci >= 0) acc += cv;
        y[o] = static_cast<VT>(yv + acc);
    }
}

// The transposed cycle's products from TransRows copies (coarse levels):
// s = g - A^T y for every row, where y vanishes outside the source rows the
// copy keeps (the F rows: the transposed F sweeps change only those)
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_residual_tr(TransRowsView<MT> T, int bs_rt, int G,
                                                         const VT *__restrict__ g, const VT *__restrict__ y,
                                                         VT *__restrict__ sout, Gate gate) {
    __shared__ double part[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int I = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const bool act = L.valid && I < T.nrows && live(gate, I);
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    const double gv = (act && L.g == 0) ? static_cast<double>(g[o]) : 0.0;
    double acc = act ? row_part_tr<BS, MT, VT>(T, I, L.g, G, L.a, bs, y) : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    if (act && L.g == 0) sout[o] = static_cast<VT>(gv - acc);
}

// transposed F sweep over the listed rows: y_out_I = D_I^{-T}(g_I - sum_{J != I} (A^T)_IJ y_in_J)
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_sweep_tr(TransRowsView<MT> T, const double *__restrict__ dinv,
                                                      const int *__restrict__ list, int nlist, int bs_rt, int G,
                                                      const VT *__restrict__ g, const VT *__restrict__ yin,
                                                      VT *__restrict__ yout, Gate gate) {
    __shared__ double part[kThreads];
    __shared__ double tb[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int f = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    int I = -1;
    if (L.valid && f < nlist) I = list[f];
    if (I >= 0 && !live(gate, I)) I = -1;
    DinvRow<BS, true> dr;   // D_I^{-T}: the coefficient of input c for output a is D^{-1}[c][a]
    const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    double gv = 0.0;
    if (I >= 0 && L.g == 0) {
        gv = static_cast<double>(g[o]);
        dr.load(D, L.a);
    }
    double acc = I >= 0 ? row_part_tr<BS, MT, VT, true>(T, I, L.g, G, L.a, bs, yin, I) : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    if (I >= 0 && L.g == 0) tb[L.lr * bs + L.a] = gv - acc;
    __syncthreads();
    if (I >= 0 && L.g == 0) yout[o] = static_cast<VT>(dr.apply(D, tb + L.lr * bs, L.a, bs));
}

// y_I += [I is C] yc_{cidx I} + (Z^T yc)_I from Z's TransRows copy
template <int BS, typename MT, typename VT>
__global__ __launch_bounds__(kThreads) void k_interp_tr(TransRowsView<MT> T, int bs_rt, int G,
                                                       const int *__restrict__ cidx, const VT *__restrict__ yc,
                                                       VT *__restrict__ y, Gate gate) {
    __shared__ double part[kThreads];
    const int bs = Bs<BS>::get(bs_rt);
    const Lane L = lane_of(G, bs);
    const int I = blockIdx.x * (kThreads / (G * bs)) + L.lr;
    const bool act = L.valid && I < T.nrows && live(gate, I);
    const int64_t o = static_cast<int64_t>(I) * bs + L.a;
    double yv = 0.0, cv = 0.0;
    int ci = -1;
    if (act && L.g == 0) {
        yv = static_cast<double>(y[o]);
        ci = cidx[I];
        if (ci >= 0) cv = static_cast<double>(yc[static_cast<int64_t>(ci) * bs + L.a]);
    }
    double acc = act ? row_part_tr<BS, MT, VT>(T, I, L.g, G, L.a, bs, yc) : 0.0;
    acc = reduce_groups(acc, L, G, bs, part);
    if (act && L.g == 0) {
        if (ci >= 0) acc += cv;
        y[o] = static_cast<VT>(yv + acc);
    }
}

template <typename VT>
__global__ __launch_bounds__(kThreads) void k_interp(const int *__restrict__ pmap, const VT *__restrict__ ec,
                                                    VT *__restrict__ e0, VT *__restrict__ e1, int nb, int bs,
                                                    Gate gate) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(g / bs);
    if (!live(gate, I)) return;
    const int a = static_cast<int>(g - static_cast<int64_t>(I) * bs);
    const int p = pmap[I];
    const VT v = (p >= 0) ? ec[static_cast<int64_t>(p) * bs + a] : VT(0);
    e0[g] = v;
    e1[g] = v;
}

// sc_j = sum over fine blocks I with pmap(I) = j of s_I
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_restrict_T(const int *__restrict__ ptptr, const int *__restrict__ ptidx,
                                                        const VT *__restrict__ s, VT *__restrict__ sc, int nc,
                                                        int bs, Gate gate) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nc) * bs) return;
    const int j = static_cast<int>(g / bs);
    if (!live(gate, j)) return;
    const int a = static_cast<int>(g - static_cast<int64_t>(j) * bs);
    double acc = 0.0;
    for (int t = ptptr[j]; t < ptptr[j + 1]; ++t) acc += static_cast<double>(s[static_cast<int64_t>(ptidx[t]) * bs + a]);
    sc[g] = static_cast<VT>(acc);
}

// y0 = y1 = (FC ? [D_C^{-T} g_C ; 0] : 0)
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_init_T(const double *__restrict__ dinv, const VT *__restrict__ g,
                                                    const int8_t *__restrict__ cf, int fc, VT *__restrict__ y0,
                                                    VT *__restrict__ y1, int nb, int bs, Gate gate) {
    const int64_t gi = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (gi >= static_cast<int64_t>(nb) * bs) return;
    const int I = static_cast<int>(gi / bs);
    if (!live(gate, I)) return;
    const int a = static_cast<int>(gi - static_cast<int64_t>(I) * bs);
    double v = 0.0;
    if (fc && cf[I] == 1) {
        const double *D = dinv + static_cast<int64_t>(I) * bs * bs;
        const VT *gI = g + static_cast<int64_t>(I) * bs;
        for (int c = 0; c < bs; ++c) v += D[c * bs + a] * static_cast<double>(gI[c]);
    }
    y0[gi] = static_cast<VT>(v);
    y1[gi] = static_cast<VT>(v);
}

template <typename VT>
__global__ __launch_bounds__(kThreads) void k_axpy(double *__restrict__ x, const VT *__restrict__ e, int64_t n) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g < n) x[g] += static_cast<double>(e[g]);
}

template <typename VT>
__global__ __launch_bounds__(kThreads) void k_axpy_active(double *__restrict__ x, const VT *__restrict__ e, int64_t n,
                                                         int bs, const int *__restrict__ bsys,
                                                         const int *__restrict__ active) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= n) return;
    const int sys = bsys ? bsys[g / bs] : 0;
    if (active[sys]) x[g] += static_cast<double>(e[g]);
}

// y_k = M_k x_k for dense segment k = blockIdx.y (order n[k], at M + off[k],
// vectors at dof0[k]) with a double M: one wave per row.
template <typename VT>
__global__ __launch_bounds__(256) void k_dense_mv(const double *__restrict__ M, const int64_t *__restrict__ off,
                                                 const int *__restrict__ dof0, const int *__restrict__ nn,
                                                 const VT *__restrict__ x, VT *__restrict__ y,
                                                 const int *__restrict__ sys, const int *__restrict__ active) {
    const int k = blockIdx.y;
    if (active && !active[sys ? sys[k] : 0]) return;
    const int n = nn[k];
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const double *m = M + off[k] + static_cast<int64_t>(row) * n;
    const VT *xk = x + dof0[k];
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += m[j] * static_cast<double>(xk[j]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) y[dof0[k] + row] = static_cast<VT>(s);
}

// part[c] = sum of v^2 over chunk c (dofs clo[c] .. clo[c] + clen[c] - 1)
__global__ __launch_bounds__(kThreads) void k_seg_sumsq(const double *__restrict__ v, const int64_t *__restrict__ clo,
                                                       const int *__restrict__ clen, double *__restrict__ part) {
    __shared__ double lds[kThreads / 64];
    const int c = blockIdx.x;
    const double *p = v + clo[c];
    const int len = clen[c];
    double acc = 0.0;
    for (int i = threadIdx.x; i < len; i += kThreads) acc += p[i] * p[i];
    const double t = block_reduce_sum(acc, lds);
    if (threadIdx.x == 0) part[c] = t;
}

// Sum of the chunk sums of system blockIdx.x (fixed order: lane-strided, then
// a wave reduction tree), valid in thread 0.  One wave per system.
__device__ inline double seg_total(const double *__restrict__ part, const int *__restrict__ cptr, int sys) {
    double ss = 0.0;
    for (int c = cptr[sys] + static_cast<int>(threadIdx.x); c < cptr[sys + 1]; c += 64) ss += part[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
    return ss;
}

// dst = src (ADD: dst += src) on the rows of live systems
template <typename VT, bool ADD>
__global__ __launch_bounds__(kThreads) void k_vec_copy(VT *__restrict__ dst, const VT *__restrict__ src, int nb,
                                                      int bs, Gate gate) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (g >= static_cast<int64_t>(nb) * bs) return;
    if (!live(gate, static_cast<int>(g / bs))) return;
    if (ADD) dst[g] = static_cast<VT>(static_cast<double>(dst[g]) + static_cast<double>(src[g]));
    else dst[g] = src[g];
}

// status codes as in the public header: 0 OK, 3 not converged, 4 non-finite
constexpr int kStOk = 0, kStNoConv = 3, kStNumeric = 4;

// Start of a batched solve, one wave per system: ||b_sys||, activity, status.
__global__ __launch_bounds__(64) void k_seg_init(const double *__restrict__ part, const int *__restrict__ cptr,
                                                double *__restrict__ bn, double *__restrict__ last,
                                                int *__restrict__ active, int *__restrict__ status,
                                                int *__restrict__ iters, int *__restrict__ nact_acc) {
    const int sys = blockIdx.x;
    const double b = sqrt(seg_total(part, cptr, sys));
    if (threadIdx.x != 0) return;
    bn[sys] = b;
    last[sys] = 1.0;
    iters[sys] = 0;
    if (!isfinite(b)) {
        active[sys] = 0;
        status[sys] = kStNumeric;
    } else if (b == 0.0) {   // x = 0 solves it
        active[sys] = 0;
        status[sys] = kStOk;
        last[sys] = 0.0;
    } else {
        active[sys] = 1;
        status[sys] = kStNoConv;
        atomicAdd(nact_acc, 1);
    }
}

// After iteration *it, one wave per system: relative residual of an active
// system, recorded in hist[sys * hist_cap + it]; converged or non-finite
// systems stop.
// With one system (tick != 0) the same wave then advances the counters as
// k_seg_tick would, saving a launch per iteration.
__global__ __launch_bounds__(64) void k_seg_check(const double *__restrict__ part, const int *__restrict__ cptr,
                                                 const double *__restrict__ bn, const double *__restrict__ rtol,
                                                 int hist_cap, double *__restrict__ hist, double *__restrict__ last,
                                                 int *__restrict__ active, int *__restrict__ status,
                                                 int *__restrict__ iters, int *__restrict__ it,
                                                 int *__restrict__ nact, int *__restrict__ nact_acc, int tick) {
    const int sys = blockIdx.x;
    if (active[sys]) {   // uniform over the wave
        const double ss = seg_total(part, cptr, sys);
        if (threadIdx.x == 0) {
            const int k = *it;
            const double rel = sqrt(ss) / bn[sys];
            if (k < hist_cap) hist[static_cast<int64_t>(sys) * hist_cap + k] = rel;
            last[sys] = rel;
            iters[sys] = k + 1;
            if (!isfinite(rel)) {
                active[sys] = 0;
                status[sys] = kStNumeric;
            } else if (rel <= *rtol) {
                active[sys] = 0;
                status[sys] = kStOk;
            } else {
                atomicAdd(nact_acc, 1);
            }
        }
    }
    if (tick && threadIdx.x == 0) {
        *it = *it + 1;
        *nact = *nact_acc;
        *nact_acc = 0;
    }
}

// Counters after k_seg_init (reset: it = 0) or k_seg_check (it += 1): the
// number of systems still iterating, and a cleared accumulator.
__global__ void k_seg_tick(int reset, int *__restrict__ it, int *__restrict__ nact, int *__restrict__ nact_acc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *it = reset ? 0 : *it + 1;
    *nact = *nact_acc;
    *nact_acc = 0;
}

__global__ __launch_bounds__(256) void k_to_float(const double *__restrict__ in, float *__restrict__ out, int64_t n,
                                                 const int *__restrict__ count) {
    if (count && *count < n) n = *count;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[g] = static_cast<float>(in[g]);
}

// Lane groups per block row: the tuned count if the view carries one, else
// from the average row length; on a level too small to fill the chip with one
// group per row, up to four times the average row length: there each row's
// chain of dependent loads, not bandwidth, sets the time (at most 256 lanes
// per row either way).
template <typename MT>
int groups_for_len(const MatView<MT> &A, double avg) {
    int G;
    if (A.groups > 0) {
        G = A.groups;
    } else if (few_lanes(A.nb, A.bs)) {
        // enough groups for rows several times the average length (the longest
        // row sets the time), within what a row can take
        G = 1;
        while (G < max_groups(A.bs) && G < 4.0 * avg) G *= 2;
    } else {
        G = avg <= 3.5 ? 1 : (avg <= 7.0 ? 2 : (avg <= 14.0 ? 4 : 8));
    }
    while (G > 1 && G * A.bs > kThreads) G >>= 1;
    return G;
}
template <typename MT>
int groups_for(const MatView<MT> &A) {
    return groups_for_len(A, A.nb > 0 ? static_cast<double>(A.nnzb) / A.nb : 1.0);
}

unsigned grid_rows(int64_t rows, int G, int bs) { return grid_for(rows, kThreads / (G * bs)); }

// A launch must not read an operator the level does not hold.
template <typename MT>
void need(const MatView<MT> &A, const char *what) {
    // (a row-compressed copy stands in for the blocks)
    if (A.nb > 0 && (!A.rowptr || !A.colidx || (!A.vals && !A.rows.mask)))
        fail(NAIR_EDEVICE, std::string(what) + ": the level holds no such operator");
    if (A.face.meta && (!A.face.vals || !A.face.dvals || A.bs > 32))
        fail(NAIR_EDEVICE, std::string(what) + ": incomplete face-compressed copy");
}

}  // namespace

#define NAIR_BS_DISPATCH(bs, KERNEL, ...)                    \
    switch (bs) {                                            \
        case 2: KERNEL<2, MT, VT> __VA_ARGS__; break;        \
        case 3: KERNEL<3, MT, VT> __VA_ARGS__; break;        \
        case 4: KERNEL<4, MT, VT> __VA_ARGS__; break;        \
        case 6: KERNEL<6, MT, VT> __VA_ARGS__; break;        \
        case 9: KERNEL<9, MT, VT> __VA_ARGS__; break;        \
        case 10: KERNEL<10, MT, VT> __VA_ARGS__; break;      \
        case 16: KERNEL<16, MT, VT> __VA_ARGS__; break;      \
        case 25: KERNEL<25, MT, VT> __VA_ARGS__; break;      \
        default: KERNEL<0, MT, VT> __VA_ARGS__; break;       \
    }

// Instances with the last flag set (face-compressed or row-compressed blocks):
// the block sizes of Q1..Q4 elements, others at run time.
#define NAIR_FACE_DISPATCH(bs, KERNEL, ...)                    \
    switch (bs) {                                              \
        case 4: KERNEL<4, MT, VT, true> __VA_ARGS__; break;    \
        case 9: KERNEL<9, MT, VT, true> __VA_ARGS__; break;    \
        case 16: KERNEL<16, MT, VT, true> __VA_ARGS__; break;  \
        case 25: KERNEL<25, MT, VT, true> __VA_ARGS__; break;  \
        default: KERNEL<0, MT, VT, true> __VA_ARGS__; break;   \
    }

int max_groups(int bs) {
    int G = 1;
    while (2 * G * bs <= kThreads && G < 32) G *= 2;
    return G;
}

bool few_lanes(int64_t rows, int bs) { return rows * bs < kFewLanes; }

template <typename MT, typename VT>
void launch_residual(const MatView<MT> &A, const VT *b, const VT *x, VT *r, float *r_lo, hipStream_t s,
                     Gate gate) {
    need(A, "launch_residual");
    const int G = groups_for(A);
    const unsigned grid = grid_rows(A.nb, G, A.bs);
    if (A.face.meta)
        NAIR_FACE_DISPATCH(A.bs, k_residual, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, A.nb, A.bs, G, b,
                                                                        x, r, r_lo, gate, A.face))
    else
        NAIR_BS_DISPATCH(A.bs, k_residual, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, A.nb, A.bs, G, b, x,
                                                                      r, r_lo, gate, A.face))
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_relax(const MatView<MT> &A, const double *dinv, bool dinv_trans, const VT *r, const VT *ein, VT *eout,
                  const int *list, int nlist, const int8_t *cf, int only_cf, hipStream_t s, Gate gate) {
    need(A, "launch_relax");
    const int N = list ? nlist : A.nb;
    if (N <= 0) return;
    const int G = groups_for(A);
    const unsigned grid = grid_rows(N, G, A.bs);
    if (list && A.sweep.rowptr) {   // F sweep from the level's sweep copy (built for this F list)
        const SweepView<MT> &S = A.sweep;
        if ((S.meta ? !S.vals : (!S.rows.mask || !S.rows.off || !S.rows.vals)) || !S.dinv || A.bs > 32)
            fail(NAIR_EDEVICE, "launch_relax: incomplete sweep copy");
        if (!S.meta && A.bs >= 8 && !few_lanes(nlist, A.bs)) {   // one lane per stored row
            const int R = std::max(1, 2 * kThreads / (G * A.bs));
            const unsigned grid_cr = grid_for(nlist, R);
            switch (A.bs) {
                case 9: k_sweep_cr<9, MT, VT><<<grid_cr, kThreads, 0, s>>>(S, list, nlist, A.bs, R, r, ein, eout, gate); break;
                case 16: k_sweep_cr<16, MT, VT><<<grid_cr, kThreads, 0, s>>>(S, list, nlist, A.bs, R, r, ein, eout, gate); break;
                case 25: k_sweep_cr<25, MT, VT><<<grid_cr, kThreads, 0, s>>>(S, list, nlist, A.bs, R, r, ein, eout, gate); break;
                default: k_sweep_cr<0, MT, VT><<<grid_cr, kThreads, 0, s>>>(S, list, nlist, A.bs, R, r, ein, eout, gate); break;
            }
            NAIR_HIP(hipGetLastError());
            return;
        }
        if (dinv_trans && S.meta) {
            NAIR_FACE_DISPATCH(A.bs, k_sweep_T, <<<grid, kThreads, 0, s>>>(S, list, nlist, A.bs, G, r, ein, eout,
                                                                           gate));
        } else if (dinv_trans) {
            NAIR_BS_DISPATCH(A.bs, k_sweep_T, <<<grid, kThreads, 0, s>>>(S, list, nlist, A.bs, G, r, ein, eout,
                                                                         gate));
        } else if (S.meta) {
            NAIR_FACE_DISPATCH(A.bs, k_sweep, <<<grid, kThreads, 0, s>>>(S, list, nlist, A.bs, G, r, ein, eout,
                                                                         gate));
        } else {
            NAIR_BS_DISPATCH(A.bs, k_sweep, <<<grid, kThreads, 0, s>>>(S, list, nlist, A.bs, G, r, ein, eout, gate));
        }
        NAIR_HIP(hipGetLastError());
        return;
    }
    if (dinv_trans && A.face.meta) {
        NAIR_FACE_DISPATCH(A.bs, k_relax_T, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, dinv, A.nb, A.bs,
                                                                       G, r, ein, eout, list, nlist, cf, only_cf,
                                                                       gate, A.face));
    } else if (dinv_trans) {
        NAIR_BS_DISPATCH(A.bs, k_relax_T, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, dinv, A.nb, A.bs, G,
                                                                     r, ein, eout, list, nlist, cf, only_cf, gate,
                                                                     A.face));
    } else if (A.face.meta) {
        NAIR_FACE_DISPATCH(A.bs, k_relax, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, dinv, A.nb, A.bs, G,
                                                                     r, ein, eout, list, nlist, cf, only_cf, gate,
                                                                     A.face));
    } else {
        NAIR_BS_DISPATCH(A.bs, k_relax, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, dinv, A.nb, A.bs, G,
                                                                   r, ein, eout, list, nlist, cf, only_cf, gate,
                                                                   A.face));
    }
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_relax_T_first(const double *dinv, const VT *r, const int8_t *cf, VT *e0, VT *e1, int nb, int bs,
                          hipStream_t s, Gate gate) {
    if (nb <= 0) return;
    k_relax_T_first<VT><<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(dinv, r, cf, e0, e1,
                                                                                                 nb, bs, gate);
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_restrict(const MatView<MT> &Z, const VT *r, const int *cpts, VT *rc, hipStream_t s, Gate gate) {
    need(Z, "launch_restrict");
    if (Z.nb <= 0) return;
    const int G = groups_for(Z);
    if (Z.bs >= 8 && !few_lanes(Z.nb, Z.bs)) {
        // one lane per stored row; the lane-group count sets the coarse rows per workgroup
        const int R = std::max(1, 2 * kThreads / (G * Z.bs));
        const unsigned grid = grid_for(Z.nb, R);
        const bool rb = Z.rows.mask != nullptr;
        if (rb && (!Z.rows.off || !Z.rows.vals || Z.bs > 32)) fail(NAIR_EDEVICE, "launch_restrict: incomplete row copy of Z");
#define NAIR_CR(BS)                                                                                                 \
    do {                                                                                                            \
        if (rb)                                                                                                     \
            k_restrict_cr<BS, MT, VT, true><<<grid, kThreads, 0, s>>>(Z.rowptr, Z.colidx, Z.vals, Z.nb, Z.bs, R, r,  \
                                                                      cpts, rc, gate, Z.rows);                      \
        else                                                                                                        \
            k_restrict_cr<BS, MT, VT, false><<<grid, kThreads, 0, s>>>(Z.rowptr, Z.colidx, Z.vals, Z.nb, Z.bs, R, r, \
                                                                       cpts, rc, gate, Z.rows);                     \
    } while (0)
        switch (Z.bs) {
            case 9: NAIR_CR(9); break;
            case 16: NAIR_CR(16); break;
            case 25: NAIR_CR(25); break;
            default: NAIR_CR(0); break;
        }
#undef NAIR_CR
        NAIR_HIP(hipGetLastError());
        return;
    }
    const unsigned grid = grid_rows(Z.nb, G, Z.bs);
    if (Z.rows.mask) {
        if (!Z.rows.off || !Z.rows.vals || Z.bs > 32) fail(NAIR_EDEVICE, "launch_restrict: incomplete row copy of Z");
        NAIR_FACE_DISPATCH(Z.bs, k_restrict, <<<grid, kThreads, 0, s>>>(Z.rowptr, Z.colidx, Z.vals, Z.nb, Z.bs, G, r,
                                                                        cpts, rc, gate, Z.rows));
    } else {
        NAIR_BS_DISPATCH(Z.bs, k_restrict, <<<grid, kThreads, 0, s>>>(Z.rowptr, Z.colidx, Z.vals, Z.nb, Z.bs, G, r,
                                                                      cpts, rc, gate, Z.rows));
    }
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_interp(const int *pmap, const VT *ec, VT *e0, VT *e1, int nb, int bs, hipStream_t s, Gate gate) {
    k_interp<VT><<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(pmap, ec, e0, e1, nb, bs,
                                                                                         gate);
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_relax_interp(const MatView<MT> &A, const double *dinv, const VT *r, const int *pmap, const VT *ec,
                         const int8_t *cf, VT *e0, VT *e1, hipStream_t s, Gate gate) {
    need(A, "launch_relax_interp");
    if (A.nb <= 0) return;
    const int G = groups_for(A);
    const unsigned grid = grid_rows(A.nb, G, A.bs);
    NAIR_BS_DISPATCH(A.bs, k_relax_interp, <<<grid, kThreads, 0, s>>>(A.rowptr, A.colidx, A.vals, dinv, A.nb, A.bs,
                                                                      G, r, pmap, ec, cf, e0, e1, gate));
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_restrict_T(const int *ptptr, const int *ptidx, const VT *sv, VT *sc, int nc, int bs, hipStream_t st,
                       Gate gate) {
    if (nc <= 0) return;
    k_restrict_T<VT><<<grid_for(static_cast<int64_t>(nc) * bs, kThreads), kThreads, 0, st>>>(ptptr, ptidx, sv, sc,
                                                                                              nc, bs, gate);
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_interp_T(const MatView<MT> &ZT, const int *cidx, const VT *yc, VT *y, hipStream_t s, Gate gate) {
    need(ZT, "launch_interp_T");
    const int G = groups_for(ZT);
    const unsigned grid = grid_rows(ZT.nb, G, ZT.bs);
    NAIR_BS_DISPATCH(ZT.bs, k_interp_T, <<<grid, kThreads, 0, s>>>(ZT.rowptr, ZT.colidx, ZT.vals, ZT.nb, ZT.bs, G,
                                                                   cidx, yc, y, gate));
    NAIR_HIP(hipGetLastError());
}

// Lane groups of a TransRows product: the tuned count, else as groups_for.
template <typename MT>
int groups_for_tr(const TransRowsView<MT> &T) {
    MatView<MT> v;
    v.nb = T.nrows;
    v.bs = T.bs;
    v.groups = T.groups;
    // (a stored row costs about a fifth of a whole block row's lane work)
    return groups_for_len(v, T.nrows > 0 ? static_cast<double>(T.nq) / (5.0 * T.nrows) : 1.0);
}

template <typename MT>
void need_tr(const TransRowsView<MT> &T, const char *what) {
    if (T.nrows > 0 && (!T.rowptr || !T.qptr || (T.nent > 0 && (!T.colidx || !T.mask || !T.off || !T.src || !T.vals))) ||
        T.bs > 32)
        fail(NAIR_EDEVICE, std::string(what) + ": incomplete transposed row copy");
}

template <typename MT, typename VT>
void launch_residual_tr(const TransRowsView<MT> &T, const VT *g, const VT *y, VT *sout, hipStream_t s, Gate gate) {
    need_tr(T, "launch_residual_tr");
    if (T.nrows <= 0) return;
    const int G = groups_for_tr(T);
    const unsigned grid = grid_rows(T.nrows, G, T.bs);
    NAIR_BS_DISPATCH(T.bs, k_residual_tr, <<<grid, kThreads, 0, s>>>(T, T.bs, G, g, y, sout, gate));
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_sweep_tr(const TransRowsView<MT> &T, const double *dinv, const VT *g, const VT *yin, VT *yout,
                     const int *list, int nlist, hipStream_t s, Gate gate) {
    need_tr(T, "launch_sweep_tr");
    if (nlist <= 0) return;
    const int G = groups_for_tr(T);
    const unsigned grid = grid_rows(nlist, G, T.bs);
    NAIR_BS_DISPATCH(T.bs, k_sweep_tr, <<<grid, kThreads, 0, s>>>(T, dinv, list, nlist, T.bs, G, g, yin, yout,
                                                                  gate));
    NAIR_HIP(hipGetLastError());
}

template <typename MT, typename VT>
void launch_interp_tr(const TransRowsView<MT> &T, const int *cidx, const VT *yc, VT *y, hipStream_t s, Gate gate) {
    need_tr(T, "launch_interp_tr");
    if (T.nrows <= 0) return;
    const int G = groups_for_tr(T);
    const unsigned grid = grid_rows(T.nrows, G, T.bs);
    NAIR_BS_DISPATCH(T.bs, k_interp_tr, <<<grid, kThreads, 0, s>>>(T, T.bs, G, cidx, yc, y, gate));
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_init_T(const double *dinv, const VT *g, const int8_t *cf, int fc, VT *y0, VT *y1, int nb, int bs,
                   hipStream_t s, Gate gate) {
    k_init_T<VT><<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(dinv, g, cf, fc, y0, y1, nb,
                                                                                         bs, gate);
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_axpy(double *x, const VT *e, int64_t n, hipStream_t s) {
    k_axpy<VT><<<grid_for(n, kThreads), kThreads, 0, s>>>(x, e, n);
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_dense_matvec(const double *M, const int64_t *off, const int *dof0, const int *n, int nseg, int max_n,
                         const VT *x, VT *y, hipStream_t s, const int *sys, const int *active) {
    if (nseg <= 0) return;
    k_dense_mv<VT><<<dim3(grid_for(max_n, 4), static_cast<unsigned>(nseg)), 256, 0, s>>>(M, off, dof0, n, x, y, sys,
                                                                                         active);
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_copy_vec(VT *dst, const VT *src, int nb, int bs, hipStream_t s, Gate gate) {
    if (nb <= 0) return;
    k_vec_copy<VT, false><<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(dst, src, nb, bs,
                                                                                                gate);
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_add_vec(VT *dst, const VT *src, int nb, int bs, hipStream_t s, Gate gate) {
    if (nb <= 0) return;
    k_vec_copy<VT, true><<<grid_for(static_cast<int64_t>(nb) * bs, kThreads), kThreads, 0, s>>>(dst, src, nb, bs,
                                                                                               gate);
    NAIR_HIP(hipGetLastError());
}

template <typename VT>
void launch_axpy_active(double *x, const VT *e, int64_t n, int bs, const int *bsys, const int *active,
                        hipStream_t s) {
    k_axpy_active<VT><<<grid_for(n, kThreads), kThreads, 0, s>>>(x, e, n, bs, bsys, active);
    NAIR_HIP(hipGetLastError());
}

void launch_seg_sumsq(const double *v, const int64_t *clo, const int *clen, int nchunk, double *part,
                      hipStream_t s) {
    if (nchunk <= 0) return;
    k_seg_sumsq<<<static_cast<unsigned>(nchunk), kThreads, 0, s>>>(v, clo, clen, part);
    NAIR_HIP(hipGetLastError());
}

void launch_seg_init(const double *part, const int *cptr, int nsys, double *bn, double *last, int *active,
                     int *status, int *iters, int *it, int *nact, int *nact_acc, hipStream_t s) {
    k_seg_tick<<<1, 64, 0, s>>>(1, it, nact, nact_acc);   // clears the accumulator
    k_seg_init<<<static_cast<unsigned>(nsys), 64, 0, s>>>(part, cptr, bn, last, active, status, iters, nact_acc);
    k_seg_tick<<<1, 64, 0, s>>>(1, it, nact, nact_acc);
    NAIR_HIP(hipGetLastError());
}

void launch_seg_check(const double *part, const int *cptr, int nsys, const double *bn, const double *rtol,
                      int hist_cap, double *hist, double *last, int *active, int *status, int *iters, int *it,
                      int *nact, int *nact_acc, hipStream_t s) {
    const int fused = nsys == 1 ? 1 : 0;
    k_seg_check<<<static_cast<unsigned>(nsys), 64, 0, s>>>(part, cptr, bn, rtol, hist_cap, hist, last, active, status,
                                                           iters, it, nact, nact_acc, fused);
    if (!fused) k_seg_tick<<<1, 64, 0, s>>>(0, it, nact, nact_acc);
    NAIR_HIP(hipGetLastError());
}

void launch_to_float(const double *in, float *out, int64_t n, hipStream_t s, const int *count) {
    if (n <= 0) return;
    const int64_t g = (n + 255) / 256;
    k_to_float<<<static_cast<unsigned>(g > 1048576 ? 1048576 : g), 256, 0, s>>>(in, out, n, count);
    NAIR_HIP(hipGetLastError());
}

// instantiations: the FP64 cycle and the FP32-stored cycle
#define NAIR_CYCLE_INST(MT, VT)                                                                                      \
    template void launch_residual<MT, VT>(const MatView<MT> &, const VT *, const VT *, VT *, float *, hipStream_t,  \
                                          Gate);                                                                     \
    template void launch_relax<MT, VT>(const MatView<MT> &, const double *, bool, const VT *, const VT *, VT *,      \
                                       const int *, int, const int8_t *, int, hipStream_t, Gate);                    \
    template void launch_restrict<MT, VT>(const MatView<MT> &, const VT *, const int *, VT *, hipStream_t, Gate);    \
    template void launch_interp<VT>(const int *, const VT *, VT *, VT *, int, int, hipStream_t, Gate);               \
    template void launch_relax_interp<MT, VT>(const MatView<MT> &, const double *, const VT *, const int *,          \
                                              const VT *, const int8_t *, VT *, VT *, hipStream_t, Gate);            \
    template void launch_relax_T_first<VT>(const double *, const VT *, const int8_t *, VT *, VT *, int, int,         \
                                           hipStream_t, Gate);                                                       \
    template void launch_restrict_T<VT>(const int *, const int *, const VT *, VT *, int, int, hipStream_t, Gate);    \
    template void launch_interp_T<MT, VT>(const MatView<MT> &, const int *, const VT *, VT *, hipStream_t, Gate);    \
    template void launch_residual_tr<MT, VT>(const TransRowsView<MT> &, const VT *, const VT *, VT *, hipStream_t,  \
                                             Gate);                                                                  \
    template void launch_sweep_tr<MT, VT>(const TransRowsView<MT> &, const double *, const VT *, const VT *, VT *,  \
                                          const int *, int, hipStream_t, Gate);                                      \
    template void launch_interp_tr<MT, VT>(const TransRowsView<MT> &, const int *, const VT *, VT *, hipStream_t,    \
                                           Gate);                                                                    \
    template void launch_init_T<VT>(const double *, const VT *, const int8_t *, int, VT *, VT *, int, int,           \
                                    hipStream_t, Gate);                                                              \
    template void launch_axpy<VT>(double *, const VT *, int64_t, hipStream_t);                                       \
    template void launch_axpy_active<VT>(double *, const VT *, int64_t, int, const int *, const int *, hipStream_t); \
    template void launch_copy_vec<VT>(VT *, const VT *, int, int, hipStream_t, Gate);                                \
    template void launch_add_vec<VT>(VT *, const VT *, int, int, hipStream_t, Gate);                                 \
    template void launch_dense_matvec<VT>(const double *, const int64_t *, const int *, const int *, int, int,       \
                                          const VT *, VT *, hipStream_t, const int *, const int *);

NAIR_CYCLE_INST(double, double)
NAIR_CYCLE_INST(float, float)

}  // namespace nair
