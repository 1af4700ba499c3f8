// Dense bs x bs block products on the FP64 matrix cores (bs <= 32), shared by
// the setup's sparse products and single block products.
//
// One wave holds one output block in NT x NT tiles of 16 x 16 (NT = ceil(bs/16)):
// entry (16 ti + i, 16 tj + j) of the block sits in accumulator acc[ti][tj], lane
// j + 16 (i % 4), register i / 4.  A product X Y adds ceil(bs/4) 16x16x4 steps per
// tile; step q takes inner indices c = 4q .. 4q+3, lane (row, kk) supplying
// X(16 ti + row, 4q + kk) and Y(4q + kk, 16 tj + row), zero outside the block.
// A 16x16x4 FP64 step updates each entry as the fma chain over its four inner
// indices in ascending order, so an entry's value is the fma chain over c
// ascending from the accumulator's start, the same as a scalar loop; padding
// adds fma(0, 0, acc) = acc (an accumulator that is -0 becomes +0: the only
// difference a zero-padded step can make, and only in the sign of a zero).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nair {

typedef double double4_t __attribute__((ext_vector_type(4)));

template <int BS>
struct MfmaShape {
    static_assert(BS >= 1 && BS <= 32, "matrix-core block products take bs <= 32");
    static constexpr int NT = (BS + 15) / 16;   // tiles per dimension
    static constexpr int KQ = (BS + 3) / 4;     // 16x16x4 steps per tile
};

template <int BS>
struct MfmaAcc {
    static constexpr int NT = MfmaShape<BS>::NT;
    double4_t t[NT][NT];
    __device__ void zero() {
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) t[ti][tj] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
    // acc += o, entry by entry (plain adds)
    __device__ void add(const MfmaAcc &o) {
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                for (int r = 0; r < 4; ++r) t[ti][tj][r] = t[ti][tj][r] + o.t[ti][tj][r];
    }
};

// One block pair's operands as the steps take them.  For an identity pair
// (X = I, x == nullptr) the lane keeps Y's entries at its accumulator positions
// instead, to be added plainly: position (ti, tj, r) in (tj == 0 ? a : b)[ti][r].
template <int BS>
struct MfmaOperands {
    static constexpr int NT = MfmaShape<BS>::NT;
    static constexpr int KQ = MfmaShape<BS>::KQ;
    static_assert(NT == 1 || KQ >= 4, "identity entries are kept in the operand registers");
    double a[NT][KQ], b[NT][KQ];
    bool ident;

    // X Y, X given (no identity pair)
    __device__ void load_product(const double *__restrict__ x, const double *__restrict__ y, int row, int kk) {
        ident = false;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const int c = 4 * q + kk;
                const int i = 16 * t + row;   // X's row of tile row t, Y's column of tile column t
                a[t][q] = (i < BS && c < BS) ? x[i * BS + c] : 0.0;
                b[t][q] = (i < BS && c < BS) ? y[c * BS + i] : 0.0;
            }
    }

    // the steps of a product loaded by load_product
    __device__ void apply_product(MfmaAcc<BS> &acc) const {
#pragma unroll
        for (int q = 0; q < KQ; ++q)
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
                    acc.t[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti][q], b[tj][q], acc.t[ti][tj], 0, 0, 0);
    }

    __device__ void load(const double *__restrict__ x, const double *__restrict__ y, int row, int kk) {
        ident = x == nullptr;
        if (ident) {
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int r = 0; r < KQ; ++r) {
                    const int i = 16 * ti + kk + 4 * r;
                    const int j0 = row, j1 = 16 + row;
                    a[ti][r] = (r < 4 && i < BS && j0 < BS) ? y[i * BS + j0] : 0.0;
                    b[ti][r] = (NT > 1 && r < 4 && i < BS && j1 < BS) ? y[i * BS + j1] : 0.0;
                }
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int q = 0; q < KQ; ++q) {
                    const int c = 4 * q + kk;
                    const int i = 16 * t + row;   // X's row of tile row t, Y's column of tile column t
                    a[t][q] = (i < BS && c < BS) ? x[i * BS + c] : 0.0;
                    b[t][q] = (i < BS && c < BS) ? y[c * BS + i] : 0.0;
                }
        }
    }

    __device__ void apply(MfmaAcc<BS> &acc, int row, int kk) const {
        if (ident) {
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * ti + kk + 4 * r, j = 16 * tj + row;
                        if (r < KQ && i < BS && j < BS)
                            acc.t[ti][tj][r] = acc.t[ti][tj][r] + (tj == 0 ? a[ti][r < KQ ? r : 0]
                                                                           : b[ti][r < KQ ? r : 0]);
                    }
        } else {
#pragma unroll
            for (int q = 0; q < KQ; ++q)
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
                        acc.t[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti][q], b[tj][q], acc.t[ti][tj], 0, 0, 0);
        }
    }
};

// Visit this lane's entries (i, j, value) of an accumulated block.
template <int BS, typename F>
__device__ inline void mfma_for_entries(const MfmaAcc<BS> &acc, int row, int kk, F &&f) {
    constexpr int NT = MfmaShape<BS>::NT;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * ti + kk + 4 * r, j = 16 * tj + row;
                if (i < BS && j < BS) f(i, j, acc.t[ti][tj][r]);
            }
}

}  // namespace nair
