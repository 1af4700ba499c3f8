// Gradient of a linear solve with respect to the matrix entries on its block
// pattern: for x = A^{-1} b and ybar = A^{-T} xbar, dL/dA_IJ = -ybar_I x_J^T.
#include "common.h"

namespace nair {
namespace {

__global__ __launch_bounds__(256) void k_grad_vals(const int *__restrict__ rowid, const int *__restrict__ colidx,
                                                  int64_t nnzb, int bs, const double *__restrict__ ybar,
                                                  const double *__restrict__ x, double *__restrict__ gvals) {
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    const int64_t total = nnzb * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t t = g / bb;
        const int e = static_cast<int>(g - t * bb);
        const int a = e / bs, b = e - a * bs;
        gvals[g] = -ybar[static_cast<int64_t>(rowid[t]) * bs + a] * x[static_cast<int64_t>(colidx[t]) * bs + b];
    }
}

}  // namespace

void grad_vals(int nb, int bs, const int *rowptr, const int *colidx, const double *ybar, const double *x,
               double *gvals, hipStream_t s) {
    const int nnzb = read_int(rowptr + nb, s);
    if (nnzb <= 0) return;
    DBuf<int> rowid(nnzb);
    launch_rows_of(rowptr, nb, rowid.get(), s);
    const int64_t total = static_cast<int64_t>(nnzb) * bs * bs;
    const int64_t g = (total + 255) / 256;
    k_grad_vals<<<static_cast<unsigned>(g > 1048576 ? 1048576 : g), 256, 0, s>>>(rowid.get(), colidx, nnzb, bs, ybar,
                                                                                 x, gvals);
    NAIR_HIP(hipGetLastError());
    NAIR_HIP(hipStreamSynchronize(s));
}

}  // namespace nair
