// Hierarchy data held by a nair_hier handle (internal).
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace nair {

struct Level {
    DevBSR A;                       // level operator (A_0 = copy of the input, then K = R A P)
    bool coarsest = false;
    // setup products
    DBuf<double> dinv, bnorm;
    DBuf<uint8_t> mask;
    DBuf<int> lambda, cidx, pmap, dround, cpts, flist;
    DBuf<int8_t> cf;
    int nc = 0, nF = 0, rounds = 0;
    DevBSR Z;                       // R = [Z I]: nc rows, fine F columns
    // coarsest level
    int dense_n = 0;
    DBuf<double> dense_inv, dense_invT;
    // transposed cycle (built on first use)
    bool have_T = false;
    DevBSR AT, ZT;
    DBuf<int> ptptr, ptidx;
    // cycle vectors
    DBuf<double> r, e0, e1, tmp;
    // FP32-stored hierarchy (precision 1): operator, Z and transposes in float,
    // and the cycle vectors
    DBuf<float> vals32, z32, at32, zt32;
    DBuf<float> r32, e0_32, e1_32, tmp32;
};

struct Hier {
    nair_params prm{};
    int bs = 0;
    int device = 0;
    std::vector<std::unique_ptr<Level>> lv;
    std::vector<double> hist;
    std::string err;
    DBuf<double> partials, scal;
    int npart = 0;
};

void build_hierarchy(Hier &h, int nb, int bs, const int *rowptr, const int *colidx, const double *vals,
                     hipStream_t s);
nair_status run_solve(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter,
                      nair_result *res, hipStream_t s);
void run_vcycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s);
void ensure_transposes(Hier &h, hipStream_t s);
void make_fp32_copies(Hier &h, hipStream_t s);
void complexity(Hier &h, double *oc, double *cc, hipStream_t s);

// validation of the input pattern (device): sets *bad != 0 on error
void launch_validate(const int *rowptr, const int *colidx, int nb, int64_t nnzb, int *bad, hipStream_t s);

}  // namespace nair
