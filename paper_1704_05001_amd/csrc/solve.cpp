// Solve phase: the V-cycle and its transpose, and the stationary iteration.
#include <algorithm>
#include <cmath>
#include <utility>

#include "hier.h"

namespace nair {
namespace {

double read_double(const double *d, hipStream_t s) {
    double v = 0.0;
    NAIR_HIP(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, s));
    NAIR_HIP(hipStreamSynchronize(s));
    return v;
}

// V-cycle on level l with right-hand side lv[l]->r and zero initial guess, no
// pre-relaxation (section 5): restrict, recurse, interpolate, nu = k+1 Jacobi
// F sweeps (section 5.1), optionally one C sweep.  Returns the correction.
const double *vcycle(Hier &h, int l, hipStream_t s) {
    Level &L = *h.lv[l];
    const int bs = h.bs;
    if (L.coarsest) {
        TimerScope ts(TK_DENSE, l, s);
        launch_dense_matvec(L.dense_inv.get(), L.r.get(), L.e0.get(), L.dense_n, s);
        return L.e0.get();
    }
    Level &C = *h.lv[l + 1];
    {
        TimerScope ts(TK_RESTRICT, l, s);
        launch_restrict(L.Z, L.r.get(), L.cpts.get(), C.r.get(), s);
    }
    const double *ec = vcycle(h, l + 1, s);
    {
        TimerScope ts(TK_INTERP, l, s);
        launch_interp(L.pmap.get(), ec, L.e0.get(), L.e1.get(), L.A.nb, bs, s);
    }
    double *cur = L.e0.get(), *oth = L.e1.get();
    {
        // the nu sweeps run back to back; the timer brackets them as one group
        TimerScope ts(TK_RELAX, l, s, h.prm.degree + 1);
        for (int k = 0; k <= h.prm.degree; ++k) {
            launch_relax(L.A, L.dinv.get(), false, L.r.get(), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s);
            std::swap(cur, oth);
        }
    }
    if (h.prm.relax == 1) {
        launch_relax(L.A, L.dinv.get(), false, L.r.get(), cur, oth, nullptr, 0, L.cf.get(), 1, s);
        std::swap(cur, oth);
    }
    return cur;
}

// The transposed cycle: optional C sweep with D^-T first, nu transposed Jacobi
// F sweeps (pre-relaxation), s = g - A^T y, restrict by P^T, recurse, and
// y += R^T y_c = [Z^T y_c ; y_c].
const double *vcycle_T(Hier &h, int l, hipStream_t s) {
    Level &L = *h.lv[l];
    const int bs = h.bs;
    if (L.coarsest) {
        TimerScope ts(TK_DENSE, l, s);
        launch_dense_matvec(L.dense_invT.get(), L.r.get(), L.e0.get(), L.dense_n, s);
        return L.e0.get();
    }
    Level &C = *h.lv[l + 1];
    launch_init_T(L.dinv.get(), L.r.get(), L.cf.get(), h.prm.relax == 1 ? 1 : 0, L.e0.get(), L.e1.get(), L.A.nb, bs,
                  s);
    double *cur = L.e0.get(), *oth = L.e1.get();
    for (int k = 0; k <= h.prm.degree; ++k) {
        launch_relax(L.AT, L.dinv.get(), true, L.r.get(), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s);
        std::swap(cur, oth);
    }
    launch_residual(L.AT, L.r.get(), cur, L.tmp.get(), nullptr, 0, s);
    launch_restrict_T(L.ptptr.get(), L.ptidx.get(), L.tmp.get(), C.r.get(), L.nc, bs, s);
    const double *yc = vcycle_T(h, l + 1, s);
    launch_interp_T(L.ZT, L.cidx.get(), yc, cur, s);
    return cur;
}

void ensure_work(Hier &h) {
    const Level &L0 = *h.lv[0];
    const int np = std::max(residual_partials_count(L0.A),
                            sumsq_partials_count(static_cast<int64_t>(L0.A.nb) * h.bs));
    if (h.npart < np) {
        h.partials.alloc(np);
        h.npart = np;
    }
    if (!h.scal.get()) h.scal.alloc(2);
}

}  // namespace

nair_status run_solve(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                      hipStream_t s) {
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    if (trans) ensure_transposes(h, s);
    ensure_work(h);
    h.hist.clear();
    nair_result rr{0, 0, 0.0, 0.0, 0.0};
    NAIR_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    launch_sumsq(b, n, h.partials.get(), h.npart, s);
    launch_reduce_partials(h.partials.get(), sumsq_partials_count(n), h.scal.get(), s);
    const double bn = std::sqrt(read_double(h.scal.get(), s));
    nair_status st = NAIR_ENOCONV;
    if (!std::isfinite(bn)) {
        st = NAIR_ENUMERIC;
    } else if (bn == 0.0) {
        rr.converged = 1;
        st = NAIR_OK;
    } else {
        NAIR_HIP(hipMemcpyAsync(L0.r.get(), b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        const DevBSR &Aop = trans ? L0.AT : L0.A;
        double rel = 1.0;
        for (int it = 0; it < max_iter; ++it) {
            const double *e = trans ? vcycle_T(h, 0, s) : vcycle(h, 0, s);
            launch_axpy(x, e, n, s);
            {
                TimerScope ts(TK_RESIDUAL, 0, s);
                launch_residual(Aop, b, x, L0.r.get(), h.partials.get(), h.npart, s);
            }
            launch_reduce_partials(h.partials.get(), residual_partials_count(L0.A), h.scal.get(), s);
            rel = std::sqrt(read_double(h.scal.get(), s)) / bn;
            h.hist.push_back(rel);
            if (!std::isfinite(rel)) {
                st = NAIR_ENUMERIC;
                break;
            }
            if (rel <= rtol) {
                st = NAIR_OK;
                rr.converged = 1;
                break;
            }
        }
        rr.relres = rel;
    }
    rr.iters = static_cast<int32_t>(h.hist.size());
    if (rr.iters > 0) {
        const double hK = h.hist.back();
        rr.rho_avg = std::pow(hK, 1.0 / rr.iters);
        rr.rho_last5 = rr.iters > 5 ? std::pow(hK / h.hist[rr.iters - 6], 0.2) : rr.rho_avg;
    }
    if (res) *res = rr;
    NAIR_HIP(hipStreamSynchronize(s));
    return st;
}

void run_vcycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s) {
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    if (trans) ensure_transposes(h, s);
    NAIR_HIP(hipMemcpyAsync(L0.r.get(), r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    const double *out = trans ? vcycle_T(h, 0, s) : vcycle(h, 0, s);
    NAIR_HIP(hipMemcpyAsync(e, out, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    NAIR_HIP(hipStreamSynchronize(s));
}

}  // namespace nair
