// Solve phase: the V-cycle and its transpose, and the stationary iteration.
//
// precision 0: everything in FP64.  precision 1: the cycle reads FP32 copies of
// the level operators and Z and keeps its vectors in FP32 (accumulating in
// FP64, applying the FP64 block inverses); the outer residual b - A x and the
// update x += e stay FP64, so the iteration is FP64 iterative refinement with
// an FP32-stored hierarchy.
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

// Per-precision access to a level's matrices and cycle vectors.
template <typename T>
struct Store;

template <>
struct Store<double> {
    static MatView<double> A(const Level &L) { return view(L.A); }
    static MatView<double> Z(const Level &L) { return view(L.Z); }
    static MatView<double> AT(const Level &L) { return view(L.AT); }
    static MatView<double> ZT(const Level &L) { return view(L.ZT); }
    static double *r(Level &L) { return L.r.get(); }
    static double *e0(Level &L) { return L.e0.get(); }
    static double *e1(Level &L) { return L.e1.get(); }
    static double *tmp(Level &L) { return L.tmp.get(); }
};

template <>
struct Store<float> {
    static MatView<float> A(const Level &L) { return view(L.A, L.vals32.get()); }
    static MatView<float> Z(const Level &L) { return view(L.Z, L.z32.get()); }
    static MatView<float> AT(const Level &L) { return view(L.AT, L.at32.get()); }
    static MatView<float> ZT(const Level &L) { return view(L.ZT, L.zt32.get()); }
    static float *r(Level &L) { return L.r32.get(); }
    static float *e0(Level &L) { return L.e0_32.get(); }
    static float *e1(Level &L) { return L.e1_32.get(); }
    static float *tmp(Level &L) { return L.tmp32.get(); }
};

// V-cycle on level l with right-hand side r_l and zero initial guess, no
// pre-relaxation (section 5): restrict, recurse, interpolate, nu = k+1 Jacobi
// F sweeps (section 5.1), optionally one C sweep.  Returns the correction.
template <typename T>
const T *vcycle(Hier &h, int l, hipStream_t s) {
    using S = Store<T>;
    Level &L = *h.lv[l];
    const int bs = h.bs;
    if (L.coarsest) {
        TimerScope ts(TK_DENSE, l, s);
        launch_dense_matvec<T>(L.dense_inv.get(), S::r(L), S::e0(L), L.dense_n, s);
        return S::e0(L);
    }
    Level &C = *h.lv[l + 1];
    {
        TimerScope ts(TK_RESTRICT, l, s);
        launch_restrict<T, T>(S::Z(L), S::r(L), L.cpts.get(), S::r(C), s);
    }
    const T *ec = vcycle<T>(h, l + 1, s);
    {
        TimerScope ts(TK_INTERP, l, s);
        launch_interp<T>(L.pmap.get(), ec, S::e0(L), S::e1(L), L.A.nb, bs, s);
    }
    T *cur = S::e0(L), *oth = S::e1(L);
    const MatView<T> A = S::A(L);
    {
        // the nu sweeps run back to back; the timer brackets them as one group
        TimerScope ts(TK_RELAX, l, s, h.prm.degree + 1);
        for (int k = 0; k <= h.prm.degree; ++k) {
            launch_relax<T, T>(A, L.dinv.get(), false, S::r(L), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s);
            std::swap(cur, oth);
        }
    }
    if (h.prm.relax == 1) {
        launch_relax<T, T>(A, L.dinv.get(), false, S::r(L), cur, oth, nullptr, 0, L.cf.get(), 1, s);
        std::swap(cur, oth);
    }
    return cur;
}

// The transposed cycle: optional C sweep with D^-T first, nu transposed Jacobi
// F sweeps (pre-relaxation), s = g - A^T y, restrict by P^T, recurse, and
// y += R^T y_c = [Z^T y_c ; y_c].
template <typename T>
const T *vcycle_T(Hier &h, int l, hipStream_t s) {
    using S = Store<T>;
    Level &L = *h.lv[l];
    const int bs = h.bs;
    if (L.coarsest) {
        TimerScope ts(TK_DENSE, l, s);
        launch_dense_matvec<T>(L.dense_invT.get(), S::r(L), S::e0(L), L.dense_n, s);
        return S::e0(L);
    }
    Level &C = *h.lv[l + 1];
    launch_init_T<T>(L.dinv.get(), S::r(L), L.cf.get(), h.prm.relax == 1 ? 1 : 0, S::e0(L), S::e1(L), L.A.nb, bs, s);
    T *cur = S::e0(L), *oth = S::e1(L);
    const MatView<T> AT = S::AT(L);
    {
        TimerScope ts(TK_RELAX, l, s, h.prm.degree + 1);
        for (int k = 0; k <= h.prm.degree; ++k) {
            launch_relax<T, T>(AT, L.dinv.get(), true, S::r(L), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s);
            std::swap(cur, oth);
        }
    }
    launch_residual<T, T>(AT, S::r(L), cur, S::tmp(L), nullptr, nullptr, s);
    launch_restrict_T<T>(L.ptptr.get(), L.ptidx.get(), S::tmp(L), S::r(C), L.nc, bs, s);
    const T *yc = vcycle_T<T>(h, l + 1, s);
    launch_interp_T<T, T>(S::ZT(L), L.cidx.get(), yc, cur, s);
    return cur;
}

void ensure_work(Hier &h) {
    const Level &L0 = *h.lv[0];
    const int np = std::max(residual_partials_count(view(L0.A)),
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
    const bool fp32 = h.prm.precision == 1;
    if (trans) ensure_transposes(h, s);
    ensure_work(h);
    h.hist.clear();
    nair_result rr{0, 0, 0.0, 0.0, 0.0};
    NAIR_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    launch_sumsq(b, n, h.partials.get(), s);
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
        if (fp32) launch_to_float(b, L0.r32.get(), n, s);
        const MatView<double> Aop = trans ? view(L0.AT) : view(L0.A);
        double rel = 1.0;
        for (int it = 0; it < max_iter; ++it) {
            if (fp32) {
                const float *e = trans ? vcycle_T<float>(h, 0, s) : vcycle<float>(h, 0, s);
                launch_axpy<float>(x, e, n, s);
            } else {
                const double *e = trans ? vcycle_T<double>(h, 0, s) : vcycle<double>(h, 0, s);
                launch_axpy<double>(x, e, n, s);
            }
            {
                TimerScope ts(TK_RESIDUAL, 0, s);
                launch_residual<double, double>(Aop, b, x, L0.r.get(), h.partials.get(),
                                                fp32 ? L0.r32.get() : nullptr, s);
            }
            launch_reduce_partials(h.partials.get(), residual_partials_count(Aop), h.scal.get(), s);
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
    if (h.prm.precision == 1) {
        launch_to_float(r, L0.r32.get(), n, s);
        const float *out = trans ? vcycle_T<float>(h, 0, s) : vcycle<float>(h, 0, s);
        NAIR_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, s));
        launch_axpy<float>(e, out, n, s);
    } else {
        const double *out = trans ? vcycle_T<double>(h, 0, s) : vcycle<double>(h, 0, s);
        NAIR_HIP(hipMemcpyAsync(e, out, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    NAIR_HIP(hipStreamSynchronize(s));
}

}  // namespace nair
