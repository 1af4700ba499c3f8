// Restarted GMRES(m) right-preconditioned by the nAIR cycle (the section
// "Non-triangular matrices" uses one nAIR V-cycle per GMRES iteration).
//
// Per iteration: z_j = B v_j (one cycle), w = A z_j, two passes of classical
// Gram-Schmidt against v_0..v_j (each one multi-dot and one multi-axpy over
// the whole basis), ||w||, and one host read of the new Hessenberg column.
// The Givens rotations, the residual estimate and the small triangular solve
// run on the host; x += Z y at the end of each cycle, and a restart begins
// from the true residual b - A x.  The basis and the directions stay on the
// device: (2m + 2) vectors of n doubles.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hier.h"

namespace nair {
namespace {

void ensure_krylov(Hier &h, int m, int64_t n) {
    Krylov &K = h.krylov;
    if (K.m == m && K.n == n) return;
    K.m = m;
    K.n = n;
    K.V.alloc(static_cast<size_t>(m + 1) * n);
    K.Z.alloc(static_cast<size_t>(m) * n);
    K.w.alloc(static_cast<size_t>(n));
    K.part.alloc(static_cast<size_t>(mdot_parts(n)) * (m + 1));
    K.hd.alloc(static_cast<size_t>(2 * m + 3));
    K.c.alloc(static_cast<size_t>(m));
}

void read_doubles(const double *d, double *hst, int cnt, hipStream_t s) {
    read_device({{d, hst, sizeof(double) * static_cast<size_t>(cnt)}}, s);
}

}  // namespace

nair_status run_gmres(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                      hipStream_t s) {
    prepare_cycle(h, trans, s);
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    const int m = h.prm.gmres;
    ensure_krylov(h, m, n);
    Krylov &K = h.krylov;
    // A (or A^T) of the system being solved: the caller's blocks in the scalar form
    MatView<double> Aop;
    if (h.prm.form == 1) Aop = trans ? view(h.A0T) : view(h.A0);
    else Aop = op_view(L0, trans).with_groups(L0.tune[trans ? TU_RESIDUAL_T : TU_RESIDUAL]);

    double *V = K.V.get(), *Z = K.Z.get(), *w = K.w.get(), *hd = K.hd.get();
    auto vec = [n](double *base, int j) { return base + static_cast<int64_t>(j) * n; };
    const int H1 = 0, H2 = m + 1, SS = 2 * m + 2;   // device scalars: two coefficient passes, ||w||^2
    std::vector<double> hh(2 * m + 3), H(static_cast<size_t>(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m),
        cneg(m);
    auto Hm = [&](int i, int j) -> double & { return H[static_cast<size_t>(i) * m + j]; };

    NAIR_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    h.hist.clear();
    auto finish = [&](nair_status st, int it, double rel) {
        if (res) {
            nair_result rr{0, 0, 0.0, 0.0, 0.0};
            rr.iters = it;
            rr.converged = st == NAIR_OK ? 1 : 0;
            rr.relres = rel;
            if (it > 0) {
                rr.rho_avg = std::pow(rel, 1.0 / it);
                rr.rho_last5 = it > 5 ? std::pow(h.hist[it - 1] / h.hist[it - 6], 0.2) : rr.rho_avg;
            }
            *res = rr;
        }
        NAIR_HIP(hipStreamSynchronize(s));
        return st;
    };

    launch_mdot(b, 0, 1, b, n, K.part.get(), hd + SS, s);
    double ssb = 0.0;
    read_doubles(hd + SS, &ssb, 1, s);
    const double bn = std::sqrt(ssb);
    if (!std::isfinite(bn)) return finish(NAIR_ENUMERIC, 0, 0.0);
    if (bn == 0.0) return finish(NAIR_OK, 0, 0.0);

    NAIR_HIP(hipMemcpyAsync(w, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));   // r_0 = b (x_0 = 0)
    nair_status st = NAIR_ENOCONV;
    double rel = 1.0;
    int it = 0;
    while (it < max_iter) {
        launch_mdot(w, 0, 1, w, n, K.part.get(), hd + SS, s);
        double ss = 0.0;
        read_doubles(hd + SS, &ss, 1, s);
        const double beta = std::sqrt(ss);
        if (!std::isfinite(beta)) {
            st = NAIR_ENUMERIC;
            break;
        }
        launch_unit(w, hd + SS, vec(V, 0), n, s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        bool done = false;
        for (; j < m && it < max_iter; ++j) {
            apply_cycle(h, trans, vec(V, j), vec(Z, j), s);
            launch_residual<double, double>(Aop, nullptr, vec(Z, j), w, nullptr, s);   // w = A z_j
            launch_mdot(V, n, j + 1, w, n, K.part.get(), hd + H1, s);
            launch_maxpy(V, n, j + 1, hd + H1, w, n, s);
            launch_mdot(V, n, j + 1, w, n, K.part.get(), hd + H2, s);
            launch_maxpy(V, n, j + 1, hd + H2, w, n, s);
            launch_mdot(w, 0, 1, w, n, K.part.get(), hd + SS, s);
            read_doubles(hd, hh.data(), 2 * m + 3, s);
            for (int i = 0; i <= j; ++i) Hm(i, j) = hh[H1 + i] + hh[H2 + i];
            const double hn = std::sqrt(hh[SS]);
            Hm(j + 1, j) = hn;
            if (hn != 0.0) launch_unit(w, hd + SS, vec(V, j + 1), n, s);
            for (int i = 0; i < j; ++i) {   // earlier rotations
                const double a = Hm(i, j), c = Hm(i + 1, j);
                Hm(i, j) = cs[i] * a + sn[i] * c;
                Hm(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            const double a = Hm(j, j), c = Hm(j + 1, j);
            const double rho = std::sqrt(a * a + c * c);
            cs[j] = rho == 0.0 ? 1.0 : a / rho;
            sn[j] = rho == 0.0 ? 0.0 : c / rho;
            Hm(j, j) = rho;
            Hm(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            rel = std::fabs(g[j + 1]) / bn;
            h.hist.push_back(rel);
            ++it;
            if (!std::isfinite(rel)) {
                st = NAIR_ENUMERIC;
                done = true;
                ++j;
                break;
            }
            if (rel <= rtol || hn == 0.0) {
                done = true;
                ++j;
                break;
            }
        }
        // x += Z y with H[0:j, 0:j] y = g[0:j] (back substitution)
        for (int i = j - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < j; ++k) acc -= Hm(i, k) * y[k];
            y[i] = acc / Hm(i, i);
        }
        for (int i = 0; i < j; ++i) cneg[i] = -y[i];
        if (j > 0) {
            NAIR_HIP(hipMemcpyAsync(K.c.get(), cneg.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
            launch_maxpy(Z, n, j, K.c.get(), x, n, s);   // x -= sum (-y_i) z_i
        }
        if (st == NAIR_ENUMERIC) break;
        launch_residual<double, double>(Aop, b, x, w, nullptr, s);   // the true residual: restart and status
        if (done) {
            st = rel <= rtol ? NAIR_OK : NAIR_ENOCONV;
            if (st != NAIR_OK) {
                launch_mdot(w, 0, 1, w, n, K.part.get(), hd + SS, s);
                double ssr = 0.0;
                read_doubles(hd + SS, &ssr, 1, s);
                if (std::sqrt(ssr) / bn <= rtol) st = NAIR_OK;
            }
            break;
        }
        // (cneg is next written after the synchronising read at the top of the loop)
    }
    return finish(st, it, rel);
}

}  // namespace nair
