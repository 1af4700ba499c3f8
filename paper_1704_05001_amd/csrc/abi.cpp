// The C ABI: argument checks, device selection, error capture.
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "hier.h"

struct nair_hier_s {
    nair::ExtAlloc ext;   // (declared before h: h's buffers go back to it when h is destroyed)
    nair::Hier h;
};

namespace {

thread_local std::string g_last_error;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename F>
nair_status guarded_on(nair_hier h, void *stream, F &&body) {
    // device memory from the handle's allocator, if it has one, for use on the call's stream
    nair::AllocScope scope(h && h->ext.on ? &h->ext : nullptr, stream);
    try {
        return body();
    } catch (const nair::Error &e) {
        g_last_error = e.msg;
        if (h) h->h.err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        if (h) h->h.err = g_last_error;
        return NAIR_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        if (h) h->h.err = g_last_error;
        return NAIR_EDEVICE;
    }
}

template <typename F>
nair_status guarded(nair_hier h, F &&body) {
    return guarded_on(h, nullptr, std::forward<F>(body));
}

nair_status bad(nair_hier h, const std::string &msg) {
    g_last_error = msg;
    if (h) h->h.err = msg;
    return NAIR_EINVAL;
}

bool unit_interval(double v) { return v >= 0.0 && v < 1.0; }

}  // namespace

extern "C" {

nair_status nair_default_params(nair_params *p) {
    if (!p) return NAIR_EINVAL;
    p->degree = 1;
    p->theta = 0.75;
    p->phi = 0.025;
    p->drop = 1e-3;
    p->relax = 0;
    p->max_levels = 30;
    p->max_coarse_dofs = 128;
    p->seed = 0;
    p->cf_override_host = nullptr;
    p->precision = 0;
    p->tuning = nullptr;
    p->form = 0;
    p->cycle = 0;
    p->gmres = 0;
    p->faces = 1;
    p->sweep_copy = -1;
    p->matrix_cores = 1;
    p->allocator = nullptr;
    return NAIR_OK;
}

}  // extern "C"

static nair_status setup_common(int32_t nsys, const int32_t *sys_nb, int32_t nb, int32_t bs, const int32_t *rowptr,
                                const int32_t *colidx, const double *vals, const nair_params *p, void *stream,
                                nair_hier *out) {
    if (!out) return bad(nullptr, "out is NULL");
    *out = nullptr;
    if (!p) return bad(nullptr, "params is NULL");
    if (nb < 1 || bs < 1 || bs > nair::kMaxBs)
        return bad(nullptr, "need nb >= 1 and 1 <= bs <= " + std::to_string(nair::kMaxBs));
    if (static_cast<int64_t>(nb) * bs > 0x7fffffffLL) return bad(nullptr, "nb*bs exceeds int32");
    if (!rowptr || !colidx || !vals) return bad(nullptr, "NULL matrix array");
    if (p->degree < 0 || p->degree > 16) return bad(nullptr, "degree must be in [0, 16]");
    if (!unit_interval(p->theta) || !unit_interval(p->phi) || !unit_interval(p->drop))
        return bad(nullptr, "theta, phi and drop must lie in [0, 1)");
    if (p->relax != 0 && p->relax != 1) return bad(nullptr, "relax must be 0 (F) or 1 (FC)");
    if (p->precision != 0 && p->precision != 1) return bad(nullptr, "precision must be 0 (FP64) or 1 (FP32 hierarchy)");
    if (p->form != 0 && p->form != 1) return bad(nullptr, "form must be 0 (block) or 1 (scalar after scaling)");
    if (p->cycle != 0 && p->cycle != 1) return bad(nullptr, "cycle must be 0 (V) or 1 (F)");
    if (p->faces != 0 && p->faces != 1) return bad(nullptr, "faces must be 0 or 1");
    if (p->sweep_copy < -1 || p->sweep_copy > 1) return bad(nullptr, "sweep_copy must be -1, 0 or 1");
    if (p->matrix_cores != 0 && p->matrix_cores != 1) return bad(nullptr, "matrix_cores must be 0 or 1");
    if (p->gmres < 0 || p->gmres > nair::kMaxGmres)
        return bad(nullptr, "gmres must be 0 (stationary iteration) or a restart length in [1, 200]");
    if (p->max_levels < 1 || p->max_levels > nair::kMaxLevels) return bad(nullptr, "max_levels must be in [1, 64]");
    if (p->max_coarse_dofs < 0 || p->max_coarse_dofs > nair::kStallDenseDofs)
        return bad(nullptr, "max_coarse_dofs must be in [0, 4096]");
    if (p->allocator && (!p->allocator->alloc || !p->allocator->free))
        return bad(nullptr, "allocator needs both alloc and free");
    nair_hier h = new (std::nothrow) nair_hier_s();
    if (!h) return NAIR_ENOMEM;
    if (p->allocator) {
        h->ext.on = true;
        h->ext.a = *p->allocator;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    nair_status st = guarded_on(h, stream, [&]() -> nair_status {
        NAIR_HIP(hipGetDevice(&h->h.device));
        h->h.prm = *p;
        nair::g_matrix_cores = p->matrix_cores != 0;
        nair::build_hierarchy(h->h, nsys, sys_nb, nb, bs, rowptr, colidx, vals, s);
        // the no-alloc solve's scratch array: its device address, looked up once per device here so that
        // nair_solve_noalloc itself loads nothing
        if (nsys == 1) nair::noalloc_prepare();
        if (p->tuning) nair::apply_tuning(h->h, p->tuning);
        h->h.prm.cf_override_host = nullptr;   // host pointers not kept past the call
        h->h.prm.tuning = nullptr;
        h->h.prm.allocator = nullptr;          // (copied into the handle)
        return NAIR_OK;
    });
    if (st != NAIR_OK) {
        (void)hipStreamSynchronize(s);
        delete h;
        return st;
    }
    *out = h;
    return NAIR_OK;
}

extern "C" {

nair_status nair_setup(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                       const nair_params *p, void *stream, nair_hier *out) {
    const int32_t one[1] = {nb};
    return setup_common(1, one, nb, bs, rowptr, colidx, vals, p, stream, out);
}

nair_status nair_setup_batch(int32_t nsys, const int32_t *sys_nb, int32_t bs, const int32_t *rowptr,
                             const int32_t *colidx, const double *vals, const nair_params *p, void *stream,
                             nair_hier *out) {
    if (out) *out = nullptr;
    if (nsys < 1 || !sys_nb) return bad(nullptr, "need nsys >= 1 and a system size array");
    int64_t nb = 0;
    for (int32_t k = 0; k < nsys; ++k) {
        if (sys_nb[k] < 1) return bad(nullptr, "every system needs at least one block row");
        nb += sys_nb[k];
    }
    if (nb > 0x7fffffffLL) return bad(nullptr, "total block rows exceed int32");
    return setup_common(nsys, sys_nb, static_cast<int32_t>(nb), bs, rowptr, colidx, vals, p, stream, out);
}

static nair_status solve_common(nair_hier h, bool trans, const double *b, double *x, double rtol, int32_t max_iter,
                                nair_result *res, void *stream) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (!b || !x) return bad(h, "NULL vector");
    if (!(rtol >= 0.0) || max_iter < 0) return bad(h, "need rtol >= 0 and max_iter >= 0");
    if (h->h.nsys != 1) return bad(h, "the handle holds several systems: use nair_solve_batch");
    DeviceGuard dg(h->h.device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return guarded_on(h, stream, [&]() { return nair::run_solve(h->h, trans, b, x, rtol, max_iter, res, s); });
}

nair_status nair_solve_batch(nair_hier h, int32_t trans, const double *b, double *x, double rtol, int32_t max_iter,
                             int32_t use_graph, nair_result *res, void *stream) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (!b || !x) return bad(h, "NULL vector");
    if (!(rtol >= 0.0) || max_iter < 0) return bad(h, "need rtol >= 0 and max_iter >= 0");
    if (trans != 0 && trans != 1) return bad(h, "trans must be 0 or 1");
    if (h->h.prm.gmres > 0) return bad(h, "GMRES acceleration solves one system: use nair_solve / nair_solve_T");
    DeviceGuard dg(h->h.device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return guarded_on(h, stream, [&]() {
        return nair::run_solve_batch(h->h, trans != 0, b, x, rtol, max_iter, use_graph != 0, res, s);
    });
}

nair_status nair_autotune(nair_hier h, int32_t reps, int8_t *table, void *stream) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (reps < 1 || reps > 10000) return bad(h, "reps must be in [1, 10000]");
    DeviceGuard dg(h->h.device);
    return guarded_on(h, stream, [&]() {
        nair::autotune(h->h, reps, table, static_cast<hipStream_t>(stream));
        return NAIR_OK;
    });
}

nair_status nair_batch_history(nair_hier h, int32_t sys, double *buf, int32_t cap, int32_t *n) {
    if (!h) return bad(nullptr, "handle is NULL");
    const auto &hh = h->h.batch.hist_host;
    if (sys < 0 || sys >= h->h.nsys) return bad(h, "system index out of range");
    const std::vector<double> empty;
    const std::vector<double> &v = sys < static_cast<int32_t>(hh.size()) ? hh[sys] : empty;
    const int32_t total = static_cast<int32_t>(v.size());
    if (n) *n = total;
    if (buf)
        for (int32_t i = 0; i < total && i < cap; ++i) buf[i] = v[i];
    return NAIR_OK;
}

nair_status nair_get_systems(nair_hier h, int32_t lvl, int32_t cap, int32_t *nsys, int32_t *seg, int8_t *mode,
                             int64_t *dense_off) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (lvl < 0 || lvl >= static_cast<int32_t>(h->h.lv.size())) return bad(h, "bad level");
    const nair::Level &L = *h->h.lv[lvl];
    const int32_t ns = h->h.nsys;
    if (nsys) *nsys = ns;
    if ((seg || mode || dense_off) && cap < ns) return bad(h, "arrays hold fewer entries than systems");
    for (int32_t k = 0; k < ns; ++k) {
        if (seg) seg[k] = L.seg[k];
        if (mode) mode[k] = L.mode[k];
        if (dense_off) dense_off[k] = -1;
    }
    if (seg) seg[ns] = L.seg[ns];
    if (dense_off)
        for (int k = 0; k < L.ndseg; ++k) dense_off[L.dsys[k]] = L.doff[k];
    return NAIR_OK;
}

nair_status nair_solve(nair_hier h, const double *b, double *x, double rtol, int32_t max_iter, nair_result *res,
                       void *stream) {
    return solve_common(h, false, b, x, rtol, max_iter, res, stream);
}

nair_status nair_solve_T(nair_hier h, const double *g, double *y, double rtol, int32_t max_iter, nair_result *res,
                         void *stream) {
    return solve_common(h, true, g, y, rtol, max_iter, res, stream);
}

nair_status nair_solve_noalloc(nair_hier h, const double *b, double *x, double rtol, int32_t max_iter,
                               nair_result *res, void *stream) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (!b || !x) return bad(h, "NULL vector");
    if (!(rtol >= 0.0) || max_iter < 0) return bad(h, "need rtol >= 0 and max_iter >= 0");
    DeviceGuard dg(h->h.device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return guarded(h, [&]() { return nair::solve_noalloc(h->h, b, x, rtol, max_iter, res, s); });
}

static nair_status vcycle_common(nair_hier h, bool trans, const double *r, double *e, void *stream) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (!r || !e) return bad(h, "NULL vector");
    DeviceGuard dg(h->h.device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return guarded_on(h, stream, [&]() {
        nair::run_vcycle(h->h, trans, r, e, s);
        return NAIR_OK;
    });
}

nair_status nair_vcycle(nair_hier h, const double *r, double *e, void *stream) {
    return vcycle_common(h, false, r, e, stream);
}

nair_status nair_vcycle_T(nair_hier h, const double *g, double *y, void *stream) {
    return vcycle_common(h, true, g, y, stream);
}

nair_status nair_grad_vals(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx, const double *ybar,
                           const double *x, double *grad_vals, void *stream) {
    if (nb < 1 || bs < 1 || bs > nair::kMaxBs) return bad(nullptr, "need nb >= 1 and 1 <= bs <= 32");
    if (!rowptr || !colidx || !ybar || !x || !grad_vals) return bad(nullptr, "NULL array");
    return guarded(nullptr, [&]() {
        nair::grad_vals(nb, bs, rowptr, colidx, ybar, x, grad_vals, static_cast<hipStream_t>(stream));
        return NAIR_OK;
    });
}

nair_status nair_history(nair_hier h, double *buf, int32_t cap, int32_t *n) {
    if (!h) return bad(nullptr, "handle is NULL");
    const int32_t total = static_cast<int32_t>(h->h.hist.size());
    if (n) *n = total;
    if (buf)
        for (int32_t i = 0; i < total && i < cap; ++i) buf[i] = h->h.hist[i];
    return NAIR_OK;
}

nair_status nair_info(nair_hier h, int32_t *levels, int32_t *nb_per_level, int64_t *nnzb_per_level, double *oc,
                      double *cc) {
    if (!h) return bad(nullptr, "handle is NULL");
    DeviceGuard dg(h->h.device);
    return guarded(h, [&]() {
        const int L = static_cast<int>(h->h.lv.size());
        if (levels) *levels = L;
        for (int l = 0; l < L && l < nair::kMaxLevels; ++l) {
            if (nb_per_level) nb_per_level[l] = h->h.lv[l]->A.nb;
            if (nnzb_per_level) nnzb_per_level[l] = h->h.lv[l]->A.nnzb;
        }
        if (oc || cc) nair::complexity(h->h, oc, cc, nullptr);
        return NAIR_OK;
    });
}

nair_status nair_get_level(nair_hier h, int32_t lvl, nair_level_view *v) {
    if (!h) return bad(nullptr, "handle is NULL");
    if (!v || lvl < 0 || lvl >= static_cast<int32_t>(h->h.lv.size())) return bad(h, "bad level or view");
    const nair::Level &L = *h->h.lv[lvl];
    std::memset(v, 0, sizeof(*v));
    v->nb = L.A.nb;
    v->bs = L.A.bs;
    v->nnzb = static_cast<int32_t>(L.A.nnzb);
    v->coarsest = L.coarsest ? 1 : 0;
    v->rowptr = L.A.rowptr.get();
    v->colidx = L.A.colidx.get();
    v->vals = L.A.vals.get();
    v->dinv = L.dinv.get();
    v->bnorm = L.bnorm.get();
    v->mask = L.mask.get();
    v->lambda = L.lambda.get();
    v->cf = L.cf.get();
    v->cidx = L.cidx.get();
    v->dround = L.dround.get();
    v->pmis_rounds = L.rounds;
    if (!L.coarsest) {
        v->pmap = L.pmap.get();
        v->nc = L.nc;
        v->z_nnzb = static_cast<int32_t>(L.Z.nnzb);
        v->z_rowptr = L.Z.rowptr.get();
        v->z_colidx = L.Z.colidx.get();
        v->z_vals = L.Z.vals.get();
    }
    v->dense_n = L.dense_n;
    v->dense_inv = L.dense_inv.get();
    if (L.margin.get() &&
        hipMemcpy(v->margin, L.margin.get(), sizeof(v->margin), hipMemcpyDeviceToHost) != hipSuccess)
        return bad(h, "reading the decision-margin counts failed");
    v->sweep_nnzb = -1;
    if (L.sweep.on && hipMemcpy(&v->sweep_nnzb, L.sweep.rowptr.get() + L.sweep.nF, sizeof(int32_t),
                                hipMemcpyDeviceToHost) != hipSuccess)
        return bad(h, "reading the sweep copy's size failed");
    if (L.face.on) {
        v->face_rmax = L.face.rmax;
        v->face_cmax = L.face.cmax;
        v->face_meta = L.face.meta.get();
        v->face_vals = L.face.vals.get();
        v->face_dvals = L.face.dvals.get();
    }
    return NAIR_OK;
}

const char *nair_last_error(nair_hier h) { return h ? h->h.err.c_str() : g_last_error.c_str(); }

void nair_destroy(nair_hier h) {
    if (!h) return;
    DeviceGuard dg(h->h.device);
    delete h;   // (buffers from a caller's allocator go back to it, by pointer, as h->h is destroyed)
}

nair_status nair_timer_select(int32_t kernel, int32_t level) {
    if (kernel < -1 || kernel > nair::TK_BLOCKPROD) return bad(nullptr, "unknown kernel id");
    nair::timer_select(kernel, level);
    return NAIR_OK;
}

nair_status nair_timer_read(int64_t *launches, double *total_ms) {
    return guarded(nullptr, [&]() {
        nair::timer_read(launches, total_ms);
        return NAIR_OK;
    });
}

nair_status nair_pool_trim(void) {
    return guarded(nullptr, []() {
        nair::pool_trim();
        return NAIR_OK;
    });
}

}  // extern "C"
