// Solve phase: the V-cycle and its transpose, and the stationary iteration.
//
// precision 0: everything in FP64.  precision 1: the cycle reads FP32 copies of
// the level operators and Z and keeps its vectors in FP32 (accumulating in
// FP64, applying the FP64 block inverses); the outer residual b - A x and the
// update x += e stay FP64, so the iteration is FP64 iterative refinement with
// an FP32-stored hierarchy.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

#include "hier.h"

namespace nair {
namespace {


// Per-precision access to a level's matrices and cycle vectors.
template <typename T>
struct Store;

template <>
struct Store<double> {
    static MatView<double> A(const Level &L) { return op_view(L, false).with_groups(L.tune[TU_RELAX]); }
    static MatView<double> Z(const Level &L) { return z_view(L).with_groups(L.tune[TU_RESTRICT]); }
    static MatView<double> AT(const Level &L) { return op_view(L, true).with_groups(L.tune[TU_RELAX_T]); }
    static MatView<double> ZT(const Level &L) { return view(L.ZT).with_groups(L.tune[TU_INTERP_T]); }
    static TransRowsView<double> ATs(const Level &L) { return tr_view(L.atF, L.A.bs).with_groups(L.tune[TU_RELAX_T]); }
    static TransRowsView<double> ATr(const Level &L) {
        return tr_view(L.atF, L.A.bs).with_groups(L.tune[TU_RESIDUAL_T]);
    }
    static TransRowsView<double> ZTr(const Level &L) { return tr_view(L.zt, L.A.bs).with_groups(L.tune[TU_INTERP_T]); }
    static double *r(Level &L) { return L.r.get(); }
    static double *e0(Level &L) { return L.e0.get(); }
    static double *e1(Level &L) { return L.e1.get(); }
    static double *tmp(Level &L) { return L.tmp.get(); }
    static double *fsave(Level &L) { return L.fsave.get(); }
};

template <>
struct Store<float> {
    static MatView<float> A(const Level &L) { return op_view32(L, false).with_groups(L.tune[TU_RELAX]); }
    static MatView<float> Z(const Level &L) { return z_view32(L).with_groups(L.tune[TU_RESTRICT]); }
    static MatView<float> AT(const Level &L) { return op_view32(L, true).with_groups(L.tune[TU_RELAX_T]); }
    static MatView<float> ZT(const Level &L) { return view(L.ZT, L.zt32.get()).with_groups(L.tune[TU_INTERP_T]); }
    static TransRowsView<float> ATs(const Level &L) { return tr_view32(L.atF, L.A.bs).with_groups(L.tune[TU_RELAX_T]); }
    static TransRowsView<float> ATr(const Level &L) {
        return tr_view32(L.atF, L.A.bs).with_groups(L.tune[TU_RESIDUAL_T]);
    }
    static TransRowsView<float> ZTr(const Level &L) { return tr_view32(L.zt, L.A.bs).with_groups(L.tune[TU_INTERP_T]); }
    static float *r(Level &L) { return L.r32.get(); }
    static float *e0(Level &L) { return L.e0_32.get(); }
    static float *e1(Level &L) { return L.e1_32.get(); }
    static float *tmp(Level &L) { return L.tmp32.get(); }
    static float *fsave(Level &L) { return L.fsave32.get(); }
};

// Dense solves of the systems that end on level l: e = A_k^{-1} r (or A_k^{-T} r).
template <typename T>
void direct_solves(const Hier &h, const Level &L, bool trans, const T *r, T *e, hipStream_t s) {
    if (L.ndseg == 0) return;
    TimerScope ts(TK_DENSE, g_timer_level, s);
    launch_dense_matvec<T>(trans ? L.dense_invT.get() : L.dense_inv.get(), L.doff_d.get(), L.ddof0_d.get(),
                           L.dn_d.get(), L.ndseg, L.dmax_n, r, e, s, L.dsys_d.get(), h.active);
}

// Rows of the level's systems that are still iterating (all rows outside batched solves).
Gate gate(const Hier &h, const Level &L) { return Gate{L.bsys.get(), h.active}; }

template <typename T>
const T *coarse_solve(Hier &h, int l, bool fcyc, hipStream_t s);
template <typename T>
const T *coarse_solve_T(Hier &h, int l, bool fcyc, hipStream_t s);

// V-cycle on level l with right-hand side r_l and zero initial guess, no
// pre-relaxation (section 5): restrict, coarse solve, interpolate, nu = k+1
// Jacobi F sweeps (section 5.1), optionally one C sweep.  Returns the
// correction.  The coarse solve is a V-cycle, or for the F-cycle (fcyc) an
// F-cycle followed by a V-cycle on its residual.
template <typename T>
const T *cycle(Hier &h, int l, bool fcyc, hipStream_t s) {
    using S = Store<T>;
    Level &L = *h.lv[l];
    const int bs = h.bs;
    g_timer_level = l;
    if (L.coarsest) {
        direct_solves<T>(h, L, false, S::r(L), S::e0(L), s);
        return S::e0(L);
    }
    Level &C = *h.lv[l + 1];
    {
        TimerScope ts(TK_RESTRICT, l, s);
        launch_restrict<T, T>(S::Z(L), S::r(L), L.cpts.get(), S::r(C), s, gate(h, C));
    }
    const T *ec = coarse_solve<T>(h, l + 1, fcyc, s);
    // on a small level the interpolation rides along with the first sweep
    const bool fuse = few_lanes(L.A.nb, bs) && !L.face.on;
    if (!fuse) {
        TimerScope ts(TK_INTERP, l, s);
        launch_interp<T>(L.pmap.get(), ec, S::e0(L), S::e1(L), L.A.nb, bs, s, gate(h, L));
    }
    const MatView<T> A = S::A(L);
    T *cur = S::e0(L), *oth = S::e1(L);
    {
        // the nu sweeps run back to back; one event pair brackets the group
        TimerScope ts(TK_RELAX, l, s, h.prm.degree + 1);
        int k = 0;
        if (fuse) {
            launch_relax_interp<T, T>(A, L.dinv.get(), S::r(L), L.pmap.get(), ec, L.cf.get(), cur, oth, s,
                                      gate(h, L));
            std::swap(cur, oth);
            k = 1;
        }
        for (; k <= h.prm.degree; ++k) {
            launch_relax<T, T>(A, L.dinv.get(), false, S::r(L), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s,
                               gate(h, L));
            std::swap(cur, oth);
        }
    }
    if (h.prm.relax == 1) {
        launch_relax<T, T>(A, L.dinv.get(), false, S::r(L), cur, oth, nullptr, 0, L.cf.get(), 1, s, gate(h, L));
        std::swap(cur, oth);
    }
    g_timer_level = l;
    direct_solves<T>(h, L, false, S::r(L), cur, s);   // systems that end on this level
    return cur;
}

// The transposed cycle: optional C sweep with D^-T first, nu transposed Jacobi
// F sweeps (pre-relaxation), s = g - A^T y, restrict by P^T, recurse, and
// y += R^T y_c = [Z^T y_c ; y_c].
template <typename T>
const T *cycle_T(Hier &h, int l, bool fcyc, hipStream_t s) {
    using S = Store<T>;
    Level &L = *h.lv[l];
    const int bs = h.bs;
    g_timer_level = l;
    if (L.coarsest) {
        direct_solves<T>(h, L, true, S::r(L), S::e0(L), s);
        return S::e0(L);
    }
    Level &C = *h.lv[l + 1];
    const bool tr = L.atF.on;   // A^T's products from the transposed row copy of A's (F) rows
    const MatView<T> AT = tr ? MatView<T>{} : S::AT(L);
    T *cur = S::e0(L), *oth = S::e1(L);
    int k0 = 0;
    if (h.prm.relax == 1) {   // C sweep first: y_C = D_C^{-T} g_C
        launch_init_T<T>(L.dinv.get(), S::r(L), L.cf.get(), 1, S::e0(L), S::e1(L), L.A.nb, bs, s, gate(h, L));
    } else {                  // the first F sweep from zero needs no product with A^T
        launch_relax_T_first<T>(L.dinv.get(), S::r(L), L.cf.get(), S::e0(L), S::e1(L), L.A.nb, bs, s, gate(h, L));
        std::swap(cur, oth);
        k0 = 1;
    }
    {
        TimerScope ts(TK_RELAX, l, s, h.prm.degree + 1 - k0);
        for (int k = k0; k <= h.prm.degree; ++k) {
            if (tr)
                launch_sweep_tr<T, T>(S::ATs(L), L.dinv.get(), S::r(L), cur, oth, L.flist.get(), L.nF, s, gate(h, L));
            else
                launch_relax<T, T>(AT, L.dinv.get(), true, S::r(L), cur, oth, L.flist.get(), L.nF, L.cf.get(), 0, s,
                                   gate(h, L));
            std::swap(cur, oth);
        }
    }
    if (tr)
        launch_residual_tr<T, T>(S::ATr(L), S::r(L), cur, S::tmp(L), s, gate(h, L));
    else
        launch_residual<T, T>(AT.with_groups(L.tune[TU_RESIDUAL_T]), S::r(L), cur, S::tmp(L), nullptr, s,
                              gate(h, L));
    launch_restrict_T<T>(L.ptptr.get(), L.ptidx.get(), S::tmp(L), S::r(C), L.nc, bs, s, gate(h, C));
    const T *yc = coarse_solve_T<T>(h, l + 1, fcyc, s);
    if (L.zt.on) launch_interp_tr<T, T>(S::ZTr(L), L.cidx.get(), yc, cur, s, gate(h, L));
    else launch_interp_T<T, T>(S::ZT(L), L.cidx.get(), yc, cur, s, gate(h, L));
    g_timer_level = l;
    direct_solves<T>(h, L, true, S::r(L), cur, s);   // systems that end on this level
    return cur;
}

// Coarse solve on level l (its right-hand side in r_l): a V-cycle, or for the
// F-cycle e = F r + V (r - A F r): the F-cycle's correction is kept, the
// residual replaces r_l, and the V-cycle's correction is added.
template <typename T>
const T *coarse_solve(Hier &h, int l, bool fcyc, hipStream_t s) {
    if (!fcyc) return cycle<T>(h, l, false, s);
    using S = Store<T>;
    Level &L = *h.lv[l];
    const Gate g = gate(h, L);
    const T *e1 = cycle<T>(h, l, true, s);
    launch_copy_vec<T>(S::fsave(L), e1, L.A.nb, h.bs, s, g);
    launch_residual<T, T>(S::A(L), S::r(L), S::fsave(L), S::tmp(L), nullptr, s, g);
    launch_copy_vec<T>(S::r(L), S::tmp(L), L.A.nb, h.bs, s, g);
    const T *e2 = cycle<T>(h, l, false, s);
    launch_add_vec<T>(S::fsave(L), e2, L.A.nb, h.bs, s, g);
    return S::fsave(L);
}

// Its transpose: y = V^T r + F^T (r - A^T V^T r).
template <typename T>
const T *coarse_solve_T(Hier &h, int l, bool fcyc, hipStream_t s) {
    if (!fcyc) return cycle_T<T>(h, l, false, s);
    using S = Store<T>;
    Level &L = *h.lv[l];
    const Gate g = gate(h, L);
    const T *y1 = cycle_T<T>(h, l, false, s);
    launch_copy_vec<T>(S::fsave(L), y1, L.A.nb, h.bs, s, g);
    launch_residual<T, T>(S::AT(L).with_groups(L.tune[TU_RESIDUAL_T]), S::r(L), S::fsave(L), S::tmp(L), nullptr, s,
                          g);
    launch_copy_vec<T>(S::r(L), S::tmp(L), L.A.nb, h.bs, s, g);
    const T *y2 = cycle_T<T>(h, l, true, s);
    launch_add_vec<T>(S::fsave(L), y2, L.A.nb, h.bs, s, g);
    return S::fsave(L);
}

// Buffers the F-cycle's coarse solves keep their first correction in.
void ensure_fcycle(Hier &h) {
    if (h.prm.cycle != 1) return;
    for (size_t l = 1; l < h.lv.size(); ++l) {
        Level &L = *h.lv[l];
        const size_t n = static_cast<size_t>(L.A.nb) * h.bs;
        if (h.prm.precision == 1) {
            if (!L.fsave32.get()) L.fsave32.alloc(n);
        } else if (!L.fsave.get()) {
            L.fsave.alloc(n);
        }
    }
}


}  // namespace

namespace {

constexpr int kChunk = kSolveChunk;   // dofs per norm chunk
constexpr int kFirstPoll = 4;       // iterations before the first host check
constexpr int kMaxRun = 64;         // most iterations launched between checks
constexpr double kAim = 0.8;        // fraction of the predicted remaining iterations launched before a check

// Chunk tables, per-system state and history storage of the batched iteration.
void ensure_batch(Hier &h, int max_iter, hipStream_t s) {
    BatchSolve &B = h.batch;
    Level &L0 = *h.lv[0];
    const int nsys = h.nsys;
    if (!B.ready) {
        std::vector<int64_t> clo;
        std::vector<int> clen, cptr(nsys + 1, 0);
        for (int k = 0; k < nsys; ++k) {
            const int64_t d0 = static_cast<int64_t>(L0.seg[k]) * h.bs, d1 = static_cast<int64_t>(L0.seg[k + 1]) * h.bs;
            for (int64_t d = d0; d < d1; d += kChunk) {
                clo.push_back(d);
                clen.push_back(static_cast<int>(std::min<int64_t>(kChunk, d1 - d)));
            }
            cptr[k + 1] = static_cast<int>(clo.size());
        }
        B.nchunk = static_cast<int>(clo.size());
        const int nch = std::max(B.nchunk, 1);
        B.clo.alloc(nch);
        B.clen.alloc(nch);
        B.cptr.alloc(nsys + 1);
        B.part.alloc(nch);
        if (B.nchunk > 0) {
            NAIR_HIP(hipMemcpyAsync(B.clo.get(), clo.data(), sizeof(int64_t) * B.nchunk, hipMemcpyHostToDevice, s));
            NAIR_HIP(hipMemcpyAsync(B.clen.get(), clen.data(), sizeof(int) * B.nchunk, hipMemcpyHostToDevice, s));
        }
        NAIR_HIP(hipMemcpyAsync(B.cptr.get(), cptr.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
        B.bn.alloc(nsys);
        B.last.alloc(nsys);
        B.rtol.alloc(1);
        B.active.alloc(nsys);
        B.status.alloc(nsys);
        B.iters.alloc(nsys);
        B.it.alloc(1);
        B.nact.alloc(1);
        B.nact_acc.alloc(1);
        NAIR_HIP(hipStreamSynchronize(s));   // the host tables end here
        B.ready = true;
    }
    if (B.hist_cap < max_iter) {
        B.hist.alloc(static_cast<size_t>(nsys) * max_iter);
        B.hist_cap = max_iter;
        for (auto &ex : B.exec)   // captured iterations write the old history buffer
            if (ex) {
                (void)hipGraphExecDestroy(ex);
                ex = nullptr;
            }
    }
}

// One iteration of every system: x += B r on the active systems, r = b - A x,
// per-system norms and convergence.  Launch-only (capturable).
template <typename T>
void batch_iteration(Hier &h, bool trans, const double *b, double *x, hipStream_t s, const SolveBufs &B) {
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    const bool fp32 = std::is_same<T, float>::value;
    const T *e = trans ? cycle_T<T>(h, 0, h.prm.cycle == 1, s) : cycle<T>(h, 0, h.prm.cycle == 1, s);
    if (h.prm.form == 1) {
        // scalar form: x += B_S D^{-1} r (transposed: x += D^{-T} B_S^T r) on the caller's block system
        const Gate g0{h.bsys0.get(), h.active};
        if (trans) {
            launch_block_diag_apply<T>(h.d0inv.get(), e, h.rres.get(), nullptr, h.A0.nb, h.bs0, true, s, g0);
            launch_axpy_active<double>(x, h.rres.get(), n, h.bs0, h.bsys0.get(), B.active, s);
        } else {
            launch_axpy_active<T>(x, e, n, h.bs0, h.bsys0.get(), B.active, s);
        }
        double *rout = trans ? L0.r.get() : h.rres.get();
        {
            TimerScope ts(TK_RESIDUAL, 0, s);
            launch_residual<double, double>(trans ? view(h.A0T) : view(h.A0), b, x, rout,
                                            (trans && fp32) ? L0.r32.get() : nullptr, s, g0);
        }
        launch_seg_sumsq(rout, B.clo, B.clen, B.nchunk, B.part, s);
        if (!trans)
            launch_block_diag_apply<double>(h.d0inv.get(), h.rres.get(), L0.r.get(), fp32 ? L0.r32.get() : nullptr,
                                            h.A0.nb, h.bs0, false, s, g0);
    } else {
        launch_axpy_active<T>(x, e, n, h.bs, L0.bsys.get(), B.active, s);
        const MatView<double> Aop = op_view(L0, trans).with_groups(L0.tune[trans ? TU_RESIDUAL_T : TU_RESIDUAL]);
        {
            TimerScope ts(TK_RESIDUAL, 0, s);
            launch_residual<double, double>(Aop, b, x, L0.r.get(), fp32 ? L0.r32.get() : nullptr, s,
                                            gate(h, L0));
        }
        launch_seg_sumsq(L0.r.get(), B.clo, B.clen, B.nchunk, B.part, s);
    }
    launch_seg_check(B.part, B.cptr, h.nsys, B.bn, B.rtol, B.hist_cap, B.hist,
                     B.last, B.active, B.status, B.iters, B.it, B.nact,
                     B.nact_acc, s);
}

// Cycles of stopped systems are skipped: the kernels read the activity flags.
void run_iteration(Hier &h, bool trans, const double *b, double *x, hipStream_t s, const SolveBufs &V) {
    // (one system: the cycle needs no gate, the loop ends when it stops; the
    // update and the norm check still read the flag)
    struct Scope {
        Hier &h;
        Scope(Hier &hh, const int *a) : h(hh) { h.active = a; }
        ~Scope() { h.active = nullptr; }
    } scope(h, h.nsys > 1 ? V.active : nullptr);
    if (h.prm.precision == 1) batch_iteration<float>(h, trans, b, x, s, V);
    else batch_iteration<double>(h, trans, b, x, s, V);
}

SolveBufs bufs_of(BatchSolve &B) {
    SolveBufs V;
    V.nchunk = B.nchunk;
    V.hist_cap = B.hist_cap;
    V.clo = B.clo.get();
    V.clen = B.clen.get();
    V.cptr = B.cptr.get();
    V.part = B.part.get();
    V.bn = B.bn.get();
    V.last = B.last.get();
    V.rtol = B.rtol.get();
    V.hist = B.hist.get();
    V.active = B.active.get();
    V.status = B.status.get();
    V.iters = B.iters.get();
    V.it = B.it.get();
    V.nact = B.nact.get();
    V.nact_acc = B.nact_acc.get();
    return V;
}

// The iteration captured once into a graph for these operands, replayed per step.
hipGraphExec_t batch_graph(Hier &h, bool trans, const double *b, double *x) {
    BatchSolve &B = h.batch;
    const int slot = trans ? 1 : 0;
    if (B.exec[slot] && B.key_b[slot] == b && B.key_x[slot] == x) return B.exec[slot];
    if (B.exec[slot]) {
        NAIR_HIP(hipGraphExecDestroy(B.exec[slot]));
        B.exec[slot] = nullptr;
    }
    if (!B.cap) NAIR_HIP(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
    NAIR_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    try {
        run_iteration(h, trans, b, x, B.cap, bufs_of(B));
    } catch (...) {
        g_capturing = false;
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    g_capturing = false;
    hipGraph_t g = nullptr;
    NAIR_HIP(hipStreamEndCapture(B.cap, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t st = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NAIR_HIP(st);
    B.exec[slot] = ex;
    B.key_b[slot] = b;
    B.key_x[slot] = x;
    return ex;
}

}  // namespace

BatchSolve::~BatchSolve() {
    for (auto ex : exec)
        if (ex) (void)hipGraphExecDestroy(ex);
    if (cap) (void)hipStreamDestroy(cap);
}

nair_status run_solve_batch(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter,
                            bool use_graph, nair_result *res, hipStream_t s) {
    Level &L0 = *h.lv[0];
    BatchSolve &B = h.batch;
    const int nsys = h.nsys;
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    const bool fp32 = h.prm.precision == 1;
    if (trans) ensure_transposes(h, s);
    ensure_batch(h, max_iter, s);
    ensure_fcycle(h);
    B.rtol_host = rtol;
    NAIR_HIP(hipMemcpyAsync(B.rtol.get(), &B.rtol_host, sizeof(double), hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    launch_seg_sumsq(b, B.clo.get(), B.clen.get(), B.nchunk, B.part.get(), s);
    launch_seg_init(B.part.get(), B.cptr.get(), nsys, B.bn.get(), B.last.get(), B.active.get(), B.status.get(),
                    B.iters.get(), B.it.get(), B.nact.get(), B.nact_acc.get(), s);
    if (h.prm.form == 1 && !trans) {   // the scaled cycle's first right-hand side: D^{-1} b
        launch_block_diag_apply<double>(h.d0inv.get(), b, L0.r.get(), fp32 ? L0.r32.get() : nullptr, h.A0.nb, h.bs0,
                                        false, s);
    } else {
        NAIR_HIP(hipMemcpyAsync(L0.r.get(), b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (fp32) launch_to_float(b, L0.r32.get(), n, s);
    }
    hipGraphExec_t ex = use_graph ? batch_graph(h, trans, b, x) : nullptr;
    const SolveBufs V = bufs_of(B);

    std::vector<double> last(nsys), prev(nsys, 1.0);
    int done = 0;        // iterations launched
    int run = std::min(kFirstPoll, max_iter);
    int nact = read_int(B.nact.get(), s);
    while (nact > 0 && done < max_iter) {
        for (int i = 0; i < run; ++i) {
            if (ex) NAIR_HIP(hipGraphLaunch(ex, s));
            else run_iteration(h, trans, b, x, s, V);
        }
        done += run;
        read_device({{B.last.get(), last.data(), sizeof(double) * nsys}, {B.nact.get(), &nact, sizeof(int)}}, s);
        if (nact == 0 || done >= max_iter) break;
        // iterations still needed by the slowest system, from its rate over the last run
        double need = 1.0;
        for (int k = 0; k < nsys; ++k) {
            if (!(last[k] > rtol)) continue;
            const double rho = std::pow(last[k] / prev[k], 1.0 / run);
            const double nk = (rho > 0.0 && rho < 1.0) ? std::log(rtol / last[k]) / std::log(rho) : run;
            need = std::max(need, nk);
        }
        prev = last;
        // aim a little short of the prediction and at most double the
        // iterations done (early iterations converge slower than later ones, so
        // an early prediction runs long): an iteration launched after every
        // system has stopped costs its launches, one more check one round trip
        const double cap = std::min<double>({static_cast<double>(kMaxRun), static_cast<double>(max_iter - done),
                                             static_cast<double>(done)});
        run = std::max(1, static_cast<int>(std::min(std::floor(kAim * need), cap)));
    }

    // status, iteration counts and histories in one read
    std::vector<int> st(nsys), it(nsys);
    std::vector<double> hist(static_cast<size_t>(nsys) * B.hist_cap);
    read_device({{B.status.get(), st.data(), sizeof(int) * nsys},
                 {B.iters.get(), it.data(), sizeof(int) * nsys},
                 {B.hist.get(), hist.data(), sizeof(double) * hist.size()}},
                s);
    B.hist_host.assign(nsys, {});
    nair_status worst = NAIR_OK;
    for (int k = 0; k < nsys; ++k) {
        auto &hk = B.hist_host[k];
        hk.assign(hist.begin() + static_cast<size_t>(k) * B.hist_cap,
                  hist.begin() + static_cast<size_t>(k) * B.hist_cap + std::min(it[k], B.hist_cap));
        nair_result rr{0, 0, 0.0, 0.0, 0.0};
        rr.iters = static_cast<int32_t>(hk.size());
        rr.converged = st[k] == 0 ? 1 : 0;
        rr.relres = hk.empty() ? 0.0 : hk.back();
        if (rr.iters > 0) {
            const double hK = hk.back();
            rr.rho_avg = std::pow(hK, 1.0 / rr.iters);
            rr.rho_last5 = rr.iters > 5 ? std::pow(hK / hk[rr.iters - 6], 0.2) : rr.rho_avg;
        }
        if (res) res[k] = rr;
        const nair_status sk = static_cast<nair_status>(st[k]);
        if (sk == NAIR_ENUMERIC) worst = NAIR_ENUMERIC;
        else if (sk == NAIR_ENOCONV && worst == NAIR_OK) worst = NAIR_ENOCONV;
    }
    h.hist = B.hist_host.empty() ? std::vector<double>() : B.hist_host[0];
    NAIR_HIP(hipStreamSynchronize(s));
    return worst;
}

// One system in caller-provided buffers (the no-alloc solve): the iteration of
// run_solve_batch, launched eagerly, with its host bookkeeping on the stack,
// reads by plain copies into it (not the pinned staging buffer) and only the
// last six history entries read back.  The kernel timer is off.  x is cleared,
// V's rtol set and its chunk tables filled by the caller, on the stream,
// before this runs.
nair_status run_solve_bufs(Hier &h, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                           hipStream_t s, const SolveBufs &V) {
    struct TimerOff {
        TimerOff() { g_timer_off = true; }
        ~TimerOff() { g_timer_off = false; }
    } timer_off;
    auto rd = [s](void *host, const void *dev, size_t bytes) {
        NAIR_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    };
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    const bool fp32 = h.prm.precision == 1;
    launch_seg_sumsq(b, V.clo, V.clen, V.nchunk, V.part, s);
    launch_seg_init(V.part, V.cptr, 1, V.bn, V.last, V.active, V.status, V.iters, V.it, V.nact, V.nact_acc, s);
    if (h.prm.form == 1) {
        launch_block_diag_apply<double>(h.d0inv.get(), b, L0.r.get(), fp32 ? L0.r32.get() : nullptr, h.A0.nb, h.bs0,
                                        false, s);
    } else {
        NAIR_HIP(hipMemcpyAsync(L0.r.get(), b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (fp32) launch_to_float(b, L0.r32.get(), n, s);
    }
    double last = 0.0, prev = 1.0;
    int done = 0;
    int run = std::min(kFirstPoll, max_iter);
    int nact = 0;
    rd(&nact, V.nact, sizeof(int));
    NAIR_HIP(hipStreamSynchronize(s));
    while (nact > 0 && done < max_iter) {
        for (int i = 0; i < run; ++i) run_iteration(h, false, b, x, s, V);
        done += run;
        rd(&last, V.last, sizeof(double));
        rd(&nact, V.nact, sizeof(int));
        NAIR_HIP(hipStreamSynchronize(s));
        if (nact == 0 || done >= max_iter) break;
        double need = 1.0;
        if (last > rtol) {
            const double rho = std::pow(last / prev, 1.0 / run);
            need = (rho > 0.0 && rho < 1.0) ? std::log(rtol / last) / std::log(rho) : run;
        }
        prev = last;
        const double cap = std::min<double>({static_cast<double>(kMaxRun), static_cast<double>(max_iter - done),
                                             static_cast<double>(done)});
        run = std::max(1, static_cast<int>(std::min(std::floor(kAim * need), cap)));
    }
    int st = 0, it = 0;
    rd(&st, V.status, sizeof(int));
    rd(&it, V.iters, sizeof(int));
    NAIR_HIP(hipStreamSynchronize(s));
    const int K = std::min(it, V.hist_cap);
    double tail[6] = {0, 0, 0, 0, 0, 0};
    const int nt = std::min(K, 6);
    if (nt > 0) rd(tail, V.hist + (K - nt), sizeof(double) * nt);
    NAIR_HIP(hipStreamSynchronize(s));
    nair_result rr{0, 0, 0.0, 0.0, 0.0};
    rr.iters = K;
    rr.converged = st == 0 ? 1 : 0;
    if (K > 0) {
        const double hK = tail[nt - 1];
        rr.relres = hK;
        rr.rho_avg = std::pow(hK, 1.0 / K);
        rr.rho_last5 = K > 5 ? std::pow(hK / tail[0], 0.2) : rr.rho_avg;
    }
    if (res) *res = rr;
    h.hist.clear();   // (keeps its storage: no history is reported for this solve)
    return static_cast<nair_status>(st);
}

// One system: the same device-side iteration, launched eagerly (a graph
// capture per call would cost more than it saves on one solve).
nair_status run_solve(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                      hipStream_t s) {
    if (h.prm.gmres > 0) return run_gmres(h, trans, b, x, rtol, max_iter, res, s);
    return run_solve_batch(h, trans, b, x, rtol, max_iter, false, res, s);
}

void prepare_cycle(Hier &h, bool trans, hipStream_t s) {
    if (trans) ensure_transposes(h, s);
    ensure_fcycle(h);
}

void apply_cycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s) {
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    const bool fp32 = h.prm.precision == 1;
    const bool scaled = h.prm.form == 1;
    if (scaled && !trans) {   // the scaled cycle reads D^{-1} r
        launch_block_diag_apply<double>(h.d0inv.get(), r, L0.r.get(), fp32 ? L0.r32.get() : nullptr, h.A0.nb, h.bs0,
                                        false, s);
    } else {
        NAIR_HIP(hipMemcpyAsync(L0.r.get(), r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (fp32) launch_to_float(r, L0.r32.get(), n, s);
    }
    if (fp32) {
        const float *out = trans ? cycle_T<float>(h, 0, h.prm.cycle == 1, s) : cycle<float>(h, 0, h.prm.cycle == 1, s);
        if (scaled && trans) {
            launch_block_diag_apply<float>(h.d0inv.get(), out, e, nullptr, h.A0.nb, h.bs0, true, s);
        } else {
            NAIR_HIP(hipMemsetAsync(e, 0, sizeof(double) * n, s));
            launch_axpy<float>(e, out, n, s);
        }
    } else {
        const double *out = trans ? cycle_T<double>(h, 0, h.prm.cycle == 1, s) : cycle<double>(h, 0, h.prm.cycle == 1, s);
        if (scaled && trans)
            launch_block_diag_apply<double>(h.d0inv.get(), out, e, nullptr, h.A0.nb, h.bs0, true, s);
        else
            NAIR_HIP(hipMemcpyAsync(e, out, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
}

void run_vcycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s) {
    prepare_cycle(h, trans, s);
    apply_cycle(h, trans, r, e, s);
    NAIR_HIP(hipStreamSynchronize(s));
}

}  // namespace nair
