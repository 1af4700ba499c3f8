// Lane-group autotuner of the cycle kernels.
//
// Every cycle kernel maps a block row onto G groups of bs lanes (G * bs <= 256).
// The default G comes from the level's average row length (the most groups on
// levels too small to fill the chip); the best choice also depends on how many
// rows a level has and on the block size, so the tuner times each power-of-two
// G on the level's own operands and keeps the fastest, per level and per
// kernel.  A choice must beat the default by 3% to replace it, so timing noise
// does not flip it.  Small levels are left at their default.
#include <algorithm>
#include <vector>

#include "hier.h"

namespace nair {
namespace {

constexpr double kKeepDefault = 0.97;

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        NAIR_HIP(hipEventCreate(&a));
        NAIR_HIP(hipEventCreate(&b));
    }
    ~Events() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Average milliseconds of `reps` launches of f after one untimed launch.
template <typename F>
double time_launches(F &&f, int reps, Events &ev, hipStream_t s) {
    f();
    NAIR_HIP(hipEventRecord(ev.a, s));
    for (int i = 0; i < reps; ++i) f();
    NAIR_HIP(hipEventRecord(ev.b, s));
    NAIR_HIP(hipEventSynchronize(ev.b));
    float ms = 0.0f;
    NAIR_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    return static_cast<double>(ms) / reps;
}

// Fastest G for one kernel (0 keeps the row-length default).
template <typename F>
int8_t pick(F &&launch_with, int bs, int reps, Events &ev, hipStream_t s) {
    const double t0 = time_launches([&] { launch_with(0); }, reps, ev, s);
    double best = t0;
    int bestG = 0;
    for (int G = 1; G <= max_groups(bs); G *= 2) {
        const double t = time_launches([&] { launch_with(G); }, reps, ev, s);
        if (t < best) {
            best = t;
            bestG = G;
        }
    }
    return (bestG != 0 && best <= kKeepDefault * t0) ? static_cast<int8_t>(bestG) : 0;
}

template <typename T>
struct Vecs;
template <>
struct Vecs<double> {
    static MatView<double> A(const Level &L) { return op_view(L, false); }
    static MatView<double> Z(const Level &L) { return z_view(L); }
    static MatView<double> AT(const Level &L) { return op_view(L, true); }
    static MatView<double> ZT(const Level &L) { return view(L.ZT); }
    static TransRowsView<double> ATr(const Level &L) { return tr_view(L.atF, L.A.bs); }
    static TransRowsView<double> ZTr(const Level &L) { return tr_view(L.zt, L.A.bs); }
    static double *r(Level &L) { return L.r.get(); }
    static double *e0(Level &L) { return L.e0.get(); }
    static double *e1(Level &L) { return L.e1.get(); }
    static double *tmp(Level &L) { return L.tmp.get(); }
};
template <>
struct Vecs<float> {
    static MatView<float> A(const Level &L) { return op_view32(L, false); }
    static MatView<float> Z(const Level &L) { return z_view32(L); }
    static MatView<float> AT(const Level &L) { return op_view32(L, true); }
    static MatView<float> ZT(const Level &L) { return view(L.ZT, L.zt32.get()); }
    static TransRowsView<float> ATr(const Level &L) { return tr_view32(L.atF, L.A.bs); }
    static TransRowsView<float> ZTr(const Level &L) { return tr_view32(L.zt, L.A.bs); }
    static float *r(Level &L) { return L.r32.get(); }
    static float *e0(Level &L) { return L.e0_32.get(); }
    static float *e1(Level &L) { return L.e1_32.get(); }
    static float *tmp(Level &L) { return L.tmp32.get(); }
};

template <typename T>
void clear_vectors(Level &L, hipStream_t s) {
    using V = Vecs<T>;
    const size_t n = static_cast<size_t>(L.A.nb) * L.A.bs;
    for (T *p : {V::r(L), V::e0(L), V::e1(L), V::tmp(L)}) NAIR_HIP(hipMemsetAsync(p, 0, sizeof(T) * n, s));
}

template <typename T>
void tune_levels(Hier &h, int reps, hipStream_t s) {
    using V = Vecs<T>;
    Events ev;
    for (auto &Lp : h.lv) clear_vectors<T>(*Lp, s);
    for (size_t l = 0; l + 1 < h.lv.size(); ++l) {
        Level &L = *h.lv[l];
        Level &C = *h.lv[l + 1];
        if (L.coarsest) break;
        // small levels keep their default (the most groups): timing their kernels
        // back to back with warm caches does not predict them inside a cycle
        if (few_lanes(L.A.nb, L.A.bs)) continue;
        const int bs = L.A.bs;
        const MatView<T> A = V::A(L), Z = V::Z(L);
        L.tune[TU_RELAX] = pick(
            [&](int G) {
                launch_relax<T, T>(A.with_groups(G), L.dinv.get(), false, V::r(L), V::e0(L), V::e1(L),
                                   L.flist.get(), L.nF, L.cf.get(), 0, s);
            },
            bs, reps, ev, s);
        // the transposed cycle's kernels: from the transposed row copies where the level has them
        if (L.atF.on) {
            const TransRowsView<T> ATr = V::ATr(L);
            L.tune[TU_RELAX_T] = pick(
                [&](int G) {
                    launch_sweep_tr<T, T>(ATr.with_groups(G), L.dinv.get(), V::r(L), V::e0(L), V::e1(L),
                                          L.flist.get(), L.nF, s);
                },
                bs, reps, ev, s);
            L.tune[TU_RESIDUAL_T] = pick(
                [&](int G) { launch_residual_tr<T, T>(ATr.with_groups(G), V::r(L), V::e0(L), V::tmp(L), s); }, bs,
                reps, ev, s);
        } else {
            const MatView<T> AT = V::AT(L);
            L.tune[TU_RELAX_T] = pick(
                [&](int G) {
                    launch_relax<T, T>(AT.with_groups(G), L.dinv.get(), true, V::r(L), V::e0(L), V::e1(L),
                                       L.flist.get(), L.nF, L.cf.get(), 0, s);
                },
                bs, reps, ev, s);
            L.tune[TU_RESIDUAL_T] = pick(
                [&](int G) {
                    launch_residual<T, T>(AT.with_groups(G), V::r(L), V::e0(L), V::tmp(L), nullptr, s);
                },
                bs, reps, ev, s);
        }
        L.tune[TU_RESTRICT] = pick(
            [&](int G) { launch_restrict<T, T>(Z.with_groups(G), V::r(L), L.cpts.get(), V::r(C), s); }, bs, reps,
            ev, s);
        if (L.zt.on) {
            const TransRowsView<T> ZTr = V::ZTr(L);
            L.tune[TU_INTERP_T] = pick(
                [&](int G) { launch_interp_tr<T, T>(ZTr.with_groups(G), L.cidx.get(), V::e0(C), V::e1(L), s); },
                bs, reps, ev, s);
        } else {
            const MatView<T> ZT = V::ZT(L);
            L.tune[TU_INTERP_T] = pick(
                [&](int G) { launch_interp_T<T, T>(ZT.with_groups(G), L.cidx.get(), V::e0(C), V::e1(L), s); }, bs,
                reps, ev, s);
        }
    }
    // the outer residual is FP64 in both precisions (the scalar form's runs on the caller's blocks, untuned)
    Level &L0 = *h.lv[0];
    if (!L0.coarsest && h.prm.form == 0) {
        clear_vectors<double>(L0, s);
        L0.tune[TU_RESIDUAL] = pick(
            [&](int G) {
                launch_residual<double, double>(op_view(L0, false).with_groups(G), L0.r.get(), L0.e0.get(), L0.tmp.get(),
                                                nullptr, s);
            },
            L0.A.bs, reps, ev, s);
    }
}

}  // namespace

void drop_graphs(Hier &h) {
    for (auto &ex : h.batch.exec)
        if (ex) {
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
}

void autotune(Hier &h, int reps, int8_t *table, hipStream_t s) {
    ensure_transposes(h, s);
    for (auto &Lp : h.lv) std::fill(Lp->tune, Lp->tune + TU_KINDS, static_cast<int8_t>(0));
    if (h.prm.precision == 1) tune_levels<float>(h, reps, s);
    else tune_levels<double>(h, reps, s);
    NAIR_HIP(hipStreamSynchronize(s));
    drop_graphs(h);   // captured iterations hold the old launch shapes
    if (table) {
        std::fill(table, table + kTuneLevels * TU_KINDS, static_cast<int8_t>(0));
        for (size_t l = 0; l < h.lv.size() && l < static_cast<size_t>(kTuneLevels); ++l)
            std::copy(h.lv[l]->tune, h.lv[l]->tune + TU_KINDS, table + l * TU_KINDS);
    }
}

void apply_tuning(Hier &h, const int8_t *table) {
    for (size_t l = 0; l < h.lv.size() && l < static_cast<size_t>(kTuneLevels); ++l)
        for (int k = 0; k < TU_KINDS; ++k) {
            const int8_t g = table[l * TU_KINDS + k];
            h.lv[l]->tune[k] = (g > 0 && (g & (g - 1)) == 0) ? g : 0;   // powers of two only
        }
    drop_graphs(h);
}

}  // namespace nair
