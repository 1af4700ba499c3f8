// Hierarchy data held by a nair_hier handle (internal).
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace nair {

// Cycle kernels with a tunable lane-group count, per level.
enum TuneKind {
    TU_RELAX = 0,       // Jacobi sweeps with A (F rows; also the C sweep)
    TU_RELAX_T = 1,     // transposed sweeps with A^T
    TU_RESIDUAL_T = 2,  // s = g - A^T y in the transposed cycle (and the outer transposed residual)
    TU_RESTRICT = 3,    // r_c = r_C + Z r_F
    TU_INTERP_T = 4,    // y += R^T y_c
    TU_RESIDUAL = 5,    // outer residual b - A x (level 0)
    TU_KINDS = 6
};
constexpr int kTuneLevels = 64;

struct Level {
    DevBSR A;                       // level operator (A_0 = copy of the input, then K = R A P)
    bool coarsest = false;          // every system left is solved directly here
    int8_t tune[TU_KINDS] = {0, 0, 0, 0, 0, 0};   // lane groups per kernel (0: from the row length)
    // systems on this level: a batched hierarchy holds several independent
    // systems, each a contiguous range of block rows (one system otherwise)
    std::vector<int> seg;           // nsys + 1 block offsets
    std::vector<int8_t> mode;       // per system: 0 no blocks left, 1 coarsened, 2 solved directly here
    DBuf<int> seg_d, lbase, bsys;   // device copy of seg; per block: first block of its system, its system
    DBuf<int8_t> mode_d, direct;    // device copy of mode; blocks of directly solved systems
    // direct solves: one dense inverse (and its transpose) per system with mode 2
    int ndseg = 0, dmax_n = 0;
    std::vector<int> dsys, dblk0, dnb;
    std::vector<int64_t> doff;
    DBuf<int> ddof0_d, dn_d, dsys_d;
    DBuf<int64_t> doff_d;
    // setup products
    DBuf<double> dinv, bnorm;
    bool bnorm_ready = false;       // bnorm came with the operator (the Galerkin step computes it)
    DBuf<uint64_t> facemeta;        // level 0: the face masks, from the same pass over A as bnorm
    DBuf<uint8_t> mask;
    DBuf<int> lambda, cidx, pmap, dround, cpts, flist;
    DBuf<int> margin;               // decision-margin audit counts (theta, phi, one-point, drop)
    DBuf<int8_t> cf;
    int nc = 0, nF = 0, rounds = 0;
    DevBSR Z;                       // R = [Z I]: nc rows, fine F columns
    int dense_n = 0;                // order of the dense inverse when one system covers the level
    DBuf<double> dense_inv, dense_invT;
    // transposed cycle (built on first use): A^T where its face copy, the
    // F-cycle's coarse residuals or small blocks need it, else A's F rows (all
    // rows with FC relaxation) and Z read transposed by their nonzero rows
    bool have_T = false;
    DevBSR AT, ZT;
    TransRows atF, zt;
    DBuf<int> ptptr, ptidx;
    // cycle vectors
    DBuf<double> r, e0, e1, tmp;
    // FP32-stored hierarchy (precision 1): operator, Z and transposes in float,
    // and the cycle vectors
    DBuf<float> vals32, z32, at32, zt32;
    DBuf<float> r32, e0_32, e1_32, tmp32;
    // F-cycle: the first coarse correction while the second is computed
    DBuf<double> fsave;
    DBuf<float> fsave32;
    // face-compressed copies of A and A^T (level 0 of a block hierarchy)
    FaceCopy face, faceT;
    // F rows of A and A^T in F-list order without their diagonal blocks, for the sweeps
    SweepCopy sweep, sweepT;
    // Z's blocks by their nonzero rows, for the restriction (levels with sweep copies)
    RowBlocks zrows;
    // bit masks of the nonzero rows of Z's and A's blocks, where the kernels
    // that form those blocks produce them (9x9 and 16x16 blocks; A below level 0)
    DBuf<uint32_t> zmask, amask;
};

// A_l (trans: A_l^T) as the cycle kernels read it: with its face-compressed
// copy where the level has one.
// The F sweeps read its sweep copy where the level has one.
inline MatView<double> op_view(const Level &L, bool trans) {
    MatView<double> v = view(trans ? L.AT : L.A);
    const FaceCopy &F = trans ? L.faceT : L.face;
    if (F.on) v.face = FaceView<double>{F.meta.get(), F.vals.get(), F.dvals.get(), F.cmax, F.rc};
    const SweepCopy &S = trans ? L.sweepT : L.sweep;
    if (S.on)
        v.sweep = SweepView<double>{S.rowptr.get(), S.colidx.get(), S.rc ? S.meta.get() : nullptr, S.vals.get(),
                                    S.dinv.get(), S.cmax, S.rc,
                                    RowBlockView<double>{S.rows.mask.get(), S.rows.off.get(), S.rows.vals.get()}};
    return v;
}
inline MatView<float> op_view32(const Level &L, bool trans) {
    MatView<float> v = view(trans ? L.AT : L.A, trans ? L.at32.get() : L.vals32.get());
    const FaceCopy &F = trans ? L.faceT : L.face;
    if (F.on) v.face = FaceView<float>{F.meta.get(), F.vals32.get(), F.dvals32.get(), F.cmax, F.rc};
    const SweepCopy &S = trans ? L.sweepT : L.sweep;
    if (S.on)
        v.sweep = SweepView<float>{S.rowptr.get(), S.colidx.get(), S.rc ? S.meta.get() : nullptr, S.vals32.get(),
                                   S.dinv.get(), S.cmax, S.rc,
                                   RowBlockView<float>{S.rows.mask.get(), S.rows.off.get(), S.rows.vals32.get()}};
    return v;
}

inline TransRowsView<double> tr_view(const TransRows &T, int bs) {
    return TransRowsView<double>{T.nrows,      bs,          T.nent,         T.nq,         T.rowptr.get(),
                                 T.colidx.get(), T.off.get(), T.mask.get(), T.qptr.get(), T.src.get(),
                                 T.vals.get(), 0};
}
inline TransRowsView<float> tr_view32(const TransRows &T, int bs) {
    return TransRowsView<float>{T.nrows,      bs,          T.nent,         T.nq,         T.rowptr.get(),
                                T.colidx.get(), T.off.get(), T.mask.get(), T.qptr.get(), T.src.get(),
                                T.vals32.get(), 0};
}

// Z as the restriction reads it: by its blocks' nonzero rows where the level keeps them.
inline MatView<double> z_view(const Level &L) {
    MatView<double> v = view(L.Z);
    if (L.zrows.on) v.rows = RowBlockView<double>{L.zrows.mask.get(), L.zrows.off.get(), L.zrows.vals.get()};
    return v;
}
inline MatView<float> z_view32(const Level &L) {
    MatView<float> v = view(L.Z, L.z32.get());
    if (L.zrows.on) v.rows = RowBlockView<float>{L.zrows.mask.get(), L.zrows.off.get(), L.zrows.vals32.get()};
    return v;
}

// Device buffers one run of the iteration works in (norm chunk tables and
// partial sums, per-system state, the history): BatchSolve's, or the no-alloc
// solve's carve of its static scratch array.
struct SolveBufs {
    int nchunk = 0, hist_cap = 0;
    int64_t *clo = nullptr;
    int *clen = nullptr, *cptr = nullptr;
    double *part = nullptr, *bn = nullptr, *last = nullptr, *rtol = nullptr, *hist = nullptr;
    int *active = nullptr, *status = nullptr, *iters = nullptr, *it = nullptr, *nact = nullptr, *nact_acc = nullptr;
};

// Per-system solve state of the batched iteration (device-side convergence).
struct BatchSolve {
    bool ready = false;
    DBuf<int64_t> clo;              // norm chunks: first dof, length, per-system chunk ranges
    DBuf<int> clen, cptr;
    int nchunk = 0;
    DBuf<double> part, bn, last, rtol;
    DBuf<double> hist;              // [nsys][hist_cap] relative residuals
    int hist_cap = 0;
    DBuf<int> active, status, iters, it, nact, nact_acc;
    double rtol_host = 0.0;
    std::vector<std::vector<double>> hist_host;
    // captured iteration (slot 0: A, slot 1: A^T), replayed per step
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    const void *key_b[2] = {nullptr, nullptr}, *key_x[2] = {nullptr, nullptr};
    ~BatchSolve();
};

// Vectors of restarted GMRES(m): the Krylov basis V (m+1 vectors), the
// preconditioned directions Z (m), the work vector w, reduction scratch and
// the device side of the Hessenberg columns.
struct Krylov {
    int m = 0;
    int64_t n = 0;
    DBuf<double> V, Z, w, part, hd, c;
};

struct Hier {
    nair_params prm{};
    int bs = 0;                     // block size of the hierarchy (1 for the scalar form)
    int device = 0;
    int nsys = 1;
    std::vector<std::unique_ptr<Level>> lv;
    // scalar form (prm.form == 1): the caller's block system, its block-diagonal
    // inverse, A0^T for the transposed residual, per-block system ids, and a
    // residual buffer; the hierarchy is built on S = D^{-1} A0
    int bs0 = 0;
    DevBSR A0, A0T;
    bool have_A0T = false;
    DBuf<double> d0inv, rres;
    DBuf<int> bsys0;
    std::vector<double> hist;
    std::string err;
    BatchSolve batch;
    Krylov krylov;
    const int *active = nullptr;    // during a batched solve: per-system "still iterating" flags
};

// nsys systems of sys_nb[s] block rows each (host array), stored one after the
// other in one BSR matrix with no block coupling two systems.
void build_hierarchy(Hier &h, int nsys, const int *sys_nb, int nb, int bs, const int *rowptr, const int *colidx,
                     const double *vals, hipStream_t s);
nair_status run_solve(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter,
                      nair_result *res, hipStream_t s);
// Every system iterated to its own relative residual; res[s] per system (host).
nair_status run_solve_batch(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter,
                            bool use_graph, nair_result *res, hipStream_t s);
void run_vcycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s);
// One system's stationary iteration A x = b in the buffers V (already carved
// and with their norm-chunk tables filled for nchunk chunks of kSolveChunk
// dofs): no device or host allocation; the history stays in V.hist.
nair_status run_solve_bufs(Hier &h, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                           hipStream_t s, const SolveBufs &V);
constexpr int kSolveChunk = 4096;   // dofs per norm chunk
// nair_solve_noalloc: the same iteration in the library's static scratch array
nair_status solve_noalloc(Hier &h, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                          hipStream_t s);
// Look up the scratch array's address on the current device (once per device).
void noalloc_prepare();
// Operators the cycle (trans: the transposed cycle) needs, built once.
void prepare_cycle(Hier &h, bool trans, hipStream_t s);
// e = B r (trans: B^T r) on the stream, no synchronisation; r and e are the
// caller's dofs (the scalar form's scaling included); prepare_cycle first.
void apply_cycle(Hier &h, bool trans, const double *r, double *e, hipStream_t s);
// Restarted GMRES(prm.gmres) right-preconditioned by the cycle (one system).
nair_status run_gmres(Hier &h, bool trans, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                      hipStream_t s);
void ensure_transposes(Hier &h, hipStream_t s);
// Time every feasible lane-group count of each cycle kernel on each level and
// keep the fastest (reps launches per candidate); table (host, may be null)
// receives [kTuneLevels][TU_KINDS].
void autotune(Hier &h, int reps, int8_t *table, hipStream_t s);
void apply_tuning(Hier &h, const int8_t *table);
void drop_graphs(Hier &h);
void make_fp32_copies(Hier &h, hipStream_t s);
// Sweep copies of A (trans: A^T) on the levels nair_params.sweep_copy selects.
void build_sweeps(Hier &h, bool trans, hipStream_t s);
void complexity(Hier &h, double *oc, double *cc, hipStream_t s);

// validation of the input pattern (device): sets *bad != 0 on error
void launch_validate(const int *rowptr, const int *colidx, int nb, int64_t nnzb, const int *seg, int nsys, int *bad,
                     hipStream_t s);

}  // namespace nair
