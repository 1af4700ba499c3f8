/*
 * nair.h -- C ABI of the MI355X (gfx950) nAIR library.
 *
 * nAIR: reduction-based algebraic multigrid with Neumann approximate ideal
 * restriction, for block lower triangular (in an unknown order) systems such
 * as upwind discontinuous-Galerkin discretisations of steady transport
 * (Manteuffel, Muenzenmaier, Ruge, Southworth, "Nonsymmetric Reduction-based
 * Algebraic Multigrid"; problem statement in sections 1 and 2.1, method in
 * sections 4.1 and 5).
 *
 * Conventions for every entry point:
 *   - Matrices are block CSR ("BSR"): nb block rows of bs x bs blocks,
 *     rowptr[nb+1] and colidx[nnzb] (int32, column indices sorted ascending
 *     and unique within a row, diagonal block present in every row), vals
 *     [nnzb][bs][bs] double, each block row-major.
 *   - Array arguments are DEVICE pointers (memory on the current HIP device),
 *     unless the comment says "host".  The caller owns them; the library
 *     never frees or keeps them past the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; every call returns only when its device
 *     work is complete, so outputs may be read right after the call.
 *   - Errors are return codes; no exception crosses the ABI.  After an error
 *     the handle (if any) stays valid; nair_last_error gives a message.
 *   - The library runs one call at a time: calls from several host threads
 *     must be serialised by the caller (temporary device memory is reused in
 *     stream order).
 */
#ifndef NAIR_H
#define NAIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NAIR_OK = 0,
    NAIR_EINVAL = 1,      /* bad sizes/parameters, unsorted/duplicate columns, missing diagonal */
    NAIR_ESINGULAR = 2,   /* a diagonal block (or the coarsest operator) has a zero pivot */
    NAIR_ENOCONV = 3,     /* max_iter reached; output holds the last iterate */
    NAIR_ENUMERIC = 4,    /* a residual norm is not finite */
    NAIR_ENOMEM = 5,      /* device allocation failed, or a row exceeds the kernels' limits */
    NAIR_EDEVICE = 6,     /* a HIP runtime call failed */
    NAIR_ECOARSEN = 7     /* the splitting stalled on a level too large to solve densely */
} nair_status;

typedef struct nair_hier_s *nair_hier;

/*
 * Device memory from the caller (for instance torch's caching allocator), in
 * place of the library's own caching pool.  alloc returns `bytes` of device
 * memory on the handle's device for use on `stream` (the stream of the call
 * that needs it), or NULL on failure (the call then returns NAIR_ENOMEM);
 * free returns a block alloc gave.  Every device buffer of a handle set up with
 * it -- the hierarchy, its copies, the solve's vectors and temporaries -- comes
 * from it, during nair_setup and during later calls on the handle, and goes
 * back to it by nair_destroy at the latest.  The struct is copied at setup;
 * alloc, free and ctx must stay valid until nair_destroy returns.
 */
typedef struct nair_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} nair_allocator;

/* Setup parameters (section 5.1 and 5.2 of the paper for the defaults). */
typedef struct {
    int32_t degree;           /* Neumann degree k >= 0 of the restriction (section 4.1);
                                 the F-relaxation does nu = k+1 Jacobi sweeps (section 5.1) */
    double theta;             /* strength threshold of the C/F splitting, in [0,1): 0.75 */
    double phi;               /* strength threshold of the Neumann expansion, in [0,1): 0.025 */
    double drop;              /* drop tolerance of coarse operators, in [0,1): 1e-3 (section 5.2) */
    int32_t relax;            /* 0: F-relaxation; 1: F then one C sweep (FC) */
    int32_t max_levels;       /* 1..64, default 30 */
    int32_t max_coarse_dofs;  /* a level with nb*bs <= this is solved densely; default 128 */
    uint64_t seed;            /* seed of the splitting's tie-break hash, default 0 */
    const int8_t *cf_override_host; /* optional, host, [nb] level-0 splitting (1 = C, 0 = F) */
    int32_t precision;        /* 0: FP64 cycle; 1: FP32-stored hierarchy (operators, Z and cycle
                                 vectors in float; FP64 block inverses, accumulation, outer
                                 residual and update: FP64 iterative refinement).  The setup and
                                 its decisions are FP64 either way. */
    const int8_t *tuning;     /* optional, host, [64][6] lane-group choices from nair_autotune for a
                                 hierarchy of the same structure (copied at setup); NULL: defaults */
    int32_t form;             /* 0: block nAIR (default); 1: scalar nAIR of the system scaled by the
                                 inverse of its block diagonal (section "Blocks, filtering, and
                                 parallelization"): the hierarchy is built on S = D^{-1} A as a
                                 scalar matrix (identity diagonal blocks exact, zeros dropped) and
                                 the solve preconditions A with B_S D^{-1} (transposed: D^{-T}
                                 B_S^T), stopping on the unscaled residual.  Levels are scalar. */
    int32_t cycle;            /* 0: V-cycle (default); 1: F-cycle -- every coarse solve is an F-cycle
                                 followed by a V-cycle on its residual (the F-cycles of the section
                                 "Scaling in h and element order"); the transposed solve applies the
                                 exact transpose */
    int32_t gmres;            /* 0: stationary iteration (default); m in [1, 200]: restarted GMRES(m)
                                 right-preconditioned by one cycle per iteration (the section "Non-
                                 triangular matrices" uses one nAIR V-cycle as a GMRES
                                 preconditioner).  The Arnoldi basis is orthogonalised by classical
                                 Gram-Schmidt applied twice (equal to modified Gram-Schmidt in exact
                                 arithmetic), the least-squares problem by Givens rotations; each
                                 restart starts from the true residual.  Iteration j's history entry
                                 is the least-squares estimate |g_{j+1}| / ||b|| of the relative
                                 residual.  Single-system handles only (nair_solve_batch returns
                                 NAIR_EINVAL); takes (2m + 2) n extra doubles on the first solve. */
    int32_t faces;            /* 1 (default): when the finest operator's off-diagonal blocks are
                                 nonzero only on a few rows and columns (upwind DG face blocks: the
                                 two elements' face nodes), keep a compact copy of them (masks of the
                                 nonzero rows and columns and the dense rectangle they span, diagonal
                                 blocks whole) and let the cycle's sweeps and residuals read that;
                                 used when the rectangles hold at most half a block.  Only exact
                                 zeros are left out: results are bit-identical to faces = 0 for
                                 finite vectors.  Block form only. */
    int32_t sweep_copy;       /* -1 (default): levels whose sweeps occupy at least 32768 lanes (block
                                 rows x bs) keep a second copy of their F rows, in F-list order and
                                 without the diagonal blocks, with D_F^{-1} in the same order (and
                                 the same for A^T once a transposed solve needs it), and the Jacobi
                                 F sweeps read that contiguously; 0: no copies; 1: every level that
                                 relaxes.  The sweep computes D_I^{-1}(r_I - sum_{J != I} A_IJ e_J)
                                 either way; with one lane group per row (nair_params.tuning) the
                                 results are bit-identical with and without copies.  Costs about
                                 the F rows' share of each selected operator in memory. */
    int32_t matrix_cores;     /* 1 (default): the setup's dense block products (Neumann products,
                                 T = -D^-1 A_ff, Z = -S D^-1 and the Galerkin blocks) of 9x9, 16x16
                                 and 25x25 blocks run on the FP64 matrix cores; 0: on the vector
                                 units.  Both evaluate every entry as the fma chain over the inner
                                 index in ascending order, so the hierarchies are identical (a zero
                                 may differ in sign); 0 is the reference for that check. */
    const nair_allocator *allocator; /* optional, host: device memory from the caller (copied at
                                 setup); NULL (default): the library's caching pool */
} nair_params;

typedef struct {
    int32_t iters;            /* iterations done */
    int32_t converged;        /* 1 if ||b - A x||_2 / ||b||_2 <= rtol */
    double relres;            /* final relative residual */
    double rho_avg;           /* relres^(1/iters) */
    double rho_last5;         /* (h_K / h_{K-5})^(1/5), or rho_avg if iters <= 5 */
} nair_result;

/* Device views of one level, for inspection and parity checks.  Pointers stay
 * valid until nair_destroy.  Arrays a level does not have are NULL. */
typedef struct {
    int32_t nb, bs, nnzb, coarsest;
    const int32_t *rowptr, *colidx;
    const double *vals;       /* A_l, [nnzb][bs][bs] */
    const double *dinv;       /* [nb][bs][bs] inverses of the diagonal blocks */
    const double *bnorm;      /* [nnzb] max-abs size of each block */
    const uint8_t *mask;      /* [nnzb] bit 0: theta-strong, bit 1: phi-strong */
    const int32_t *lambda;    /* [nb] number of rows depending theta-strongly on each block */
    const int8_t *cf;         /* [nb] 1 = C, 0 = F */
    const int32_t *cidx;      /* [nb] coarse index of C blocks, -1 for F */
    const int32_t *pmap;      /* [nb] one-point interpolation source (coarse index) or -1 */
    const int32_t *dround;    /* [nb] splitting round that decided each block (0 = start) */
    int32_t nc;               /* number of C blocks */
    int32_t pmis_rounds;
    int32_t z_nnzb;
    const int32_t *z_rowptr, *z_colidx;  /* Z of R = [Z I]: nc rows, fine F columns */
    const double *z_vals;
    int32_t dense_n;          /* one system solved directly on this level: order of its dense operator */
    const double *dense_inv;  /* dense inverses of the systems solved directly on this level, row-major,
                                 each at its offset from nair_get_systems ([dense_n][dense_n] for one) */
    int32_t face_rmax, face_cmax;  /* face-compressed copy (nair_params.faces), else 0 and NULL: */
    const uint64_t *face_meta;     /* [nnzb] nonzero rows (bits 0..31), columns (bits 32..63); 0 on
                                      diagonal blocks */
    const double *face_vals;       /* [nnzb][rmax][cmax] entries on those rows x columns, ascending */
    const double *face_dvals;      /* [nb][bs][bs] diagonal blocks by columns: entry (a, c) at c * bs + a */
    int32_t margin[4];             /* decision-margin audit (host copy): comparisons whose two sides lie
                                      within 1e-12 relative in the theta and phi strength tests, F rows
                                      whose one-point choice has a rival that close, and drop tests of
                                      the coarse operator built from this level.  Setup decisions are
                                      bit-exact with the reference arithmetic either way; the counts
                                      show how close they came to flipping.  A batch counts the rows of
                                      systems solved directly on the level too. */
    int32_t sweep_nnzb;            /* blocks held by the level's sweep copy of A (nair_params.sweep_copy),
                                      -1 when its F sweeps read A itself */
} nair_level_view;

/* Fill *p with the defaults (degree 1, theta 0.75, phi 0.025, drop 1e-3, F
 * relaxation, 30 levels, 128 dense DOFs, seed 0, FP64 cycle).  Host only. */
nair_status nair_default_params(nair_params *p);

/*
 * Build the nAIR hierarchy of A (sections 2.2, 4.1, 5.1, 5.2): per level,
 * block-diagonal inverses by batched LU, strength and a seeded parallel C/F
 * splitting, one-point interpolation, the degree-k Neumann restriction
 * Z = -A_cf sum_{i<=k} (D_ff^-1 L_ff)^i D_ff^-1 on phi-strong F-F blocks, and
 * the filtered Galerkin operator K = R A P; the coarsest level is inverted
 * densely.  A is copied; the caller may free it on return.  *out receives
 * the handle (NULL on error).
 */
nair_status nair_setup(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx,
                       const double *vals, const nair_params *p, void *stream, nair_hier *out);

/*
 * One hierarchy for nsys independent systems (many discrete-ordinate angles of
 * the transport problem, each its own block triangular system; the paper's
 * introduction and numerical results motivate the method by such sweeps).
 * System k owns block rows [o_k, o_k + sys_nb[k]) with o_k = sum_{j<k}
 * sys_nb[j]; rowptr/colidx/vals hold them one after another in one BSR
 * (global column indices; a block coupling two systems is NAIR_EINVAL).
 * Every system gets exactly the hierarchy nair_setup would build for it alone
 * (splitting hashes use indices within the system); a system at its coarsest
 * size is inverted densely on that level while the others keep coarsening.
 * sys_nb is host memory (every entry >= 1).  Solve with nair_solve_batch;
 * nair_vcycle / nair_vcycle_T apply all systems' cycles at once.
 */
nair_status nair_setup_batch(int32_t nsys, const int32_t *sys_nb, int32_t bs, const int32_t *rowptr,
                             const int32_t *colidx, const double *vals, const nair_params *p, void *stream,
                             nair_hier *out);

/*
 * Solve A x = b by the stationary iteration x += B (b - A x), x_0 = 0, with B
 * one V-cycle (no pre-relaxation, section 5), until ||b - A x||_2 / ||b||_2 <=
 * rtol or max_iter iterations.  b and x are device vectors of nb*bs doubles;
 * x is overwritten.  res (host, may be NULL) receives the statistics.
 * Returns NAIR_OK, NAIR_ENOCONV (x = last iterate) or NAIR_ENUMERIC.  With
 * nair_params.gmres = m > 0 the iteration is GMRES(m) preconditioned by the
 * cycle instead; it stops when the least-squares estimate reaches rtol and
 * reports NAIR_OK if the estimate or the true residual of x is within rtol.
 */
nair_status nair_solve(nair_hier h, const double *b, double *x, double rtol, int32_t max_iter,
                       nair_result *res, void *stream);

/*
 * Solve A^T y = g with the transposed cycle B^T: pre-relaxation with D^-T on
 * F points, restriction by P^T and interpolation by R^T (the ideal
 * interpolation dual of the paper's section 2.2 corollary).  The transposed
 * operators are built on the first call.
 */
nair_status nair_solve_T(nair_hier h, const double *g, double *y, double rtol, int32_t max_iter,
                         nair_result *res, void *stream);

/*
 * Solve every system of a handle (batched or not) to its own relative residual:
 * A x = b (trans = 0) or A^T x = b (trans = 1), the same stationary iteration
 * as nair_solve / nair_solve_T, with each system's norm, convergence test and
 * history kept on the device; a converged system's x stops changing.  With
 * use_graph != 0 one iteration of all systems is captured once into a HIP
 * graph (per operand pair) and replayed; the host only checks the number of
 * systems still iterating every few iterations.  b, x: device vectors of all
 * systems' dofs one after another.  res (host, may be NULL) gets nsys results.
 * Returns NAIR_OK when every system converged, else NAIR_ENUMERIC if any
 * residual turned non-finite, else NAIR_ENOCONV.  nair_solve and nair_solve_T
 * reject handles with more than one system.
 */
nair_status nair_solve_batch(nair_hier h, int32_t trans, const double *b, double *x, double rtol,
                             int32_t max_iter, int32_t use_graph, nair_result *res, void *stream);

/* Relative residual history of system sys in the last nair_solve_batch (host buf, min(cap, n)). */
nair_status nair_batch_history(nair_hier h, int32_t sys, double *buf, int32_t cap, int32_t *n);

/*
 * The systems on level lvl (host outputs, each may be NULL; cap = entries the
 * arrays hold, at least nsys, seg one more): seg = block offsets of each system
 * on this level, mode = 0 (no blocks left), 1 (coarsened here), 2 (solved
 * directly here), dense_off = offset of its dense inverse in the level view's
 * dense_inv (-1 unless mode 2).
 */
nair_status nair_get_systems(nair_hier h, int32_t lvl, int32_t cap, int32_t *nsys, int32_t *seg, int8_t *mode,
                             int64_t *dense_off);

/*
 * Autotune the cycle kernels of this hierarchy: every cycle kernel maps a block
 * row onto G groups of bs lanes; for each level and each kernel (0 Jacobi
 * sweep with A, 1 with A^T, 2 transposed residual, 3 restriction, 4 transposed
 * interpolation, 5 outer residual) each power of two G with G*bs <= 256 is
 * timed over reps launches on the level's own operands and the fastest kept
 * (it must beat the row-length default by 3%).  Results do not change: only
 * the launch shape does.  table (host, may be NULL) receives [64][6] choices
 * (0 = default) that nair_params.tuning applies to later hierarchies of the
 * same structure.  Builds the transposed operators.
 */
nair_status nair_autotune(nair_hier h, int32_t reps, int8_t *table, void *stream);

/* One cycle application e = B r (resp. y = B^T g), zero initial guess. */
nair_status nair_vcycle(nair_hier h, const double *r, double *e, void *stream);
nair_status nair_vcycle_T(nair_hier h, const double *g, double *y, void *stream);

/*
 * Gradient of a solve with respect to the matrix entries, on A's block pattern:
 * for x = A^{-1} b and ybar = A^{-T} xbar (the adjoint solve, nair_solve_T),
 * dL/dA_IJ = -ybar_I x_J^T for every stored block (I,J).  rowptr/colidx are the
 * pattern (as for nair_setup); ybar and x are device vectors of nb*bs doubles;
 * grad_vals (device, [nnzb][bs][bs]) is written.  Needs no handle.
 */
nair_status nair_grad_vals(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx,
                           const double *ybar, const double *x, double *grad_vals, void *stream);

#define NAIR_NOALLOC_SCRATCH_BYTES 4194304
/*
 * nair_solve for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * stationary iteration and the same results as nair_solve on a single-system
 * handle with gmres = 0 (else NAIR_EINVAL), but every buffer the iteration
 * needs beyond the handle (allocated by nair_setup), b and x --
 * norm partial sums and their chunk tables, per-system state, the residual
 * history -- lives in one static device array of NAIR_NOALLOC_SCRATCH_BYTES
 * (4 MiB) per device, held until the process ends.  It calls no hipMalloc,
 * hipFree or allocating routine.  A solve of n dofs with max_iter iterations
 * needs about 2.5 ceil(n / 4096) + max_iter + 8 doubles of it (a solve of
 * 850 million dofs at 200 iterations fits); larger ones return NAIR_EINVAL
 * with the sizes in nair_last_error.  Every call on a device shares that
 * device's array: calls that overlap on one device race (serialise them).
 * The history of this solve is not kept: nair_history reports none after it.
 * It synchronises the stream to read its convergence counters, as nair_solve
 * does, and the kernel timer does not see its launches.
 */
nair_status nair_solve_noalloc(nair_hier h, const double *b, double *x, double rtol, int32_t max_iter,
                               nair_result *res, void *stream);

/* Relative residual history of the last solve: buf (host) gets min(cap, n). */
nair_status nair_history(nair_hier h, double *buf, int32_t cap, int32_t *n);

/* Hierarchy statistics (host outputs; per-level arrays hold up to 64 entries;
 * any pointer may be NULL).  oc/cc: operator and cycle complexity in work
 * units of one level-0 SpMV (section 6). */
nair_status nair_info(nair_hier h, int32_t *levels, int32_t *nb_per_level, int64_t *nnzb_per_level,
                      double *oc, double *cc);

/* Device views of level lvl (0 = finest). */
nair_status nair_get_level(nair_hier h, int32_t lvl, nair_level_view *v);

/* Last error message of h (or of the last failed setup if h is NULL). Host string. */
const char *nair_last_error(nair_hier h);

/* Free the hierarchy (its memory returns to the library's device pool). */
void nair_destroy(nair_hier h);

/* Return all cached, unused device memory of the pool to HIP. */
nair_status nair_pool_trim(void);

/*
 * Kernel timer (profiling).  nair_timer_select(kernel, level) makes the
 * library bracket every later launch of that kernel on that level (-1: all
 * levels) with a pair of HIP events on the launch's stream (the F sweeps of
 * one cycle visit run back to back and are bracketed as one group);
 * kernel = -1 turns the timer off.  Kernels: 0 Jacobi F sweep over
 * the F-row list (both cycles; the FC C sweep and the transposed cycle's first
 * sweep from zero, which reads no matrix, are not timed), 1 outer residual,
 * 2 restriction, 3 interpolation, 4 SpGEMM numeric, 5 SpGEMM symbolic,
 * 6 block inverse,
 * 7 Galerkin blocks (with the R A products where they are fused), 8 dense
 * coarsest product, 9 single block products of the setup (T, Z).  nair_timer_read (host outputs)
 * synchronises the device and returns the number of timed launches and their
 * total duration in milliseconds, then resets the counters.  Host only; one
 * timed kernel at a time.
 */
nair_status nair_timer_select(int32_t kernel, int32_t level);
nair_status nair_timer_read(int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif
