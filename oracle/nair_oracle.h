/*
 * nair_oracle.h -- plain single-threaded CPU oracle for nAIR (test infrastructure).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the tests,
 * the smoke check and the bench's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * It implements, step by step and in the paper's order, the nAIR hierarchy
 * build and V-cycle of "Nonsymmetric Reduction-based Algebraic Multigrid"
 * (Manteuffel, Muenzenmaier, Ruge, Southworth):
 *   - 2x2 block reduction form A = [A_ff A_fc; A_cf A_cc], P = [W; I],
 *     R = [Z I], coarse operator K = R A P   (section 2.2, eqs. "block", "rap")
 *   - Neumann approximate ideal restriction, degree k, on strong F-F
 *     connections                           (section 4.1, eq. "neumann")
 *   - strength |a_ij| >= phi * sup_j |a_ij|  (section 4.2, 4.1)
 *   - Jacobi F-relaxation with k+1 sweeps, no pre-relaxation, one-point
 *     interpolation                          (section 5.1)
 *   - block nAIR and the drop filter         (section 5.2)
 *   - C-point relaxation option              (section 3.1, remark "C-point relaxation")
 * with the readings the paper leaves open stated at each function.
 *
 * All arrays are host arrays.  Status codes are the oracle's own.
 */
#ifndef NAIR_ORACLE_H
#define NAIR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORA_OK = 0,
    ORA_EINVAL = 1,
    ORA_ESINGULAR = 2,
    ORA_ENOCONV = 3,
    ORA_ENUMERIC = 4,
    ORA_ENOMEM = 5,
    ORA_ECOARSEN = 7
};

typedef struct {
    int32_t degree;           /* Neumann degree k >= 0; nu = k+1 Jacobi F sweeps */
    double theta;             /* strength threshold for splitting (default 0.75) */
    double phi;               /* strength threshold of the Neumann mask (0.025) */
    double drop;              /* coarse-operator drop tolerance (1e-3) */
    int32_t relax;            /* 0: F-relaxation, 1: F then one C sweep (FC) */
    int32_t max_levels;       /* maximum number of levels */
    int32_t max_coarse_dofs;  /* dense LU once nb*bs <= this */
    uint64_t seed;            /* seed of the independent-set tie-break hash */
    const int8_t *cf_override;/* optional level-0 splitting (1 = C, 0 = F), NULL = computed */
    int32_t form;             /* 0: block nAIR; 1: scalar nAIR of the system scaled by the
                                 block-diagonal inverse (the paper's default form) */
    int32_t cycle;            /* 0: V-cycle; 1: F-cycle (section "Scaling in h and element order") */
    int32_t gmres;            /* 0: stationary iteration; m > 0: right-preconditioned GMRES(m)
                                 with the cycle as preconditioner (the paper's "nAIR-preconditioned
                                 GMRES") */
} ora_params;

/* A view of one level, valid until ora_free.  Arrays that do not exist on a
 * level (everything but A and the dense factors on the coarsest) are NULL. */
typedef struct {
    int32_t nb, bs, nnzb, coarsest;
    const int32_t *rowptr, *colidx;
    const double *vals;          /* [nnzb][bs][bs] */
    const double *dinv;          /* [nb][bs][bs] */
    const double *bnorm;         /* [nnzb] max-abs norm of each block */
    const uint8_t *mask;         /* [nnzb] bit0: theta-strong, bit1: phi-strong */
    const int32_t *lambda;       /* [nb] number of rows strongly depending on each block */
    const int8_t *cf;            /* [nb] 1 = C, 0 = F */
    const int32_t *cidx;         /* [nb] rank among C points, -1 for F */
    const int32_t *pmap;         /* [nb] coarse index each block interpolates from, -1 none */
    int32_t nc;                  /* number of C blocks */
    int32_t pmis_rounds;
    const int32_t *dround;       /* [nb] splitting round that decided each block, 0 = start */
    int32_t z_nnzb;
    const int32_t *z_rowptr, *z_colidx;   /* Z: nc rows, fine F columns */
    const double *z_vals;
    int32_t dense_n;             /* coarsest: dense order nb*bs */
    const double *dense_lu;      /* coarsest: LU factors with partial pivoting, row-major */
    const int32_t *dense_piv;
    int64_t margin[4];           /* decision-margin audit: comparisons within 1e-12 relative in the
                                    theta and phi strength tests, one-point choices with a rival
                                    candidate that close, and the drop test of the coarse operator
                                    built from this level */
} ora_level_view;

typedef struct ora_hier ora_hier;

void ora_default_params(ora_params *p);

/* Build the hierarchy.  A is copied.  Returns ORA_OK or an error code. */
int ora_setup(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx,
              const double *vals, const ora_params *p, ora_hier **out);

/* Stationary nAIR iteration x_{j+1} = x_j + B (b - A x_j) from x_0 = 0 until
 * ||b - A x||_2 / ||b||_2 <= rtol.  hist (may be NULL) receives one relative
 * residual per iteration (capacity max_iter).  Returns ORA_OK, ORA_ENOCONV or
 * ORA_ENUMERIC; *iters is the number of iterations done. */
int ora_solve(ora_hier *h, const double *b, double *x, double rtol, int32_t max_iter,
              double *hist, int32_t *iters, double *relres);
/* The same for A^T y = g with the transposed cycle B^T. */
int ora_solve_T(ora_hier *h, const double *g, double *y, double rtol, int32_t max_iter,
                double *hist, int32_t *iters, double *relres);

/* One application of the cycle operator: e = B r, and y = B^T g. */
int ora_vcycle(ora_hier *h, const double *r, double *e);
int ora_vcycle_T(ora_hier *h, const double *g, double *y);

int32_t ora_num_levels(const ora_hier *h);
int ora_level(const ora_hier *h, int32_t lvl, ora_level_view *v);

/* Operator and cycle complexity (work units of one level-0 SpMV). */
void ora_complexity(const ora_hier *h, double *oc, double *cc);

/* Inverse of one bs x bs block by the LU recipe used for every diagonal block.
 * Returns ORA_OK or ORA_ESINGULAR. */
int ora_block_inverse(int32_t bs, const double *m, double *inv);

/* The splitmix64 finaliser used for the splitting's tie-break keys. */
uint64_t ora_splitmix64(uint64_t x);

void ora_free(ora_hier *h);

#ifdef __cplusplus
}
#endif
#endif
