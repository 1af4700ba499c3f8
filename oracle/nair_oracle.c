/*
 * nair_oracle.c -- plain single-threaded CPU oracle for nAIR.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * bench's CPU-baseline leg; never by the product path.  It shares no code with
 * the HIP library.  Build: gcc -O2 -ffp-contract=off -shared -fPIC (fma() from
 * libm is correctly rounded, and no multiply-add is contracted implicitly).
 *
 * Arithmetic order.  Every value that later feeds a comparison (block
 * inverses, the Neumann terms, Z, R A and the coarse operator) is computed in
 * one fixed order, stated at each function:
 *   - a block product  acc[a][b] = fma(X[a][c], Y[c][b], acc[a][b]), c ascending;
 *   - a sparse product sums its contributions in ascending order of the inner
 *     block index K, each contribution being the c-ascending chain above, all
 *     in one accumulator per entry starting from +0;
 *   - identity blocks are added plainly, sums of matrices go left to right.
 * Solve-phase arithmetic has no such constraint.
 */
#include "nair_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAX_LEVELS 64
/* If the splitting stalls (no C points, or all C), a level this small is
 * solved densely; a larger one is an error. */
#define ORA_STALL_DENSE_DOFS 4096

typedef struct {
    int32_t nb, bs, ncols;      /* ncols: number of block columns */
    int32_t *rowptr, *colidx;
    double *vals;
} bsr_t;

typedef struct {
    bsr_t A;
    int coarsest;
    double *dinv, *bnorm;
    uint8_t *mask;
    int32_t *lambda;
    int8_t *cf;
    int32_t *cidx, *pmap, *cpts;   /* cpts[i]: fine index of the i-th C block */
    int32_t *dround;               /* splitting round that decided each block (0: start) */
    int32_t nc, pmis_rounds;
    bsr_t Z;
    int32_t dense_n;
    double *lu;
    int32_t *piv;
    /* decision-margin audit: comparisons whose two sides lie within 1e-12
     * relative (theta strength, phi strength, one-point choice, drop filter of
     * the coarse operator built from this level) */
    int64_t margin[4];
} level_t;

/* The two sides of a comparison are within 1e-12 of each other, relative to
 * the larger (both zero counts as a tie). */
static int near_tie(double a, double b) {
    return fabs(a - b) <= 1e-12 * fmax(fabs(a), fabs(b));
}

struct ora_hier {
    ora_params prm;
    int32_t nlev;
    level_t lv[ORA_MAX_LEVELS];
    /* scalar form: the caller's block system and its block-diagonal inverse */
    bsr_t A0;
    double *d0inv;
};

/* ------------------------------------------------------------------ utils */

static void *xcalloc(size_t n, size_t sz) {
    if (n == 0) n = 1;
    return calloc(n, sz);
}

static void bsr_free(bsr_t *m) {
    free(m->rowptr);
    free(m->colidx);
    free(m->vals);
    memset(m, 0, sizeof(*m));
}

static int bsr_alloc(bsr_t *m, int32_t nb, int32_t ncols, int32_t bs, int64_t nnzb) {
    m->nb = nb;
    m->ncols = ncols;
    m->bs = bs;
    m->rowptr = (int32_t *)xcalloc((size_t)nb + 1, sizeof(int32_t));
    m->colidx = (int32_t *)xcalloc((size_t)nnzb, sizeof(int32_t));
    m->vals = (double *)xcalloc((size_t)nnzb * bs * bs, sizeof(double));
    return (m->rowptr && m->colidx && m->vals) ? ORA_OK : ORA_ENOMEM;
}

static double block_maxabs(int32_t bs, const double *blk) {
    double m = 0.0;
    for (int32_t e = 0; e < bs * bs; ++e) {
        double v = fabs(blk[e]);
        if (v > m) m = v;
    }
    return m;
}

/* out = X * Y for bs x bs blocks: out[a][b] = fma chain over c ascending from +0. */
static void block_mul(int32_t bs, const double *X, const double *Y, double *out) {
    for (int32_t a = 0; a < bs; ++a)
        for (int32_t b = 0; b < bs; ++b) {
            double acc = 0.0;
            for (int32_t c = 0; c < bs; ++c) acc = fma(X[a * bs + c], Y[c * bs + b], acc);
            out[a * bs + b] = acc;
        }
}

/* acc += X * Y, continuing each entry's fma chain (c ascending). */
static void block_mul_acc(int32_t bs, const double *X, const double *Y, double *acc) {
    for (int32_t a = 0; a < bs; ++a)
        for (int32_t b = 0; b < bs; ++b) {
            double s = acc[a * bs + b];
            for (int32_t c = 0; c < bs; ++c) s = fma(X[a * bs + c], Y[c * bs + b], s);
            acc[a * bs + b] = s;
        }
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------- block inverse */

/*
 * Inverse of one diagonal block (block nAIR inverts the diagonal blocks
 * directly, section 5.2).  Recipe: LU with partial pivoting -- pivot = first
 * row i >= k with the largest |M_ik|, whole rows swapped; multipliers
 * M_ik /= M_kk; trailing update M_ij = fma(-M_ik, M_kj, M_ij) -- then each
 * column j of the inverse by forward substitution of P e_j with the unit lower
 * factor (fma over m ascending) and back substitution with U (fma over m > i
 * ascending, then one division by U_ii).
 */
int ora_block_inverse(int32_t bs, const double *m, double *inv) {
    double *a = (double *)malloc(sizeof(double) * bs * bs);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * bs);
    double *y = (double *)malloc(sizeof(double) * bs);
    int st = ORA_OK;
    memcpy(a, m, sizeof(double) * bs * bs);
    for (int32_t i = 0; i < bs; ++i) perm[i] = i;
    for (int32_t k = 0; k < bs && st == ORA_OK; ++k) {
        int32_t p = k;
        double best = fabs(a[k * bs + k]);
        for (int32_t i = k + 1; i < bs; ++i)
            if (fabs(a[i * bs + k]) > best) {
                best = fabs(a[i * bs + k]);
                p = i;
            }
        if (!(best > 0.0)) {
            st = ORA_ESINGULAR;
            break;
        }
        if (p != k) {
            for (int32_t j = 0; j < bs; ++j) {
                double t = a[k * bs + j];
                a[k * bs + j] = a[p * bs + j];
                a[p * bs + j] = t;
            }
            int32_t t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
        for (int32_t i = k + 1; i < bs; ++i) a[i * bs + k] = a[i * bs + k] / a[k * bs + k];
        for (int32_t i = k + 1; i < bs; ++i)
            for (int32_t j = k + 1; j < bs; ++j)
                a[i * bs + j] = fma(-a[i * bs + k], a[k * bs + j], a[i * bs + j]);
    }
    if (st == ORA_OK) {
        for (int32_t j = 0; j < bs; ++j) {
            for (int32_t i = 0; i < bs; ++i) y[i] = (perm[i] == j) ? 1.0 : 0.0;
            for (int32_t i = 0; i < bs; ++i)
                for (int32_t mm = 0; mm < i; ++mm) y[i] = fma(-a[i * bs + mm], y[mm], y[i]);
            for (int32_t i = bs - 1; i >= 0; --i) {
                double s = y[i];
                for (int32_t mm = i + 1; mm < bs; ++mm) s = fma(-a[i * bs + mm], y[mm], s);
                y[i] = s / a[i * bs + i];
            }
            for (int32_t i = 0; i < bs; ++i) inv[i * bs + j] = y[i];
        }
    }
    free(a);
    free(perm);
    free(y);
    return st;
}

/* ----------------------------------------------------------- strength */

/*
 * Strength of connection (sections 4.1 and 4.2): a_ij is strong when
 * |a_ij| >= phi * sup_j |a_ij|.  Block reading: the size of a block is its
 * max-abs entry; the supremum runs over the off-diagonal blocks of the row;
 * a row whose off-diagonal blocks are all zero has no strong connection.
 * Two thresholds: theta (splitting, one-point candidates are not masked) and
 * phi (the Neumann mask).  lambda_J counts the rows that depend strongly
 * (theta) on J.
 */
static void strength(level_t *L, double theta, double phi) {
    const bsr_t *A = &L->A;
    int32_t bs = A->bs;
    for (int32_t I = 0; I < A->nb; ++I) {
        double m = 0.0;
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
            L->bnorm[t] = block_maxabs(bs, A->vals + (size_t)t * bs * bs);
            if (A->colidx[t] != I && L->bnorm[t] > m) m = L->bnorm[t];
        }
        double thr_theta = theta * m, thr_phi = phi * m;
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
            uint8_t mk = 0;
            if (A->colidx[t] != I && m > 0.0) {
                if (L->bnorm[t] >= thr_theta) mk |= 1;
                if (L->bnorm[t] >= thr_phi) mk |= 2;
                L->margin[0] += near_tie(L->bnorm[t], thr_theta);
                L->margin[1] += near_tie(L->bnorm[t], thr_phi);
            }
            L->mask[t] = mk;
            if (mk & 1) L->lambda[A->colidx[t]] += 1;
        }
    }
}

/* -------------------------------------------------------- C/F splitting */

/* splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014), written from its
 * published definition. */
uint64_t ora_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* key(I) = (lambda_I, hash_I, I), compared lexicographically. */
static int key_greater(const int32_t *lambda, const uint64_t *hash, int32_t I, int32_t J) {
    if (lambda[I] != lambda[J]) return lambda[I] > lambda[J];
    if (hash[I] != hash[J]) return hash[I] > hash[J];
    return I > J;
}

/*
 * C/F splitting.  The paper uses the classical first-pass splitting (section
 * 5.1), which is sequential.  This is the parallel reading: independent-set
 * rounds on the symmetrised theta-strong graph G = S u S^T.
 *   start : blocks with lambda = 0 are F, the rest undecided;
 *   round : reading only the previous round's state, an undecided block whose
 *           key exceeds the key of every undecided G-neighbour becomes C; then
 *           every undecided block that depends strongly on a new C becomes F.
 * Repeats until no block is undecided.
 */
static int split_cf(level_t *L, int32_t lvl, uint64_t seed) {
    const bsr_t *A = &L->A;
    int32_t nb = A->nb;
    int32_t *tptr = (int32_t *)xcalloc((size_t)nb + 1, sizeof(int32_t));
    int32_t *tidx = (int32_t *)xcalloc((size_t)A->rowptr[nb], sizeof(int32_t));
    int32_t *fill = (int32_t *)xcalloc((size_t)nb, sizeof(int32_t));
    uint64_t *hash = (uint64_t *)xcalloc((size_t)nb, sizeof(uint64_t));
    int8_t *state = (int8_t *)xcalloc((size_t)nb, 1);
    int8_t *newc = (int8_t *)xcalloc((size_t)nb, 1);
    if (!tptr || !tidx || !fill || !hash || !state || !newc) return ORA_ENOMEM;
    /* transpose of the theta-strong graph: rows I that depend strongly on J */
    for (int32_t I = 0; I < nb; ++I)
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
            if (L->mask[t] & 1) tptr[A->colidx[t] + 1] += 1;
    for (int32_t J = 0; J < nb; ++J) tptr[J + 1] += tptr[J];
    for (int32_t I = 0; I < nb; ++I)
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
            if (L->mask[t] & 1) {
                int32_t J = A->colidx[t];
                tidx[tptr[J] + fill[J]++] = I;
            }
    for (int32_t I = 0; I < nb; ++I)
        hash[I] = ora_splitmix64(seed ^ ((uint64_t)lvl << 40) ^ (uint64_t)I);
    const int8_t UND = -1, FPT = 0, CPT = 1;
    int32_t undecided = 0;
    for (int32_t I = 0; I < nb; ++I) {
        state[I] = (L->lambda[I] == 0) ? FPT : UND;
        L->dround[I] = 0;
        if (state[I] == UND) undecided++;
    }
    int32_t rounds = 0;
    while (undecided > 0) {
        rounds++;
        for (int32_t I = 0; I < nb; ++I) {
            newc[I] = 0;
            if (state[I] != UND) continue;
            int is_max = 1;
            for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1] && is_max; ++t) {
                int32_t J = A->colidx[t];
                if ((L->mask[t] & 1) && state[J] == UND && !key_greater(L->lambda, hash, I, J))
                    is_max = 0;
            }
            for (int32_t t = tptr[I]; t < tptr[I + 1] && is_max; ++t) {
                int32_t J = tidx[t];
                if (state[J] == UND && !key_greater(L->lambda, hash, I, J)) is_max = 0;
            }
            newc[I] = (int8_t)is_max;
        }
        for (int32_t I = 0; I < nb; ++I) {
            if (state[I] != UND) continue;
            if (newc[I]) {
                state[I] = CPT;
                L->dround[I] = rounds;
                undecided--;
                continue;
            }
            for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
                if ((L->mask[t] & 1) && newc[A->colidx[t]]) {
                    state[I] = FPT;
                    L->dround[I] = rounds;
                    undecided--;
                    break;
                }
        }
    }
    for (int32_t I = 0; I < nb; ++I) L->cf[I] = state[I];
    L->pmis_rounds = rounds;
    free(tptr);
    free(tidx);
    free(fill);
    free(hash);
    free(state);
    free(newc);
    return ORA_OK;
}

/* --------------------------------------------------- one-point interpolation */

/*
 * One-point interpolation (section 5.1): each F block takes the value of its
 * strongest C connection, with weight identity.  Reading: candidates are all
 * stored C blocks of the row with nonzero size (not only theta-strong ones);
 * ties go to the lowest column; no candidate gives a zero row (pmap = -1).
 * C blocks map to their own coarse index.
 */
static void one_point(level_t *L) {
    const bsr_t *A = &L->A;
    for (int32_t I = 0; I < A->nb; ++I) {
        if (L->cf[I] == 1) {
            L->pmap[I] = L->cidx[I];
            continue;
        }
        int32_t best = -1;
        double bestn = 0.0;
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
            int32_t J = A->colidx[t];
            if (J != I && L->cf[J] == 1 && L->bnorm[t] > bestn) {
                bestn = L->bnorm[t];
                best = J;
            }
        }
        L->pmap[I] = (best >= 0) ? L->cidx[best] : -1;
        /* audit: another candidate within 1e-12 of the chosen one's size */
        if (best >= 0)
            for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
                int32_t J = A->colidx[t];
                if (J != I && J != best && L->cf[J] == 1 && L->bnorm[t] > 0.0 && near_tie(L->bnorm[t], bestn)) {
                    L->margin[2] += 1;
                    break;
                }
            }
    }
}

/* ---------------------------------------------------- sparse block products */

/*
 * C = X * Y (Gustavson, row by row).  For each output entry the contributions
 * arrive in ascending inner index K, each as the c-ascending fma chain, all in
 * one accumulator that starts at +0.  Output columns sorted ascending.
 * If `xdiag` is not NULL, row i of X also holds an identity block in column
 * xdiag[i] (which X itself does not store); its contribution, Y's row
 * xdiag[i], is added plainly at its place in the K order.
 */
static int spgemm(const bsr_t *X, const int32_t *xdiag, const bsr_t *Y, bsr_t *C) {
    int32_t bs = X->bs, bb = bs * bs;
    int32_t m = X->nb, ncy = Y->ncols;
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncy > 0 ? ncy : 1));
    int32_t *cols = NULL;
    double *acc = NULL;
    int64_t cap = 0;
    for (int32_t J = 0; J < ncy; ++J) slot[J] = -1;
    /* pass 1: row counts */
    int32_t *cnt = (int32_t *)xcalloc((size_t)m + 1, sizeof(int32_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncy > 0 ? ncy : 1));
    for (int32_t i = 0; i < m; ++i) {
        int32_t nt = 0;
        int32_t nk = X->rowptr[i + 1] - X->rowptr[i] + (xdiag ? 1 : 0);
        for (int32_t q = 0; q < nk; ++q) {
            int32_t K = (q < X->rowptr[i + 1] - X->rowptr[i]) ? X->colidx[X->rowptr[i] + q] : xdiag[i];
            for (int32_t u = Y->rowptr[K]; u < Y->rowptr[K + 1]; ++u) {
                int32_t J = Y->colidx[u];
                if (slot[J] < 0) {
                    slot[J] = 1;
                    touched[nt++] = J;
                }
            }
        }
        for (int32_t q = 0; q < nt; ++q) slot[touched[q]] = -1;
        cnt[i + 1] = nt;
        if (nt > cap) cap = nt;
    }
    for (int32_t i = 0; i < m; ++i) cnt[i + 1] += cnt[i];
    int st = bsr_alloc(C, m, ncy, bs, cnt[m]);
    if (st != ORA_OK) return st;
    memcpy(C->rowptr, cnt, sizeof(int32_t) * ((size_t)m + 1));
    cols = (int32_t *)xcalloc((size_t)cap, sizeof(int32_t));
    acc = (double *)xcalloc((size_t)cap * bb, sizeof(double));
    /* pass 2: sorted pattern and values */
    for (int32_t i = 0; i < m; ++i) {
        int32_t nt = 0;
        int32_t xlo = X->rowptr[i], xhi = X->rowptr[i + 1];
        for (int32_t q = xlo; q < xhi; ++q) {
            int32_t K = X->colidx[q];
            for (int32_t u = Y->rowptr[K]; u < Y->rowptr[K + 1]; ++u)
                if (slot[Y->colidx[u]] < 0) {
                    slot[Y->colidx[u]] = 0;
                    cols[nt++] = Y->colidx[u];
                }
        }
        if (xdiag) {
            int32_t K = xdiag[i];
            for (int32_t u = Y->rowptr[K]; u < Y->rowptr[K + 1]; ++u)
                if (slot[Y->colidx[u]] < 0) {
                    slot[Y->colidx[u]] = 0;
                    cols[nt++] = Y->colidx[u];
                }
        }
        qsort(cols, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int32_t q = 0; q < nt; ++q) slot[cols[q]] = q;
        memset(acc, 0, sizeof(double) * (size_t)nt * bb);
        /* K ascending, merging the implicit identity column into X's sorted row */
        int32_t q = xlo;
        int diag_done = (xdiag == NULL);
        while (q < xhi || !diag_done) {
            int take_diag = !diag_done && (q >= xhi || xdiag[i] < X->colidx[q]);
            if (take_diag) {
                int32_t K = xdiag[i];
                for (int32_t u = Y->rowptr[K]; u < Y->rowptr[K + 1]; ++u) {
                    double *dst = acc + (size_t)slot[Y->colidx[u]] * bb;
                    const double *src = Y->vals + (size_t)u * bb;
                    for (int32_t e = 0; e < bb; ++e) dst[e] = dst[e] + src[e];
                }
                diag_done = 1;
            } else {
                int32_t K = X->colidx[q];
                const double *xb = X->vals + (size_t)q * bb;
                for (int32_t u = Y->rowptr[K]; u < Y->rowptr[K + 1]; ++u)
                    block_mul_acc(bs, xb, Y->vals + (size_t)u * bb,
                                  acc + (size_t)slot[Y->colidx[u]] * bb);
                ++q;
            }
        }
        int32_t base = C->rowptr[i];
        for (int32_t t = 0; t < nt; ++t) {
            C->colidx[base + t] = cols[t];
            memcpy(C->vals + (size_t)(base + t) * bb, acc + (size_t)t * bb, sizeof(double) * bb);
            slot[cols[t]] = -1;
        }
    }
    free(slot);
    free(cnt);
    free(touched);
    free(cols);
    free(acc);
    return ORA_OK;
}

/* S = S + W entrywise (union pattern, plain adds, S's value first). */
static int bsr_add_inplace(bsr_t *S, const bsr_t *W) {
    int32_t bb = S->bs * S->bs;
    bsr_t O;
    int64_t nnz = 0;
    for (int32_t i = 0; i < S->nb; ++i) {
        int32_t p = S->rowptr[i], q = W->rowptr[i];
        while (p < S->rowptr[i + 1] || q < W->rowptr[i + 1]) {
            if (q >= W->rowptr[i + 1] || (p < S->rowptr[i + 1] && S->colidx[p] < W->colidx[q])) p++;
            else if (p >= S->rowptr[i + 1] || W->colidx[q] < S->colidx[p]) q++;
            else { p++; q++; }
            nnz++;
        }
    }
    int st = bsr_alloc(&O, S->nb, S->ncols, S->bs, nnz);
    if (st != ORA_OK) return st;
    int64_t o = 0;
    for (int32_t i = 0; i < S->nb; ++i) {
        int32_t p = S->rowptr[i], q = W->rowptr[i];
        while (p < S->rowptr[i + 1] || q < W->rowptr[i + 1]) {
            double *dst = O.vals + (size_t)o * bb;
            if (q >= W->rowptr[i + 1] || (p < S->rowptr[i + 1] && S->colidx[p] < W->colidx[q])) {
                O.colidx[o] = S->colidx[p];
                memcpy(dst, S->vals + (size_t)p * bb, sizeof(double) * bb);
                p++;
            } else if (p >= S->rowptr[i + 1] || W->colidx[q] < S->colidx[p]) {
                O.colidx[o] = W->colidx[q];
                memcpy(dst, W->vals + (size_t)q * bb, sizeof(double) * bb);
                q++;
            } else {
                O.colidx[o] = S->colidx[p];
                const double *x = S->vals + (size_t)p * bb, *y = W->vals + (size_t)q * bb;
                for (int32_t e = 0; e < bb; ++e) dst[e] = x[e] + y[e];
                p++;
                q++;
            }
            o++;
        }
        O.rowptr[i + 1] = (int32_t)o;
    }
    bsr_free(S);
    *S = O;
    return ORA_OK;
}

/* -------------------------------------------------------- Neumann restriction */

/*
 * Neumann approximate ideal restriction (section 4.1, eq. "neumann", and the
 * restriction R = [-A_cf Delta^(k), I]) in block form.  With A_ff = D_ff - L,
 * where L holds the phi-strong off-diagonal F-F blocks negated (weak ones are
 * left out of the expansion, section 5.1),
 *     A_ff^{-1} ~ sum_{i<=k} (D_ff^{-1} L)^i D_ff^{-1},
 * so with T = D_ff^{-1} L, i.e. T_IJ = -(Dinv_I A_IJ) for phi-strong F-F
 * blocks J != I, and W_0 = A_cf (every stored C-row, F-column block):
 *     W_i = W_{i-1} T,   S = ((W_0 + W_1) + W_2) + ...,   Z_IJ = -(S_IJ Dinv_J).
 * Z has nc rows (coarse numbering) and fine F columns.  R is not filtered.
 */
static int neumann_Z(level_t *L, int32_t degree) {
    const bsr_t *A = &L->A;
    int32_t nb = A->nb, bs = A->bs, bb = bs * bs;
    bsr_t T, W, S, Wn;
    int st;
    /* T over fine indices (C rows empty) */
    int64_t nT = 0;
    for (int32_t I = 0; I < nb; ++I)
        if (L->cf[I] == 0)
            for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
                int32_t J = A->colidx[t];
                if (J != I && L->cf[J] == 0 && (L->mask[t] & 2)) nT++;
            }
    if ((st = bsr_alloc(&T, nb, nb, bs, nT)) != ORA_OK) return st;
    int64_t o = 0;
    for (int32_t I = 0; I < nb; ++I) {
        if (L->cf[I] == 0)
            for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
                int32_t J = A->colidx[t];
                if (J != I && L->cf[J] == 0 && (L->mask[t] & 2)) {
                    double *dst = T.vals + (size_t)o * bb;
                    block_mul(bs, L->dinv + (size_t)I * bb, A->vals + (size_t)t * bb, dst);
                    for (int32_t e = 0; e < bb; ++e) dst[e] = -dst[e];
                    T.colidx[o++] = J;
                }
            }
        T.rowptr[I + 1] = (int32_t)o;
    }
    /* W_0 = A_cf */
    int64_t nW = 0;
    for (int32_t i = 0; i < L->nc; ++i) {
        int32_t I = L->cpts[i];
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
            if (L->cf[A->colidx[t]] == 0) nW++;
    }
    if ((st = bsr_alloc(&W, L->nc, nb, bs, nW)) != ORA_OK) return st;
    o = 0;
    for (int32_t i = 0; i < L->nc; ++i) {
        int32_t I = L->cpts[i];
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
            if (L->cf[A->colidx[t]] == 0) {
                W.colidx[o] = A->colidx[t];
                memcpy(W.vals + (size_t)o * bb, A->vals + (size_t)t * bb, sizeof(double) * bb);
                o++;
            }
        W.rowptr[i + 1] = (int32_t)o;
    }
    /* S = W_0 (copy), then add W_1..W_k */
    if ((st = bsr_alloc(&S, W.nb, nb, bs, W.rowptr[W.nb])) != ORA_OK) return st;
    memcpy(S.rowptr, W.rowptr, sizeof(int32_t) * ((size_t)W.nb + 1));
    memcpy(S.colidx, W.colidx, sizeof(int32_t) * (size_t)W.rowptr[W.nb]);
    memcpy(S.vals, W.vals, sizeof(double) * (size_t)W.rowptr[W.nb] * bb);
    for (int32_t d = 1; d <= degree; ++d) {
        if ((st = spgemm(&W, NULL, &T, &Wn)) != ORA_OK) return st;
        bsr_free(&W);
        W = Wn;
        if ((st = bsr_add_inplace(&S, &W)) != ORA_OK) return st;
    }
    /* Z_IJ = -(S_IJ Dinv_J) */
    L->Z = S;
    double *tmp = (double *)malloc(sizeof(double) * bb);
    for (int32_t t = 0; t < S.rowptr[S.nb]; ++t) {
        double *blk = L->Z.vals + (size_t)t * bb;
        block_mul(bs, blk, L->dinv + (size_t)L->Z.colidx[t] * bb, tmp);
        for (int32_t e = 0; e < bb; ++e) blk[e] = -tmp[e];
    }
    free(tmp);
    bsr_free(&T);
    bsr_free(&W);
    return ORA_OK;
}

/* ------------------------------------------------------------- Galerkin RAP */

/*
 * M P for one-point P given by pmap (column J of M goes to column pmap(J), or
 * is dropped when pmap(J) < 0): row i of the result holds, at each column t,
 * the blocks M_iJ with pmap(J) = t summed in ascending J (entry by entry, from
 * +0).  Columns ascending.
 */
static int merge_columns(const bsr_t *M, const int32_t *pmap, int32_t ncols, bsr_t *out) {
    int32_t bs = M->bs, bb = bs * bs, m = M->nb;
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
    for (int32_t j = 0; j < ncols; ++j) slot[j] = -1;
    int64_t total = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t nt = 0;
        for (int32_t u = M->rowptr[i]; u < M->rowptr[i + 1]; ++u) {
            int32_t t = pmap[M->colidx[u]];
            if (t >= 0 && slot[t] < 0) {
                slot[t] = 0;
                cols[nt++] = t;
            }
        }
        for (int32_t q = 0; q < nt; ++q) slot[cols[q]] = -1;
        total += nt;
    }
    int st = bsr_alloc(out, m, ncols, bs, total);
    if (st != ORA_OK) {
        free(slot);
        free(cols);
        return st;
    }
    int64_t o = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t nt = 0;
        for (int32_t u = M->rowptr[i]; u < M->rowptr[i + 1]; ++u) {
            int32_t t = pmap[M->colidx[u]];
            if (t >= 0 && slot[t] < 0) {
                slot[t] = 0;
                cols[nt++] = t;
            }
        }
        qsort(cols, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int32_t q = 0; q < nt; ++q) {
            slot[cols[q]] = (int32_t)(o + q);
            out->colidx[o + q] = cols[q];
        }
        for (int32_t u = M->rowptr[i]; u < M->rowptr[i + 1]; ++u) {
            int32_t t = pmap[M->colidx[u]];
            if (t < 0) continue;
            double *dst = out->vals + (size_t)slot[t] * bb;
            const double *src = M->vals + (size_t)u * bb;
            for (int32_t e = 0; e < bb; ++e) dst[e] = dst[e] + src[e];
        }
        for (int32_t q = 0; q < nt; ++q) slot[cols[q]] = -1;
        o += nt;
        out->rowptr[i + 1] = (int32_t)o;
    }
    free(slot);
    free(cols);
    return ORA_OK;
}

/*
 * Coarse operator K = R A P (eq. "rap") with R = [Z I] and one-point P, then
 * the drop filter of section 5.2.
 *   AP = A P: each row of A with its columns merged through pmap (a sum of
 *        A's blocks per coarse column; P has one unit block per row, so A P
 *        is formed before the product with R -- reading: the association
 *        R (A P), which needs fewer block products than (R A) P);
 *   K_i = sum over R's row i in ascending column of R_iK AP_K (the identity
 *        block at C column cpts[i] is added plainly);
 *   off-diagonal K blocks with ||K_it||_max <= drop * ||K_ii||_max are removed.
 * Reading: the filter applies to the coarse operators only, never to the
 * input matrix or to R; block max-abs norms; "<=" as printed.
 */
static int galerkin(level_t *L, double drop, bsr_t *Kout) {
    const bsr_t *A = &L->A;
    int32_t bs = A->bs, bb = bs * bs, nc = L->nc;
    (void)bb;
    bsr_t AP, K;
    int st = merge_columns(A, L->pmap, nc, &AP);
    if (st != ORA_OK) return st;
    st = spgemm(&L->Z, L->cpts, &AP, &K);
    bsr_free(&AP);
    if (st != ORA_OK) return st;
    int64_t total = K.rowptr[nc];
    double *kn = (double *)xcalloc((size_t)(total > 0 ? total : 1), sizeof(double));
    int64_t kept = 0;
    for (int32_t i = 0; i < nc; ++i) {
        double dn = 0.0;
        for (int32_t t = K.rowptr[i]; t < K.rowptr[i + 1]; ++t) {
            kn[t] = block_maxabs(bs, K.vals + (size_t)t * bb);
            if (K.colidx[t] == i) dn = kn[t];
        }
        double thr = drop * dn;
        for (int32_t t = K.rowptr[i]; t < K.rowptr[i + 1]; ++t) {
            if (K.colidx[t] == i || kn[t] > thr) kept++;
            if (K.colidx[t] != i) L->margin[3] += near_tie(kn[t], thr);
        }
    }
    if ((st = bsr_alloc(Kout, nc, nc, bs, kept)) != ORA_OK) {
        free(kn);
        bsr_free(&K);
        return st;
    }
    int64_t o = 0;
    for (int32_t i = 0; i < nc; ++i) {
        double dn = 0.0;
        for (int32_t t = K.rowptr[i]; t < K.rowptr[i + 1]; ++t)
            if (K.colidx[t] == i) dn = kn[t];
        double thr = drop * dn;
        for (int32_t t = K.rowptr[i]; t < K.rowptr[i + 1]; ++t)
            if (K.colidx[t] == i || kn[t] > thr) {
                Kout->colidx[o] = K.colidx[t];
                memcpy(Kout->vals + (size_t)o * bb, K.vals + (size_t)t * bb, sizeof(double) * bb);
                o++;
            }
        Kout->rowptr[i + 1] = (int32_t)o;
    }
    free(kn);
    bsr_free(&K);
    return ORA_OK;
}

/* ------------------------------------------------------------ dense coarsest */

/* Dense LU with partial pivoting of the coarsest operator (the paper leaves the
 * coarsest solve open; it is solved directly). */
static int dense_factor(level_t *L) {
    const bsr_t *A = &L->A;
    int32_t bs = A->bs, n = A->nb * bs;
    L->dense_n = n;
    L->lu = (double *)xcalloc((size_t)n * n, sizeof(double));
    L->piv = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    if (!L->lu || !L->piv) return ORA_ENOMEM;
    for (int32_t I = 0; I < A->nb; ++I)
        for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t)
            for (int32_t a = 0; a < bs; ++a)
                for (int32_t b = 0; b < bs; ++b)
                    L->lu[(size_t)(I * bs + a) * n + A->colidx[t] * bs + b] =
                        A->vals[(size_t)t * bs * bs + a * bs + b];
    double *a = L->lu;
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int32_t i = k + 1; i < n; ++i)
            if (fabs(a[(size_t)i * n + k]) > best) {
                best = fabs(a[(size_t)i * n + k]);
                p = i;
            }
        if (!(best > 0.0)) return ORA_ESINGULAR;
        L->piv[k] = p;
        if (p != k)
            for (int32_t j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        for (int32_t i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            a[(size_t)i * n + k] = l;
            for (int32_t j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return ORA_OK;
}

static void dense_solve(const level_t *L, const double *r, double *x) {
    int32_t n = L->dense_n;
    const double *a = L->lu;
    for (int32_t i = 0; i < n; ++i) x[i] = r[i];
    for (int32_t k = 0; k < n; ++k)
        if (L->piv[k] != k) {
            double t = x[k];
            x[k] = x[L->piv[k]];
            x[L->piv[k]] = t;
        }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t m = 0; m < i; ++m) x[i] -= a[(size_t)i * n + m] * x[m];
    for (int32_t i = n - 1; i >= 0; --i) {
        for (int32_t m = i + 1; m < n; ++m) x[i] -= a[(size_t)i * n + m] * x[m];
        x[i] /= a[(size_t)i * n + i];
    }
}

/* x = A^{-T} r with P A = L U:  A^T = U^T L^T P, so solve U^T w = r, L^T v = w, x = P^T v. */
static void dense_solve_T(const level_t *L, const double *r, double *x) {
    int32_t n = L->dense_n;
    const double *a = L->lu;
    for (int32_t i = 0; i < n; ++i) x[i] = r[i];
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t m = 0; m < i; ++m) x[i] -= a[(size_t)m * n + i] * x[m];
        x[i] /= a[(size_t)i * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i)
        for (int32_t m = i + 1; m < n; ++m) x[i] -= a[(size_t)m * n + i] * x[m];
    for (int32_t k = n - 1; k >= 0; --k)
        if (L->piv[k] != k) {
            double t = x[k];
            x[k] = x[L->piv[k]];
            x[L->piv[k]] = t;
        }
}

/* ------------------------------------------------------------------ setup */

void ora_default_params(ora_params *p) {
    p->degree = 1;
    p->theta = 0.75;
    p->phi = 0.025;
    p->drop = 1e-3;
    p->relax = 0;
    p->max_levels = 30;
    p->max_coarse_dofs = 128;
    p->seed = 0;
    p->cf_override = NULL;
    p->form = 0;
    p->cycle = 0;
    p->gmres = 0;
}

static int validate(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx) {
    if (nb < 1 || bs < 1 || !rowptr || !colidx) return ORA_EINVAL;
    if (rowptr[0] != 0) return ORA_EINVAL;
    for (int32_t I = 0; I < nb; ++I) {
        if (rowptr[I + 1] < rowptr[I]) return ORA_EINVAL;
        int has_diag = 0;
        for (int32_t t = rowptr[I]; t < rowptr[I + 1]; ++t) {
            if (colidx[t] < 0 || colidx[t] >= nb) return ORA_EINVAL;
            if (t > rowptr[I] && colidx[t] <= colidx[t - 1]) return ORA_EINVAL;
            if (colidx[t] == I) has_diag = 1;
        }
        if (!has_diag) return ORA_EINVAL;
    }
    return ORA_OK;
}

static void level_free(level_t *L) {
    bsr_free(&L->A);
    bsr_free(&L->Z);
    free(L->dinv);
    free(L->bnorm);
    free(L->mask);
    free(L->lambda);
    free(L->cf);
    free(L->cidx);
    free(L->pmap);
    free(L->cpts);
    free(L->dround);
    free(L->lu);
    free(L->piv);
    memset(L, 0, sizeof(*L));
}

void ora_free(ora_hier *h) {
    if (!h) return;
    for (int32_t l = 0; l < ORA_MAX_LEVELS; ++l) level_free(&h->lv[l]);
    bsr_free(&h->A0);
    free(h->d0inv);
    free(h);
}

/*
 * Scalar form (section "Blocks, filtering, and parallelization": most of the
 * paper's results scale the system by the inverse of its block diagonal and
 * run scalar nAIR on it).  S = D^{-1} A as a scalar CSR (1 x 1 blocks): the
 * diagonal blocks of D^{-1} A are the identity by definition and are taken
 * exactly (one entry 1 per row); an off-diagonal block is D_I^{-1} A_IJ (fma
 * chains, c ascending from +0) and contributes every entry that is not exactly
 * zero.  Columns ascend within each row.
 */
static int scaled_scalar(const bsr_t *A, const double *dinv, bsr_t *S) {
    const int32_t bs = A->bs, bb = bs * bs;
    const int64_t n = (int64_t)A->nb * bs;
    double *M = (double *)malloc(sizeof(double) * (size_t)bb);
    int64_t nnz = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t o = 0;
        for (int32_t I = 0; I < A->nb; ++I)
            for (int32_t a = 0; a < bs; ++a) {
                for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
                    const int32_t J = A->colidx[t];
                    if (J == I) {
                        if (pass) {
                            S->colidx[o] = I * bs + a;
                            S->vals[o] = 1.0;
                        }
                        ++o;
                        continue;
                    }
                    block_mul(bs, dinv + (size_t)I * bb, A->vals + (size_t)t * bb, M);
                    for (int32_t b = 0; b < bs; ++b)
                        if (M[a * bs + b] != 0.0) {
                            if (pass) {
                                S->colidx[o] = J * bs + b;
                                S->vals[o] = M[a * bs + b];
                            }
                            ++o;
                        }
                }
                if (pass) S->rowptr[(int64_t)I * bs + a + 1] = (int32_t)o;
            }
        if (!pass) {
            nnz = o;
            if (nnz > 2147483647LL || bsr_alloc(S, (int32_t)n, (int32_t)n, 1, nnz) != ORA_OK) {
                free(M);
                return ORA_ENOMEM;
            }
            S->rowptr[0] = 0;
        }
    }
    free(M);
    return ORA_OK;
}

int ora_setup(int32_t nb, int32_t bs, const int32_t *rowptr, const int32_t *colidx,
              const double *vals, const ora_params *prm, ora_hier **out) {
    if (!prm || !out || !vals) return ORA_EINVAL;
    *out = NULL;
    if (prm->degree < 0 || prm->max_levels < 1 || prm->max_levels > ORA_MAX_LEVELS) return ORA_EINVAL;
    if (prm->cycle != 0 && prm->cycle != 1) return ORA_EINVAL;
    if (prm->gmres < 0 || prm->gmres > 200) return ORA_EINVAL;
    if (!(prm->theta >= 0.0 && prm->theta < 1.0) || !(prm->phi >= 0.0 && prm->phi < 1.0) ||
        !(prm->drop >= 0.0 && prm->drop < 1.0))
        return ORA_EINVAL;
    int st = validate(nb, bs, rowptr, colidx);
    if (st != ORA_OK) return st;
    ora_hier *h = (ora_hier *)calloc(1, sizeof(ora_hier));
    if (!h) return ORA_ENOMEM;
    h->prm = *prm;
    int32_t bb = bs * bs;
    int64_t nnzb = rowptr[nb];
    level_t *L0 = &h->lv[0];
    if (prm->form == 1) {
        /* the caller's system, its block-diagonal inverse, and S = D^{-1} A as level 0 */
        if ((st = bsr_alloc(&h->A0, nb, nb, bs, nnzb)) != ORA_OK) goto fail;
        memcpy(h->A0.rowptr, rowptr, sizeof(int32_t) * ((size_t)nb + 1));
        memcpy(h->A0.colidx, colidx, sizeof(int32_t) * (size_t)nnzb);
        memcpy(h->A0.vals, vals, sizeof(double) * (size_t)nnzb * bb);
        h->d0inv = (double *)xcalloc((size_t)nb * bb, sizeof(double));
        if (!h->d0inv) {
            st = ORA_ENOMEM;
            goto fail;
        }
        for (int32_t I = 0; I < nb; ++I) {
            int32_t t = rowptr[I];
            while (colidx[t] != I) ++t;
            if ((st = ora_block_inverse(bs, vals + (size_t)t * bb, h->d0inv + (size_t)I * bb)) != ORA_OK) goto fail;
        }
        if ((st = scaled_scalar(&h->A0, h->d0inv, &L0->A)) != ORA_OK) goto fail;
        bs = 1;   /* the hierarchy is scalar */
        bb = 1;
    } else if (prm->form != 0) {
        st = ORA_EINVAL;
        goto fail;
    } else {
        if ((st = bsr_alloc(&L0->A, nb, nb, bs, nnzb)) != ORA_OK) goto fail;
        memcpy(L0->A.rowptr, rowptr, sizeof(int32_t) * ((size_t)nb + 1));
        memcpy(L0->A.colidx, colidx, sizeof(int32_t) * (size_t)nnzb);
        memcpy(L0->A.vals, vals, sizeof(double) * (size_t)nnzb * bb);
    }

    for (int32_t l = 0;; ++l) {
        level_t *L = &h->lv[l];
        int32_t n = L->A.nb;
        h->nlev = l + 1;
        if ((int64_t)n * bs <= prm->max_coarse_dofs || l == prm->max_levels - 1) {
            L->coarsest = 1;
            if ((st = dense_factor(L)) != ORA_OK) goto fail;
            break;
        }
        int64_t nz = L->A.rowptr[n];
        L->dinv = (double *)xcalloc((size_t)n * bb, sizeof(double));
        L->bnorm = (double *)xcalloc((size_t)nz, sizeof(double));
        L->mask = (uint8_t *)xcalloc((size_t)nz, 1);
        L->lambda = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
        L->cf = (int8_t *)xcalloc((size_t)n, 1);
        L->cidx = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
        L->pmap = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
        L->cpts = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
        L->dround = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
        if (!L->dround || !L->dinv || !L->bnorm || !L->mask || !L->lambda || !L->cf || !L->cidx || !L->pmap || !L->cpts) {
            st = ORA_ENOMEM;
            goto fail;
        }
        for (int32_t I = 0; I < n; ++I) {
            int32_t t = L->A.rowptr[I];
            while (L->A.colidx[t] != I) ++t;
            if ((st = ora_block_inverse(bs, L->A.vals + (size_t)t * bb, L->dinv + (size_t)I * bb)) != ORA_OK)
                goto fail;
        }
        strength(L, prm->theta, prm->phi);
        if (l == 0 && prm->cf_override) {
            for (int32_t I = 0; I < n; ++I) L->cf[I] = prm->cf_override[I] ? 1 : 0;
            L->pmis_rounds = 0;
        } else if ((st = split_cf(L, l, prm->seed)) != ORA_OK) {
            goto fail;
        }
        L->nc = 0;
        for (int32_t I = 0; I < n; ++I) {
            if (L->cf[I] == 1) {
                L->cidx[I] = L->nc;
                L->cpts[L->nc++] = I;
            } else {
                L->cidx[I] = -1;
            }
        }
        if (L->nc == 0 || L->nc == n) {
            if ((int64_t)n * bs > ORA_STALL_DENSE_DOFS) {
                st = ORA_ECOARSEN;
                goto fail;
            }
            L->coarsest = 1;
            if ((st = dense_factor(L)) != ORA_OK) goto fail;
            break;
        }
        one_point(L);
        if ((st = neumann_Z(L, prm->degree)) != ORA_OK) goto fail;
        if ((st = galerkin(L, prm->drop, &h->lv[l + 1].A)) != ORA_OK) goto fail;
    }
    *out = h;
    return ORA_OK;
fail:
    ora_free(h);
    return st;
}

/* ------------------------------------------------------------------ cycle */

/* y = b - A x over the given rows only (rows == NULL: all rows). */
static void block_row_residual(const bsr_t *A, int32_t I, const double *b, const double *x, double *out) {
    int32_t bs = A->bs;
    for (int32_t a = 0; a < bs; ++a) out[a] = b[(size_t)I * bs + a];
    for (int32_t t = A->rowptr[I]; t < A->rowptr[I + 1]; ++t) {
        const double *blk = A->vals + (size_t)t * bs * bs;
        const double *xj = x + (size_t)A->colidx[t] * bs;
        for (int32_t a = 0; a < bs; ++a) {
            double s = 0.0;
            for (int32_t c = 0; c < bs; ++c) s += blk[a * bs + c] * xj[c];
            out[a] -= s;
        }
    }
}

/* out = b - A^T y (transposed blocks scattered by column). */
static void residual_T(const bsr_t *A, const double *g, const double *y, double *out) {
    int32_t bs = A->bs;
    int64_t n = (int64_t)A->nb * bs;
    for (int64_t i = 0; i < n; ++i) out[i] = g[i];
    for (int32_t J = 0; J < A->nb; ++J)
        for (int32_t t = A->rowptr[J]; t < A->rowptr[J + 1]; ++t) {
            const double *blk = A->vals + (size_t)t * bs * bs;
            int32_t I = A->colidx[t];
            for (int32_t c = 0; c < bs; ++c) {
                double s = 0.0;
                for (int32_t a = 0; a < bs; ++a) s += blk[a * bs + c] * y[(size_t)J * bs + a];
                out[(size_t)I * bs + c] -= s;
            }
        }
}

/* v_out = M v (trans = 0) or M^T v (trans = 1) for one bs x bs block. */
static void block_apply(int32_t bs, const double *M, const double *v, double *out, int trans) {
    for (int32_t a = 0; a < bs; ++a) {
        double s = 0.0;
        for (int32_t c = 0; c < bs; ++c) s += (trans ? M[c * bs + a] : M[a * bs + c]) * v[c];
        out[a] = s;
    }
}

/* One Jacobi sweep over blocks with cf == which:  e_I += Dinv_I (r - A e)_I. */
static void jacobi_sweep(const level_t *L, int8_t which, const double *r, double *e, double *work) {
    const bsr_t *A = &L->A;
    int32_t bs = A->bs;
    double *t = (double *)malloc(sizeof(double) * bs);
    double *d = (double *)malloc(sizeof(double) * bs);
    int64_t n = (int64_t)A->nb * bs;
    memcpy(work, e, sizeof(double) * (size_t)n);
    for (int32_t I = 0; I < A->nb; ++I) {
        if (L->cf[I] != which) continue;
        block_row_residual(A, I, r, e, t);
        block_apply(bs, L->dinv + (size_t)I * bs * bs, t, d, 0);
        for (int32_t a = 0; a < bs; ++a) work[(size_t)I * bs + a] = e[(size_t)I * bs + a] + d[a];
    }
    memcpy(e, work, sizeof(double) * (size_t)n);
    free(t);
    free(d);
}

/* Transposed Jacobi sweep:  y_I += Dinv_I^T (g - A^T y)_I for cf == which. */
static void jacobi_sweep_T(const level_t *L, int8_t which, const double *g, double *y, double *work) {
    const bsr_t *A = &L->A;
    int32_t bs = A->bs;
    int64_t n = (int64_t)A->nb * bs;
    double *d = (double *)malloc(sizeof(double) * bs);
    residual_T(A, g, y, work);
    for (int32_t I = 0; I < A->nb; ++I) {
        if (L->cf[I] != which) continue;
        block_apply(bs, L->dinv + (size_t)I * bs * bs, work + (size_t)I * bs, d, 1);
        for (int32_t a = 0; a < bs; ++a) y[(size_t)I * bs + a] += d[a];
    }
    (void)n;
    free(d);
}

/*
 * V-cycle from a zero initial guess with no pre-relaxation (section 5):
 * restrict r_c = r_C + Z r_F, recurse, interpolate e = P e_c, then nu = k+1
 * Jacobi F sweeps (section 5.1) and, for FC, one Jacobi C sweep.  The F-cycle
 * (compared with V-cycles in the section "Scaling in h and element order")
 * differs only in its coarse solve, an F-cycle followed by a V-cycle.
 */
/* The coarse-grid correction's coarse solve on level l: one V-cycle, or (fcyc)
 * one F-cycle followed by one V-cycle on its residual,
 * e_c = F r_c + V (r_c - A_c F r_c). */
static void coarse_solve(const ora_hier *h, int32_t l, int fcyc, const double *rc, double *ec);

/* fcyc = 0: V-cycle; 1: F-cycle (its coarse solve is an F-cycle then a V-cycle). */
static void cycle(const ora_hier *h, int32_t l, int fcyc, const double *r, double *e) {
    const level_t *L = &h->lv[l];
    int32_t bs = L->A.bs;
    int64_t n = (int64_t)L->A.nb * bs;
    if (L->coarsest) {
        dense_solve(L, r, e);
        return;
    }
    int64_t nc = (int64_t)L->nc * bs;
    double *rc = (double *)xcalloc((size_t)nc, sizeof(double));
    double *ec = (double *)xcalloc((size_t)nc, sizeof(double));
    double *work = (double *)xcalloc((size_t)n, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * bs);
    for (int32_t i = 0; i < L->nc; ++i) {
        for (int32_t a = 0; a < bs; ++a) rc[(size_t)i * bs + a] = r[(size_t)L->cpts[i] * bs + a];
        for (int32_t t = L->Z.rowptr[i]; t < L->Z.rowptr[i + 1]; ++t) {
            block_apply(bs, L->Z.vals + (size_t)t * bs * bs, r + (size_t)L->Z.colidx[t] * bs, tmp, 0);
            for (int32_t a = 0; a < bs; ++a) rc[(size_t)i * bs + a] += tmp[a];
        }
    }
    coarse_solve(h, l + 1, fcyc, rc, ec);
    for (int32_t I = 0; I < L->A.nb; ++I)
        for (int32_t a = 0; a < bs; ++a)
            e[(size_t)I * bs + a] = (L->pmap[I] >= 0) ? ec[(size_t)L->pmap[I] * bs + a] : 0.0;
    for (int32_t s = 0; s <= h->prm.degree; ++s) jacobi_sweep(L, 0, r, e, work);
    if (h->prm.relax == 1) jacobi_sweep(L, 1, r, e, work);
    free(rc);
    free(ec);
    free(work);
    free(tmp);
}

/*
 * The transpose of the V-cycle operator B: with FC, y_C = Dinv_C^T g_C first;
 * then nu transposed Jacobi F sweeps (pre-relaxation, the ordering that suits
 * ideal interpolation, section 2.2 corollary and section 3.1 remark); then
 * s = g - A^T y, s_c = P^T s, recurse, and y += R^T y_c = [Z^T y_c; y_c].
 */
static void coarse_solve_T(const ora_hier *h, int32_t l, int fcyc, const double *sc, double *yc);

static void cycle_T(const ora_hier *h, int32_t l, int fcyc, const double *g, double *y) {
    const level_t *L = &h->lv[l];
    int32_t bs = L->A.bs;
    int64_t n = (int64_t)L->A.nb * bs;
    if (L->coarsest) {
        dense_solve_T(L, g, y);
        return;
    }
    int64_t nc = (int64_t)L->nc * bs;
    double *sc = (double *)xcalloc((size_t)nc, sizeof(double));
    double *yc = (double *)xcalloc((size_t)nc, sizeof(double));
    double *work = (double *)xcalloc((size_t)n, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * bs);
    for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
    if (h->prm.relax == 1)
        for (int32_t I = 0; I < L->A.nb; ++I)
            if (L->cf[I] == 1) block_apply(bs, L->dinv + (size_t)I * bs * bs, g + (size_t)I * bs, y + (size_t)I * bs, 1);
    for (int32_t s = 0; s <= h->prm.degree; ++s) jacobi_sweep_T(L, 0, g, y, work);
    residual_T(&L->A, g, y, work);
    for (int32_t I = 0; I < L->A.nb; ++I)
        if (L->pmap[I] >= 0)
            for (int32_t a = 0; a < bs; ++a) sc[(size_t)L->pmap[I] * bs + a] += work[(size_t)I * bs + a];
    coarse_solve_T(h, l + 1, fcyc, sc, yc);
    for (int32_t i = 0; i < L->nc; ++i) {
        for (int32_t a = 0; a < bs; ++a) y[(size_t)L->cpts[i] * bs + a] += yc[(size_t)i * bs + a];
        for (int32_t t = L->Z.rowptr[i]; t < L->Z.rowptr[i + 1]; ++t) {
            block_apply(bs, L->Z.vals + (size_t)t * bs * bs, yc + (size_t)i * bs, tmp, 1);
            for (int32_t a = 0; a < bs; ++a) y[(size_t)L->Z.colidx[t] * bs + a] += tmp[a];
        }
    }
    free(sc);
    free(yc);
    free(work);
    free(tmp);
}

static void coarse_solve(const ora_hier *h, int32_t l, int fcyc, const double *rc, double *ec) {
    if (!fcyc) {
        cycle(h, l, 0, rc, ec);
        return;
    }
    const bsr_t *A = &h->lv[l].A;
    const int64_t n = (int64_t)A->nb * A->bs;
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double *e2 = (double *)malloc(sizeof(double) * (size_t)n);
    cycle(h, l, 1, rc, ec);
    for (int32_t I = 0; I < A->nb; ++I) block_row_residual(A, I, rc, ec, res + (size_t)I * A->bs);
    cycle(h, l, 0, res, e2);
    for (int64_t i = 0; i < n; ++i) ec[i] += e2[i];
    free(res);
    free(e2);
}

/* The transpose of coarse_solve: y_c = V^T s_c + F^T (s_c - A_c^T V^T s_c). */
static void coarse_solve_T(const ora_hier *h, int32_t l, int fcyc, const double *sc, double *yc) {
    if (!fcyc) {
        cycle_T(h, l, 0, sc, yc);
        return;
    }
    const bsr_t *A = &h->lv[l].A;
    const int64_t n = (int64_t)A->nb * A->bs;
    double *res = (double *)malloc(sizeof(double) * (size_t)n);
    double *y2 = (double *)malloc(sizeof(double) * (size_t)n);
    cycle_T(h, l, 0, sc, yc);
    residual_T(A, sc, yc, res);
    cycle_T(h, l, 1, res, y2);
    for (int64_t i = 0; i < n; ++i) yc[i] += y2[i];
    free(res);
    free(y2);
}

static void precondition(const ora_hier *h, int trans, const double *r, double *e);

int ora_vcycle(ora_hier *h, const double *r, double *e) {
    if (!h) return ORA_EINVAL;
    precondition(h, 0, r, e);
    return ORA_OK;
}

int ora_vcycle_T(ora_hier *h, const double *g, double *y) {
    if (!h) return ORA_EINVAL;
    precondition(h, 1, g, y);
    return ORA_OK;
}

static double norm2(const double *v, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* Stationary iteration x += B(b - A x) (or its transpose) from x = 0 with the
 * relative residual ||b - A x||_2 / ||b||_2 as the stopping test. */
/* The preconditioner applied to a residual: B r, or for the scalar form
 * B_S D^{-1} r (B_S the cycle of the scaled system); transposed: B^T r, or
 * D^{-T} B_S^T r. */
static void precondition(const ora_hier *h, int trans, const double *r, double *e) {
    const int f = h->prm.cycle == 1;
    if (h->prm.form != 1) {
        if (trans) cycle_T(h, 0, f, r, e);
        else cycle(h, 0, f, r, e);
        return;
    }
    const int32_t bs = h->A0.bs, bb = bs * bs;
    const int64_t n = (int64_t)h->A0.nb * bs;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!trans) {
        for (int32_t I = 0; I < h->A0.nb; ++I)
            block_apply(bs, h->d0inv + (size_t)I * bb, r + (size_t)I * bs, w + (size_t)I * bs, 0);
        cycle(h, 0, f, w, e);
    } else {
        cycle_T(h, 0, f, r, w);
        for (int32_t I = 0; I < h->A0.nb; ++I)
            block_apply(bs, h->d0inv + (size_t)I * bb, w + (size_t)I * bs, e + (size_t)I * bs, 1);
    }
    free(w);
}

static double dot(const double *u, const double *v, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += u[i] * v[i];
    return s;
}

/* y = A v (trans: A^T v) */
static void matvec(const bsr_t *A, int trans, const double *v, double *y) {
    const int64_t n = (int64_t)A->nb * A->bs;
    double *zero = (double *)calloc((size_t)n, sizeof(double));
    if (trans) residual_T(A, zero, v, y);
    else
        for (int32_t I = 0; I < A->nb; ++I) block_row_residual(A, I, zero, v, y + (size_t)I * A->bs);
    for (int64_t i = 0; i < n; ++i) y[i] = -y[i];
    free(zero);
}

/*
 * Right-preconditioned restarted GMRES(m) (Saad and Schultz) with the cycle B
 * as preconditioner: Arnoldi on A B with modified Gram-Schmidt, Givens
 * rotations of the Hessenberg matrix, x = x_0 + Z y with Z = B V kept.  The
 * history is the least-squares residual |g_{j+1}| / ||b|| of every inner step
 * (the true relative residual in exact arithmetic); each restart starts from
 * the true residual.
 */
static int gmres_impl(ora_hier *h, int trans, const double *b, double *x, double rtol, int32_t max_iter,
                      double *hist, int32_t *iters, double *relres) {
    const bsr_t *A = h->prm.form == 1 ? &h->A0 : &h->lv[0].A;
    const int64_t n = (int64_t)A->nb * A->bs;
    const int32_t m = h->prm.gmres;
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    double bn = norm2(b, n);
    if (!isfinite(bn)) return ORA_ENUMERIC;
    if (bn == 0.0) return ORA_OK;
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
    double *Z = (double *)malloc(sizeof(double) * (size_t)n * m);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));   /* H[i*m + j] */
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1)), *y = (double *)malloc(sizeof(double) * m);
    int st = ORA_ENOCONV;
    double rel = 1.0;
    int32_t it = 0;
    memcpy(w, b, sizeof(double) * (size_t)n);   /* r_0 = b (x_0 = 0) */
    while (it < max_iter) {
        const double beta = norm2(w, n);
        if (!isfinite(beta)) {
            st = ORA_ENUMERIC;
            break;
        }
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int32_t i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int32_t j = 0, done = 0;
        for (; j < m && it < max_iter; ++j) {
            precondition(h, trans, V + (size_t)j * n, Z + (size_t)j * n);
            matvec(A, trans, Z + (size_t)j * n, w);
            for (int32_t i = 0; i <= j; ++i) {
                const double hij = dot(w, V + (size_t)i * n, n);
                H[i * m + j] = hij;
                for (int64_t k = 0; k < n; ++k) w[k] -= hij * V[(size_t)i * n + k];
            }
            const double hn = norm2(w, n);
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0)
                for (int64_t k = 0; k < n; ++k) V[(size_t)(j + 1) * n + k] = w[k] / hn;
            for (int32_t i = 0; i < j; ++i) {   /* earlier rotations */
                const double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[j * m + j], c = H[(j + 1) * m + j];
            const double rho = sqrt(a * a + c * c);
            cs[j] = rho == 0.0 ? 1.0 : a / rho;
            sn[j] = rho == 0.0 ? 0.0 : c / rho;
            H[j * m + j] = rho;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            rel = fabs(g[j + 1]) / bn;
            if (hist) hist[it] = rel;
            ++it;
            if (!isfinite(rel)) {
                st = ORA_ENUMERIC;
                done = 1;
                ++j;
                break;
            }
            if (rel <= rtol || hn == 0.0) {
                done = 1;
                ++j;
                break;
            }
        }
        /* x += Z y, H[0:j, 0:j] y = g[0:j] (back substitution) */
        for (int32_t i = j - 1; i >= 0; --i) {
            double sacc = g[i];
            for (int32_t k = i + 1; k < j; ++k) sacc -= H[i * m + k] * y[k];
            y[i] = sacc / H[i * m + i];
        }
        for (int32_t i = 0; i < j; ++i)
            for (int64_t k = 0; k < n; ++k) x[k] += y[i] * Z[(size_t)i * n + k];
        if (st == ORA_ENUMERIC) break;
        /* the true residual for the restart (and the final status) */
        matvec(A, trans, x, w);
        for (int64_t k = 0; k < n; ++k) w[k] = b[k] - w[k];
        if (done) {
            st = (rel <= rtol) ? ORA_OK : ORA_ENOCONV;
            if (st != ORA_OK && norm2(w, n) / bn <= rtol) st = ORA_OK;
            break;
        }
    }
    if (iters) *iters = it;
    if (relres) *relres = rel;
    free(V);
    free(Z);
    free(w);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(y);
    return st;
}

static int solve_impl(ora_hier *h, int trans, const double *b, double *x, double rtol, int32_t max_iter,
                      double *hist, int32_t *iters, double *relres) {
    if (!h || !b || !x) return ORA_EINVAL;
    if (h->prm.gmres > 0) return gmres_impl(h, trans, b, x, rtol, max_iter, hist, iters, relres);
    const bsr_t *A = h->prm.form == 1 ? &h->A0 : &h->lv[0].A;
    int64_t n = (int64_t)A->nb * A->bs;
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    double bn = norm2(b, n);
    if (!isfinite(bn)) return ORA_ENUMERIC;
    if (bn == 0.0) return ORA_OK;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(r, b, sizeof(double) * (size_t)n);
    int st = ORA_ENOCONV;
    double rel = 1.0;
    int32_t it = 0;
    while (it < max_iter) {
        precondition(h, trans, r, e);
        for (int64_t i = 0; i < n; ++i) x[i] += e[i];
        if (trans) residual_T(A, b, x, r);
        else
            for (int32_t I = 0; I < A->nb; ++I) block_row_residual(A, I, b, x, r + (size_t)I * A->bs);
        rel = norm2(r, n) / bn;
        if (hist) hist[it] = rel;
        it++;
        if (!isfinite(rel)) {
            st = ORA_ENUMERIC;
            break;
        }
        if (rel <= rtol) {
            st = ORA_OK;
            break;
        }
    }
    if (iters) *iters = it;
    if (relres) *relres = rel;
    free(r);
    free(e);
    return st;
}

int ora_solve(ora_hier *h, const double *b, double *x, double rtol, int32_t max_iter, double *hist,
              int32_t *iters, double *relres) {
    return solve_impl(h, 0, b, x, rtol, max_iter, hist, iters, relres);
}

int ora_solve_T(ora_hier *h, const double *g, double *y, double rtol, int32_t max_iter, double *hist,
                int32_t *iters, double *relres) {
    return solve_impl(h, 1, g, y, rtol, max_iter, hist, iters, relres);
}

/* ---------------------------------------------------------------- queries */

int32_t ora_num_levels(const ora_hier *h) { return h ? h->nlev : 0; }

int ora_level(const ora_hier *h, int32_t lvl, ora_level_view *v) {
    if (!h || !v || lvl < 0 || lvl >= h->nlev) return ORA_EINVAL;
    const level_t *L = &h->lv[lvl];
    memset(v, 0, sizeof(*v));
    v->nb = L->A.nb;
    v->bs = L->A.bs;
    v->nnzb = L->A.rowptr[L->A.nb];
    v->coarsest = L->coarsest;
    v->rowptr = L->A.rowptr;
    v->colidx = L->A.colidx;
    v->vals = L->A.vals;
    v->dinv = L->dinv;
    v->bnorm = L->bnorm;
    v->mask = L->mask;
    v->lambda = L->lambda;
    v->cf = L->cf;
    v->cidx = L->cidx;
    v->dround = L->dround;
    v->pmap = L->coarsest ? NULL : L->pmap;
    v->nc = L->nc;
    v->pmis_rounds = L->pmis_rounds;
    if (!L->coarsest) {
        v->z_nnzb = L->Z.rowptr ? L->Z.rowptr[L->Z.nb] : 0;
        v->z_rowptr = L->Z.rowptr;
        v->z_colidx = L->Z.colidx;
        v->z_vals = L->Z.vals;
    }
    v->dense_n = L->dense_n;
    v->dense_lu = L->lu;
    v->dense_piv = L->piv;
    for (int k = 0; k < 4; ++k) v->margin[k] = L->margin[k];
    return ORA_OK;
}

/*
 * Complexities in work units (section 6: one WU = one SpMV with A_0).
 * OC = sum_l nnzb_l / nnzb_0.  CC (a reading; the paper gives only the
 * definition) = 1 (outer residual) + sum over non-coarsest levels of
 * [nu * nnzb(F rows) + FC * nnzb(C rows) + nnzb(Z) + nb_F] / nnzb_0, plus the
 * coarsest level's dense solve counted as dense_n^2 / (bs^2 nnzb_0).
 */
void ora_complexity(const ora_hier *h, double *oc, double *cc) {
    double nnz0 = (double)h->lv[0].A.rowptr[h->lv[0].A.nb];
    double o = 0.0;
    int32_t nu = h->prm.degree + 1;
    double w[ORA_MAX_LEVELS], nz[ORA_MAX_LEVELS];   /* per-level V-cycle work, operator size */
    for (int32_t l = 0; l < h->nlev; ++l) {
        const level_t *L = &h->lv[l];
        nz[l] = (double)L->A.rowptr[L->A.nb] / nnz0;
        o += nz[l];
        if (L->coarsest) {
            double bb = (double)L->A.bs * L->A.bs;
            w[l] = (double)L->dense_n * L->dense_n / bb / nnz0;
            continue;
        }
        double nzF = 0.0, nzC = 0.0, nbF = 0.0;
        for (int32_t I = 0; I < L->A.nb; ++I) {
            double rn = (double)(L->A.rowptr[I + 1] - L->A.rowptr[I]);
            if (L->cf[I] == 1) nzC += rn;
            else {
                nzF += rn;
                nbF += 1.0;
            }
        }
        w[l] = (nu * nzF + (h->prm.relax == 1 ? nzC : 0.0) + (double)L->Z.rowptr[L->Z.nb] + nbF) / nnz0;
    }
    /* V: each level once.  F: a level's coarse solve is an F-cycle, a residual
     * with the coarse operator and a V-cycle, recursively. */
    double cv = 0.0, cf = 0.0;
    for (int32_t l = h->nlev - 1; l >= 0; --l) {
        if (l == h->nlev - 1) {
            cv = w[l];
            cf = w[l];
        } else {
            cf = w[l] + cf + nz[l + 1] + cv;
            cv = w[l] + cv;
        }
    }
    if (oc) *oc = o;
    if (cc) *cc = 1.0 + (h->prm.cycle == 1 ? cf : cv);
}
