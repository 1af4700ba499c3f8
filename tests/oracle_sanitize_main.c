/*
 * Driver that runs the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure; built and run by
 * tests/test_oracle_sanitize.py with gcc on the host, never on a GPU).
 *
 * Input file (native endianness): int32 nb, bs, nnzb, nvar; rowptr[nb+1],
 * colidx[nnzb] (int32); vals[nnzb*bs*bs], rhs[nb*bs] (double); then nvar
 * records of int32 {degree, relax, cycle, gmres, form}.
 * For every record it builds the hierarchy, reads every level view, computes
 * the complexities, applies both cycles and solves A x = b and A^T y = b to
 * 1e-10; it writes, per record, int32 {status, iters, status_T, iters_T,
 * levels} and then x and y (double[nb*bs] each) to the output file.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nair_oracle.h"

static void *read_n(FILE *f, size_t n, size_t sz) {
    void *p = malloc(n * sz > 0 ? n * sz : 1);
    if (!p || fread(p, sz, n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t *hdr = (int32_t *)read_n(f, 4, sizeof(int32_t));
    int32_t nb = hdr[0], bs = hdr[1], nnzb = hdr[2], nvar = hdr[3];
    int32_t *rowptr = (int32_t *)read_n(f, (size_t)nb + 1, sizeof(int32_t));
    int32_t *colidx = (int32_t *)read_n(f, (size_t)nnzb, sizeof(int32_t));
    double *vals = (double *)read_n(f, (size_t)nnzb * bs * bs, sizeof(double));
    size_t n = (size_t)nb * bs;
    double *rhs = (double *)read_n(f, n, sizeof(double));
    int32_t *var = (int32_t *)read_n(f, (size_t)nvar * 5, sizeof(int32_t));
    fclose(f);

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 2;
    double *x = (double *)calloc(n, sizeof(double));
    double *y = (double *)calloc(n, sizeof(double));
    double *e = (double *)calloc(n, sizeof(double));
    double *hist = (double *)calloc(200, sizeof(double));
    for (int32_t v = 0; v < nvar; ++v) {
        ora_params p;
        ora_default_params(&p);
        p.degree = var[5 * v + 0];
        p.relax = var[5 * v + 1];
        p.cycle = var[5 * v + 2];
        p.gmres = var[5 * v + 3];
        p.form = var[5 * v + 4];
        p.max_coarse_dofs = 16;
        ora_hier *h = NULL;
        int st = ora_setup(nb, bs, rowptr, colidx, vals, &p, &h);
        if (st != ORA_OK) {
            fprintf(stderr, "setup failed: %d\n", st);
            return 3;
        }
        int32_t levels = ora_num_levels(h);
        double check = 0.0;
        for (int32_t l = 0; l < levels; ++l) {
            ora_level_view lv;
            if (ora_level(h, l, &lv) != ORA_OK) return 4;
            /* touch every array of the view */
            for (int64_t t = 0; t < (int64_t)lv.nnzb * lv.bs * lv.bs; ++t) check += lv.vals[t];
            if (lv.dinv)
                for (int64_t t = 0; t < (int64_t)lv.nb * lv.bs * lv.bs; ++t) check += lv.dinv[t];
            if (lv.z_vals)
                for (int64_t t = 0; t < (int64_t)lv.z_nnzb * lv.bs * lv.bs; ++t) check += lv.z_vals[t];
            if (lv.dense_lu)
                for (int64_t t = 0; t < (int64_t)lv.dense_n * lv.dense_n; ++t) check += lv.dense_lu[t];
        }
        double oc = 0.0, cc = 0.0;
        ora_complexity(h, &oc, &cc);
        if (ora_vcycle(h, rhs, e) != ORA_OK || ora_vcycle_T(h, rhs, e) != ORA_OK) return 5;
        int32_t it = 0, itT = 0;
        double rel = 0.0, relT = 0.0;
        int stx = ora_solve(h, rhs, x, 1e-10, 200, hist, &it, &rel);
        int sty = ora_solve_T(h, rhs, y, 1e-10, 200, hist, &itT, &relT);
        int32_t rec[5] = {stx, it, sty, itT, levels};
        fwrite(rec, sizeof(int32_t), 5, o);
        fwrite(x, sizeof(double), n, o);
        fwrite(y, sizeof(double), n, o);
        printf("variant %d: levels %d oc %.3f cc %.3f iters %d/%d check %.3e\n", v, levels, oc, cc, it, itT,
               check);
        ora_free(h);
    }
    fclose(o);
    free(x);
    free(y);
    free(e);
    free(hist);
    free(hdr);
    free(rowptr);
    free(colidx);
    free(vals);
    free(rhs);
    free(var);
    return 0;
}
