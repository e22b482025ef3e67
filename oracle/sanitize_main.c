/*
 * Driver of the sanitizer build of the reference CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer together with tmm_oracle.c, it reads one set of
 * inputs from a file, runs every entry point of the oracle on them and writes
 * the results to a second file, so that a test can compare them with the plain
 * build.  Any out-of-bounds access, use after free, leak or undefined
 * operation in the oracle stops the program with a report.
 *
 * Input (native byte order): eleven int32
 *   n ncol nlayer nmat nstep model neuphotic nbgc ae_nnz ai_nnz nbatch
 * then col_start, lat, area, dz, ae_rowptr, ae_colidx, ae_val, ai_rowptr,
 * ai_colidx, ai_val, u [nbatch][nparam], y0, v, wbar (n x W each) and
 * obs [nmat][n][W].
 * Output (float64, in this order): step 0, step nstep/2, one year, its
 * residuals [nbatch], tangent phi and jv, FD phi and jv, misfit J [nbatch],
 * adjoint J, dJdu, dJdy0, vjp ybar and ubar.
 */
#include "oracle.h"

#include <stdio.h>
#include <stdlib.h>

static void *take(FILE *f, size_t count, size_t size)
{
    void *p = malloc(count * size > 0 ? count * size : 1);
    if (!p || fread(p, size, count, f) != count) {
        fprintf(stderr, "sanitize_main: short input\n");
        exit(2);
    }
    return p;
}

static void put(FILE *f, const double *x, size_t count)
{
    if (fwrite(x, sizeof(double), count, f) != count) {
        fprintf(stderr, "sanitize_main: write failed\n");
        exit(2);
    }
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int *hd = take(in, 11, sizeof(int));
    oracle_desc g;
    g.n = hd[0]; g.ncol = hd[1]; g.nlayer = hd[2]; g.nmat = hd[3]; g.nstep = hd[4];
    g.model = hd[5]; g.neuphotic = hd[6]; g.nbgc = hd[7]; g.ae_nnz = hd[8]; g.ai_nnz = hd[9];
    int nbatch = hd[10];
    int ntr = oracle_ntracer(g.model), np = oracle_nparam(g.model);
    if (ntr < 1 || nbatch < 1) return 2;
    size_t len = (size_t)g.n * nbatch * ntr;
    int *col_start = take(in, g.ncol + 1, sizeof(int));
    double *lat = take(in, g.ncol, sizeof(double));
    double *area = take(in, g.ncol, sizeof(double));
    double *dz = take(in, g.nlayer, sizeof(double));
    int *ae_rowptr = take(in, g.n + 1, sizeof(int));
    int *ae_colidx = take(in, g.ae_nnz, sizeof(int));
    double *ae_val = take(in, (size_t)g.nmat * g.ae_nnz, sizeof(double));
    int *ai_rowptr = take(in, g.n + 1, sizeof(int));
    int *ai_colidx = take(in, g.ai_nnz, sizeof(int));
    double *ai_val = take(in, (size_t)g.nmat * g.ai_nnz, sizeof(double));
    double *u = take(in, (size_t)nbatch * np, sizeof(double));
    double *y0 = take(in, len, sizeof(double));
    double *v = take(in, len, sizeof(double));
    double *wbar = take(in, len, sizeof(double));
    double *obs = take(in, (size_t)g.nmat * len, sizeof(double));
    fclose(in);
    g.col_start = col_start; g.lat = lat; g.area = area; g.dz = dz;
    g.ae_rowptr = ae_rowptr; g.ae_colidx = ae_colidx; g.ae_val = ae_val;
    g.ai_rowptr = ai_rowptr; g.ai_colidx = ai_colidx; g.ai_val = ai_val;

    double *a = malloc(sizeof(double) * len), *b = malloc(sizeof(double) * len);
    double *r = malloc(sizeof(double) * nbatch), *J = malloc(sizeof(double) * nbatch);
    double *G = malloc(sizeof(double) * (size_t)nbatch * np);
    FILE *out = fopen(argv[2], "wb");
    if (!a || !b || !r || !J || !G || !out) return 2;
    int rc = 0;
    rc |= oracle_step(&g, nbatch, u, 0, y0, a);
    put(out, a, len);
    rc |= oracle_step(&g, nbatch, u, g.nstep / 2, y0, a);
    put(out, a, len);
    rc |= oracle_year(&g, nbatch, u, 1, y0, a, r);
    put(out, a, len);
    put(out, r, nbatch);
    rc |= oracle_year_tangent(&g, nbatch, u, y0, v, a, b);
    put(out, a, len);
    put(out, b, len);
    rc |= oracle_year_jvp_fd(&g, nbatch, u, y0, v, a, b);
    put(out, a, len);
    put(out, b, len);
    rc |= oracle_year_misfit(&g, nbatch, u, y0, obs, J);
    put(out, J, nbatch);
    rc |= oracle_year_adjoint(&g, nbatch, u, y0, obs, J, G, a);
    put(out, J, nbatch);
    put(out, G, (size_t)nbatch * np);
    put(out, a, len);
    rc |= oracle_year_vjp(&g, nbatch, u, y0, wbar, a, G);
    put(out, a, len);
    put(out, G, (size_t)nbatch * np);
    fclose(out);
    free(a); free(b); free(r); free(J); free(G);
    free(hd); free(col_start); free(lat); free(area); free(dz);
    free(ae_rowptr); free(ae_colidx); free(ae_val); free(ai_rowptr); free(ai_colidx); free(ai_val);
    free(u); free(y0); free(v); free(wbar); free(obs);
    if (rc) {
        fprintf(stderr, "sanitize_main: an oracle entry point failed\n");
        return 1;
    }
    return 0;
}
