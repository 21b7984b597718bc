/*
 * Test driver for the C oracle (no Python): reads one LP, a reference point
 * and run parameters from a binary file, runs the oracle's PDHG solve, KKT
 * evaluation and both fix-and-propagate roundings, and writes the results
 * as raw arrays.  Built with AddressSanitizer / UBSan by the tests, which
 * compare its outputs with the regular build's.
 *
 * Input:  int32 m, n; int64 nnz; int64 row_ptr[m+1]; int32 col_idx[nnz];
 *         double val[nnz], c[n], b[m]; uint8 sense[m]; double l[n], u[n];
 *         uint8 is_int[n]; double x_ref[n];
 *         double tol; int64 iter_limit; int32 check_period, restarts,
 *         adaptive, K (batched rounding).
 * Output: double x[n], y[m]; int32 status, restarts; int64 iterations;
 *         double rel, rho_p, rho_d, rho_g, pobj, dobj, omega, eta;
 *         double kkt[8]; double xhat[n]; int32 info[2];
 *         double xhat_b[n]; int32 info_b[2]; uint8 mask[max(m,1)].
 */
#include "../../oracle/scylla_oracle.c"

#include <stdio.h>

static void *rd(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (bytes && fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 1;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t mn[2];
    int64_t nnz;
    if (fread(mn, 4, 2, f) != 2 || fread(&nnz, 8, 1, f) != 1) return 2;
    const int32_t m = mn[0], n = mn[1];
    int64_t *row_ptr = rd(f, 8 * (size_t)(m + 1));
    int32_t *col = rd(f, 4 * (size_t)nnz);
    double *val = rd(f, 8 * (size_t)nnz);
    double *c = rd(f, 8 * (size_t)n), *b = rd(f, 8 * (size_t)m);
    char *sense = rd(f, (size_t)m);
    double *l = rd(f, 8 * (size_t)n), *u = rd(f, 8 * (size_t)n);
    uint8_t *is_int = rd(f, (size_t)n);
    double *xref = rd(f, 8 * (size_t)n);
    double tol;
    int64_t iter_limit;
    int32_t ip[4];
    if (fread(&tol, 8, 1, f) != 1 || fread(&iter_limit, 8, 1, f) != 1 || fread(ip, 4, 4, f) != 4) return 2;
    fclose(f);

    orc_lp lp = {m, n, row_ptr, col, val, c, b, sense, l, u, NULL};
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.tol = tol;
    p.iter_limit = iter_limit;
    p.check_period = ip[0];
    p.restarts = ip[1];
    p.eta = 0.99;
    p.ruiz_iters = 10;
    p.pock_chambolle = 1;
    p.adaptive = ip[2];
    p.infeas_tol = 1e-8;
    p.stall_checks = 3;
    double *x = malloc(8 * (size_t)(n ? n : 1)), *y = malloc(8 * (size_t)(m ? m : 1));
    orc_result res;
    if (orc_pdhg(&lp, &p, NULL, NULL, x, y, &res)) return 3;
    double kkt[8];
    orc_kkt(&lp, x, y, kkt);
    double *xh = malloc(8 * (size_t)(n ? n : 1)), *xb = malloc(8 * (size_t)(n ? n : 1));
    int32_t info[2], info_b[2];
    uint8_t *mask = calloc((size_t)(m ? m : 1), 1);
    if (orc_fix_propagate(&lp, is_int, xref, xh, info)) return 4;
    if (orc_fix_propagate_batched(&lp, is_int, xref, ip[3], 1000, xb, info_b, mask)) return 5;

    FILE *o = fopen(argv[2], "wb");
    if (!o) return 6;
    fwrite(x, 8, (size_t)n, o);
    fwrite(y, 8, (size_t)m, o);
    fwrite(&res.status, 4, 1, o);
    fwrite(&res.restarts, 4, 1, o);
    fwrite(&res.iterations, 8, 1, o);
    const double rv[8] = {res.rel_kkt, res.rho_p, res.rho_d, res.rho_g, res.pobj, res.dobj, res.omega, res.eta};
    fwrite(rv, 8, 8, o);
    fwrite(kkt, 8, 8, o);
    fwrite(xh, 8, (size_t)n, o);
    fwrite(info, 4, 2, o);
    fwrite(xb, 8, (size_t)n, o);
    fwrite(info_b, 4, 2, o);
    fwrite(mask, 1, (size_t)(m ? m : 1), o);
    fclose(o);
    free(row_ptr); free(col); free(val); free(c); free(b); free(sense); free(l); free(u);
    free(is_int); free(xref); free(x); free(y); free(xh); free(xb); free(mask);
    return 0;
}
