/* Host sanitizer run of the C oracle (built with -fsanitize=address,undefined):
 * exercises every exported routine on a small scan and checks identities that
 * hold exactly (brute force == Siddon, <Ax, y> == <x, A^T y>, sampled rows and
 * columns == the CSR matrix, CG residual).  Exit status 0 = clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t nx, ny, nz, nu, nv;
    int32_t pad_;
    double du, dv, src_iso, src_det, off_u, off_v;
} or_geom;

void or_ray(const or_geom *g, double theta, int32_t iu, int32_t iv, double *S, double *D);
int32_t or_brute(const or_geom *g, const double *S, const double *D, int32_t *idx, double *len, int32_t cap);
int32_t or_siddon(const or_geom *g, const double *S, const double *D, int32_t *idx, double *len, int32_t cap);
int64_t or_csr_count(const or_geom *g, const double *angles, int32_t nviews, int32_t method, int64_t *rowptr);
void or_csr_fill(const or_geom *g, const double *angles, int32_t nviews, int32_t method, const int64_t *rowptr,
                 int32_t *col, double *val);
void or_csr_transpose(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col, const double *val,
                      int64_t *trp, int32_t *tcol, double *tval);
void or_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val, const double *x, double *y);
int32_t or_prox_cg(int64_t nr, int64_t nc, const int64_t *rp, const int32_t *ci, const double *va,
                   const int64_t *trp, const int32_t *tci, const double *tva, const double *lam, const double *y,
                   const double *v, double sigma, const double *x0, double tol, int32_t max_iter, double *x,
                   double *out_stats);
void or_backproject_voxels(const or_geom *g, const double *angles, int32_t nviews, const double *y,
                           const int64_t *vox, int32_t nsel, double *out);
void or_voxel_columns(const or_geom *g, const double *angles, int32_t nviews, const int64_t *vox, int32_t nsel,
                      int32_t *count, int64_t *ray, double *len, int32_t cap);
void or_project_rays(const or_geom *g, const double *angles, const int32_t *view, const int32_t *iv,
                     const int32_t *iu, int32_t nsel, const double *x, double *out);
int32_t or_num_threads(void);
void or_set_num_threads(int32_t n);

static int failures = 0;
static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

int main(void)
{
    const or_geom g = {10, 9, 8, 14, 12, 0, 2.0, 2.0, 60.0, 120.0, 0.3, -0.2};
    const double angles[3] = {0.1, 1.3, 2.9};
    const int nviews = 3;
    const int64_t nrows = (int64_t)nviews * g.nv * g.nu, ncols = (int64_t)g.nx * g.ny * g.nz;
    uint64_t seed = 12345;

    /* brute force and Siddon give the same ray (total length and every voxel) */
    const int cap = g.nx * g.ny * g.nz;
    int32_t *ia = malloc(sizeof(int32_t) * cap), *ib = malloc(sizeof(int32_t) * cap);
    double *la = malloc(sizeof(double) * cap), *lb = malloc(sizeof(double) * cap);
    for (int v = 0; v < nviews; v++)
        for (int iv = 0; iv < g.nv; iv++)
            for (int iu = 0; iu < g.nu; iu++) {
                double S[3], D[3];
                or_ray(&g, angles[v], iu, iv, S, D);
                int na = or_brute(&g, S, D, ia, la, cap);
                int nb = or_siddon(&g, S, D, ib, lb, g.nx + g.ny + g.nz + 4);
                double sa = 0.0, sb = 0.0;
                for (int k = 0; k < na; k++) sa += la[k];
                for (int k = 0; k < nb; k++) sb += lb[k];
                check(fabs(sa - sb) <= 1e-12 * (1.0 + sa), "brute == siddon (ray length)");
            }

    /* CSR by both methods, transpose, dot-product test */
    int64_t *rp = malloc(sizeof(int64_t) * (nrows + 1)), *rp2 = malloc(sizeof(int64_t) * (nrows + 1));
    int64_t nnz = or_csr_count(&g, angles, nviews, 0, rp);
    int64_t nnz2 = or_csr_count(&g, angles, nviews, 1, rp2);
    check(nnz > 0 && nnz == nnz2, "nnz of both routes");
    int32_t *ci = malloc(sizeof(int32_t) * nnz), *ci2 = malloc(sizeof(int32_t) * nnz2);
    double *va = malloc(sizeof(double) * nnz), *va2 = malloc(sizeof(double) * nnz2);
    or_csr_fill(&g, angles, nviews, 0, rp, ci, va);
    or_csr_fill(&g, angles, nviews, 1, rp2, ci2, va2);
    int64_t *trp = malloc(sizeof(int64_t) * (ncols + 1));
    int32_t *tci = malloc(sizeof(int32_t) * nnz);
    double *tva = malloc(sizeof(double) * nnz);
    or_csr_transpose(nrows, ncols, rp, ci, va, trp, tci, tva);
    double *x = malloc(sizeof(double) * ncols), *y = malloc(sizeof(double) * nrows);
    double *ax = malloc(sizeof(double) * nrows), *aty = malloc(sizeof(double) * ncols);
    double *ax2 = malloc(sizeof(double) * nrows);
    for (int64_t i = 0; i < ncols; i++) x[i] = urand(&seed) - 0.5;
    for (int64_t i = 0; i < nrows; i++) y[i] = urand(&seed) - 0.5;
    or_spmv(nrows, rp, ci, va, x, ax);
    or_spmv(nrows, rp2, ci2, va2, x, ax2);
    or_spmv(ncols, trp, tci, tva, y, aty);
    double d1 = 0.0, d2 = 0.0, dd = 0.0, n2 = 0.0;
    for (int64_t i = 0; i < nrows; i++) {
        d1 += ax[i] * y[i];
        dd += (ax[i] - ax2[i]) * (ax[i] - ax2[i]);
        n2 += ax[i] * ax[i];
    }
    for (int64_t i = 0; i < ncols; i++) d2 += x[i] * aty[i];
    check(fabs(d1 - d2) <= 1e-12 * fabs(d1), "dot-product test");
    check(sqrt(dd) <= 1e-12 * sqrt(n2), "siddon CSR == brute-force CSR");

    /* sampled rays and voxels against the CSR matrix */
    int32_t sv[4] = {0, 1, 2, 1}, siv[4] = {3, 6, 5, 11}, siu[4] = {2, 7, 9, 13};
    double pr[4];
    or_project_rays(&g, angles, sv, siv, siu, 4, x, pr);
    for (int s = 0; s < 4; s++) {
        int64_t r = ((int64_t)sv[s] * g.nv + siv[s]) * g.nu + siu[s];
        check(fabs(pr[s] - ax[r]) <= 1e-12 * (1.0 + fabs(ax[r])), "sampled ray == CSR row");
    }
    int64_t vox[3] = {0, ncols / 2 + 3, ncols - 5};
    double bv[3];
    or_backproject_voxels(&g, angles, nviews, y, vox, 3, bv);
    for (int s = 0; s < 3; s++) check(fabs(bv[s] - aty[vox[s]]) <= 1e-12 * (1.0 + fabs(aty[vox[s]])),
                                      "sampled voxel == CSR column");
    const int ccap = 256;
    int32_t cnt[3];
    int64_t *cray = malloc(sizeof(int64_t) * 3 * ccap);
    double *clen = malloc(sizeof(double) * 3 * ccap);
    or_voxel_columns(&g, angles, nviews, vox, 3, cnt, cray, clen, ccap);
    for (int s = 0; s < 3; s++) {
        int64_t want = trp[vox[s] + 1] - trp[vox[s]];
        check(cnt[s] == want, "voxel column length == CSR column");
    }

    /* proximal-map CG: converges, the true residual agrees */
    double *lam = malloc(sizeof(double) * nrows), *v = malloc(sizeof(double) * ncols);
    double *xs = malloc(sizeof(double) * ncols), st[4];
    for (int64_t i = 0; i < nrows; i++) lam[i] = 0.5 + urand(&seed);
    for (int64_t i = 0; i < ncols; i++) v[i] = urand(&seed);
    int it = or_prox_cg(nrows, ncols, rp, ci, va, trp, tci, tva, lam, y, v, 0.5, NULL, 1e-10, 5000, xs, st);
    check(it > 0 && st[1] <= 1e-10 && st[2] <= 1e-9, "prox CG converges");
    int32_t th = or_num_threads();
    or_set_num_threads(1);
    check(or_num_threads() == 1, "thread count set");
    or_set_num_threads(th);

    free(ia); free(ib); free(la); free(lb); free(rp); free(rp2); free(ci); free(ci2); free(va); free(va2);
    free(trp); free(tci); free(tva); free(x); free(y); free(ax); free(aty); free(ax2); free(cray); free(clen);
    free(lam); free(v); free(xs);
    if (failures) return 1;
    printf("oracle sanitizer run: clean (nnz %lld, CG %d iterations)\n", (long long)nnz, it);
    return 0;
}
