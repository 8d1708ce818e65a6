/*
 * FP64 CPU oracle for the forward-model proximal map of multi-slice fusion.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the HIP library: it is plain, slow and written to be checked by eye.
 *
 * What it computes (paper Sec. II, eq. (2), and Sec. III,
 * eq. (4)):  for every time frame n the data term is
 *     l_n(x) = 1/2 || y_n - A_n x ||^2_{Lambda_n}
 * and the proximal map of the data term is the minimiser of
 *     l_n(z) + ||x - z||^2 / (2 sigma^2),
 * i.e. the solution of (A^T Lambda A + sigma^-2 I) z = A^T Lambda y + sigma^-2 x.
 *
 * A_n[i][j] is the length of the segment (point source -> centre of detector
 * pixel i) inside voxel j.  The paper does not fix the discretisation of its
 * system matrix, so this exact ray-voxel length is the reading taken here.
 * Two independent routes produce the same matrix:
 *   - or_brute:  every voxel's half-open cube clipped against the segment
 *                (slab test), O(voxels) per ray;
 *   - or_siddon: Siddon's merged-plane-crossing method (Siddon, Med. Phys.
 *                12(2), 1985): all x/y/z plane crossings of the segment,
 *                sorted; each gap is one voxel, found from its midpoint.
 * A^T is the transpose of the same CSR matrix, so the adjoint is exact.
 *
 * Geometry (voxel units, voxel side 1, origin at the volume centre):
 *   voxel (i,j,k) spans [i - nx/2, i + 1 - nx/2) x ... (half-open);
 *   source  S = (R_s cos t, R_s sin t, 0);
 *   detector centre D0 = S + R_sd (-cos t, -sin t, 0);
 *   e_u = (-sin t, cos t, 0), e_v = (0, 0, 1);
 *   pixel (iu, iv) centre = D0 + u e_u + v e_v with
 *   u = (iu - (nu-1)/2) du + off_u,  v = (iv - (nv-1)/2) dv + off_v.
 * Rows of a view are ordered iv-major (u fastest); voxel indices are
 * k*ny*nx + j*nx + i (x fastest).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz, nu, nv;
    int32_t pad_;
    double du, dv, src_iso, src_det, off_u, off_v;
} or_geom;

/* ---------------------------------------------------------------- rays -- */

void or_ray(const or_geom *g, double theta, int32_t iu, int32_t iv, double *S, double *D)
{
    double c = cos(theta), s = sin(theta);
    double u = (iu - 0.5 * (g->nu - 1)) * g->du + g->off_u;
    double v = (iv - 0.5 * (g->nv - 1)) * g->dv + g->off_v;
    S[0] = g->src_iso * c;
    S[1] = g->src_iso * s;
    S[2] = 0.0;
    double d0x = S[0] - g->src_det * c;
    double d0y = S[1] - g->src_det * s;
    D[0] = d0x - u * s;
    D[1] = d0y + u * c;
    D[2] = v;
}

/* ------------------------------------------------------------ brute force */

/* Parametric interval of the segment S + a (D - S), a in [0,1], inside the
 * half-open slab [lo, hi) of one axis.  Returns 0 if empty. */
static int slab(double s, double d, double lo, double hi, double *a0, double *a1)
{
    if (d == 0.0) {
        if (s >= lo && s < hi) { *a0 = -INFINITY; *a1 = INFINITY; return 1; }
        return 0;
    }
    double t0 = (lo - s) / d, t1 = (hi - s) / d;
    if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
    *a0 = t0;
    *a1 = t1;
    return 1;
}

/* All voxels crossed by the segment, by clipping the segment against every
 * voxel cube.  Returns the number of entries written (at most cap). */
int32_t or_brute(const or_geom *g, const double *S, const double *D, int32_t *idx, double *len, int32_t cap)
{
    double d[3] = {D[0] - S[0], D[1] - S[1], D[2] - S[2]};
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int n = 0;
    for (int k = 0; k < g->nz; k++) {
        double zlo = k - 0.5 * g->nz;
        double za0, za1;
        if (!slab(S[2], d[2], zlo, zlo + 1.0, &za0, &za1)) continue;
        for (int j = 0; j < g->ny; j++) {
            double ylo = j - 0.5 * g->ny;
            double ya0, ya1;
            if (!slab(S[1], d[1], ylo, ylo + 1.0, &ya0, &ya1)) continue;
            for (int i = 0; i < g->nx; i++) {
                double xlo = i - 0.5 * g->nx;
                double xa0, xa1;
                if (!slab(S[0], d[0], xlo, xlo + 1.0, &xa0, &xa1)) continue;
                double a0 = fmax(fmax(0.0, xa0), fmax(ya0, za0));
                double a1 = fmin(fmin(1.0, xa1), fmin(ya1, za1));
                if (a1 > a0 && n < cap) {
                    idx[n] = (k * g->ny + j) * g->nx + i;
                    len[n] = (a1 - a0) * L;
                    n++;
                }
            }
        }
    }
    return n;
}

/* -------------------------------------------------------------- Siddon -- */

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int32_t or_siddon(const or_geom *g, const double *S, const double *D, int32_t *idx, double *len, int32_t cap)
{
    int nn[3] = {g->nx, g->ny, g->nz};
    double d[3] = {D[0] - S[0], D[1] - S[1], D[2] - S[2]};
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    /* parametric range of the segment inside the volume box */
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; a++) {
        double a0, a1;
        if (!slab(S[a], d[a], -0.5 * nn[a], 0.5 * nn[a], &a0, &a1)) return 0;
        amin = fmax(amin, a0);
        amax = fmin(amax, a1);
    }
    if (!(amax > amin)) return 0;
    /* every plane crossing strictly inside (amin, amax), plus the two ends */
    int cnt = 2 + nn[0] + nn[1] + nn[2] + 3;
    double *al = (double *)malloc(sizeof(double) * cnt);
    int m = 0;
    al[m++] = amin;
    al[m++] = amax;
    for (int a = 0; a < 3; a++) {
        if (d[a] == 0.0) continue;
        for (int p = 0; p <= nn[a]; p++) {
            double t = (p - 0.5 * nn[a] - S[a]) / d[a];
            if (t > amin && t < amax) al[m++] = t;
        }
    }
    qsort(al, m, sizeof(double), cmp_double);
    int n = 0;
    for (int q = 0; q + 1 < m; q++) {
        if (!(al[q + 1] > al[q])) continue;
        double mid = 0.5 * (al[q] + al[q + 1]);
        int ii[3];
        int ok = 1;
        for (int a = 0; a < 3; a++) {
            double pos = S[a] + mid * d[a] + 0.5 * nn[a];
            ii[a] = (int)floor(pos);
            if (ii[a] < 0 || ii[a] >= nn[a]) ok = 0;
        }
        if (!ok || n >= cap) continue;
        idx[n] = (ii[2] * g->ny + ii[1]) * g->nx + ii[0];
        len[n] = (al[q + 1] - al[q]) * L;
        n++;
    }
    free(al);
    return n;
}

/* Length of the segment inside one voxel (slab test on one cube). */
double or_voxel_length(const or_geom *g, const double *S, const double *D, int64_t vox)
{
    int i = (int)(vox % g->nx);
    int j = (int)((vox / g->nx) % g->ny);
    int k = (int)(vox / ((int64_t)g->nx * g->ny));
    double d[3] = {D[0] - S[0], D[1] - S[1], D[2] - S[2]};
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double lo[3] = {i - 0.5 * g->nx, j - 0.5 * g->ny, k - 0.5 * g->nz};
    double a0 = 0.0, a1 = 1.0;
    for (int a = 0; a < 3; a++) {
        double t0, t1;
        if (!slab(S[a], d[a], lo[a], lo[a] + 1.0, &t0, &t1)) return 0.0;
        a0 = fmax(a0, t0);
        a1 = fmin(a1, t1);
    }
    return a1 > a0 ? (a1 - a0) * L : 0.0;
}

/* ----------------------------------------------------------------- CSR -- */

static int32_t row_entries(const or_geom *g, int method, double theta, int iu, int iv,
                           int32_t *idx, double *len, int32_t cap)
{
    double S[3], D[3];
    or_ray(g, theta, iu, iv, S, D);
    return method ? or_brute(g, S, D, idx, len, cap) : or_siddon(g, S, D, idx, len, cap);
}

/* Row pointer of the system matrix of one frame (its nviews views); method 0
 * = Siddon, 1 = brute force.  rowptr has nviews*nv*nu + 1 entries. */
int64_t or_csr_count(const or_geom *g, const double *angles, int32_t nviews, int32_t method, int64_t *rowptr)
{
    int64_t nr = (int64_t)nviews * g->nv * g->nu;
    int cap = g->nx + g->ny + g->nz + 4;
    if (method) cap = g->nx * g->ny * g->nz;
    rowptr[0] = 0;
#pragma omp parallel
    {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nr; r++) {
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            rowptr[r + 1] = row_entries(g, method, angles[view], rem % g->nu, rem / g->nu, idx, len, cap);
        }
        free(idx);
        free(len);
    }
    for (int64_t r = 0; r < nr; r++) rowptr[r + 1] += rowptr[r];
    return rowptr[nr];
}

void or_csr_fill(const or_geom *g, const double *angles, int32_t nviews, int32_t method,
                 const int64_t *rowptr, int32_t *col, double *val)
{
    int64_t nr = (int64_t)nviews * g->nv * g->nu;
    int cap = g->nx + g->ny + g->nz + 4;
    if (method) cap = g->nx * g->ny * g->nz;
#pragma omp parallel
    {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nr; r++) {
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            int n = row_entries(g, method, angles[view], rem % g->nu, rem / g->nu, idx, len, cap);
            memcpy(col + rowptr[r], idx, sizeof(int32_t) * n);
            memcpy(val + rowptr[r], len, sizeof(double) * n);
        }
        free(idx);
        free(len);
    }
}

/* CSR of the transpose (counting sort by column). */
void or_csr_transpose(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *col, const double *val,
                      int64_t *trowptr, int32_t *tcol, double *tval)
{
    memset(trowptr, 0, sizeof(int64_t) * (ncols + 1));
    int64_t nnz = rowptr[nrows];
    for (int64_t e = 0; e < nnz; e++) trowptr[col[e] + 1]++;
    for (int64_t c = 0; c < ncols; c++) trowptr[c + 1] += trowptr[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ncols + 1));
    memcpy(fill, trowptr, sizeof(int64_t) * (ncols + 1));
    for (int64_t r = 0; r < nrows; r++)
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; e++) {
            int64_t p = fill[col[e]]++;
            tcol[p] = (int32_t)r;
            tval[p] = val[e];
        }
    free(fill);
}

/* y = M x for a CSR matrix M. */
void or_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; r++) {
        double s = 0.0;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; e++) s += val[e] * x[col[e]];
        y[r] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* H p = A^T (Lambda (A p)) + p / sigma^2, with scratch t of length nrows. */
static void apply_h(int64_t nr, int64_t nc, const int64_t *rp, const int32_t *ci, const double *va,
                    const int64_t *trp, const int32_t *tci, const double *tva, const double *lam,
                    double inv_s2, const double *p, double *t, double *out)
{
    or_spmv(nr, rp, ci, va, p, t);
    for (int64_t r = 0; r < nr; r++) t[r] *= lam[r];
    or_spmv(nc, trp, tci, tva, t, out);
    for (int64_t c = 0; c < nc; c++) out[c] += inv_s2 * p[c];
}

/*
 * Conjugate gradients (Hestenes & Stiefel, 1952) on the normal equations of
 * the proximal map for one frame, in FP64:
 *   H = A^T Lambda A + sigma^-2 I,   b = A^T Lambda y + sigma^-2 v.
 * Starts from x0 (x0 == NULL: from v).  Stops when ||b - H x|| <= tol ||b||
 * on the recursively updated residual, or after max_iter steps.
 * out_stats: [iterations, recursive rel. residual, true rel. residual, ||b||].
 */
int32_t or_prox_cg(int64_t nr, int64_t nc, const int64_t *rp, const int32_t *ci, const double *va,
                   const int64_t *trp, const int32_t *tci, const double *tva,
                   const double *lam, const double *y, const double *v, double sigma,
                   const double *x0, double tol, int32_t max_iter, double *x, double *out_stats)
{
    double inv_s2 = 1.0 / (sigma * sigma);
    double *t = (double *)malloc(sizeof(double) * (nr > 0 ? nr : 1));
    double *b = (double *)malloc(sizeof(double) * nc);
    double *r = (double *)malloc(sizeof(double) * nc);
    double *p = (double *)malloc(sizeof(double) * nc);
    double *q = (double *)malloc(sizeof(double) * nc);
    for (int64_t i = 0; i < nr; i++) t[i] = lam[i] * y[i];
    or_spmv(nc, trp, tci, tva, t, b);
    for (int64_t c = 0; c < nc; c++) b[c] += inv_s2 * v[c];
    double bnorm = sqrt(dot(nc, b, b));
    memcpy(x, x0 ? x0 : v, sizeof(double) * nc);
    apply_h(nr, nc, rp, ci, va, trp, tci, tva, lam, inv_s2, x, t, q);
    for (int64_t c = 0; c < nc; c++) r[c] = b[c] - q[c];
    memcpy(p, r, sizeof(double) * nc);
    double gamma = dot(nc, r, r);
    int it = 0;
    while (it < max_iter && sqrt(gamma) > tol * bnorm) {
        apply_h(nr, nc, rp, ci, va, trp, tci, tva, lam, inv_s2, p, t, q);
        double pq = dot(nc, p, q);
        if (!(pq > 0.0)) break;
        double alpha = gamma / pq;
        for (int64_t c = 0; c < nc; c++) {
            x[c] += alpha * p[c];
            r[c] -= alpha * q[c];
        }
        double gnew = dot(nc, r, r);
        double beta = gnew / gamma;
        gamma = gnew;
        for (int64_t c = 0; c < nc; c++) p[c] = r[c] + beta * p[c];
        it++;
    }
    /* true residual */
    apply_h(nr, nc, rp, ci, va, trp, tci, tva, lam, inv_s2, x, t, q);
    for (int64_t c = 0; c < nc; c++) q[c] = b[c] - q[c];
    double tr = sqrt(dot(nc, q, q));
    out_stats[0] = it;
    out_stats[1] = bnorm > 0 ? sqrt(gamma) / bnorm : sqrt(gamma);
    out_stats[2] = bnorm > 0 ? tr / bnorm : tr;
    out_stats[3] = bnorm;
    free(t); free(b); free(r); free(p); free(q);
    return it;
}

/* Backprojection of one frame's sinogram at selected voxels by the voxel's
 * own slab test against every ray of the frame: out[s] = sum_i a_{i,vox_s} y_i. */
void or_backproject_voxels(const or_geom *g, const double *angles, int32_t nviews, const double *y,
                           const int64_t *vox, int32_t nsel, double *out)
{
    int64_t per_view = (int64_t)g->nv * g->nu;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nsel; s++) {
        double acc = 0.0;
        for (int view = 0; view < nviews; view++)
            for (int iv = 0; iv < g->nv; iv++)
                for (int iu = 0; iu < g->nu; iu++) {
                    double S[3], D[3];
                    or_ray(g, angles[view], iu, iv, S, D);
                    double l = or_voxel_length(g, S, D, vox[s]);
                    if (l > 0.0) acc += l * y[view * per_view + (int64_t)iv * g->nu + iu];
                }
        out[s] = acc;
    }
}

/* Column vox of one frame's system matrix: every ray (view, iv, iu) that
 * meets the voxel, by the voxel's own slab test, with its length.  Writes at
 * most cap entries (ray index view*nv*nu + iv*nu + iu) and returns the count. */
int32_t or_voxel_column(const or_geom *g, const double *angles, int32_t nviews, int64_t vox, int64_t *ray,
                        double *len, int32_t cap)
{
    int32_t n = 0;
    for (int view = 0; view < nviews; view++)
        for (int iv = 0; iv < g->nv; iv++)
            for (int iu = 0; iu < g->nu; iu++) {
                double S[3], D[3];
                or_ray(g, angles[view], iu, iv, S, D);
                double l = or_voxel_length(g, S, D, vox);
                if (l > 0.0) {
                    if (n < cap) {
                        ray[n] = ((int64_t)view * g->nv + iv) * g->nu + iu;
                        len[n] = l;
                    }
                    n++;
                }
            }
    return n;
}

/* or_voxel_column for nsel voxels (in parallel): entries of voxel s at
 * ray[s*cap ..], len[s*cap ..], their count in count[s]. */
void or_voxel_columns(const or_geom *g, const double *angles, int32_t nviews, const int64_t *vox, int32_t nsel,
                      int32_t *count, int64_t *ray, double *len, int32_t cap)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nsel; s++)
        count[s] = or_voxel_column(g, angles, nviews, vox[s], ray + (int64_t)s * cap, len + (int64_t)s * cap, cap);
}

/* Projection of selected rays (view, iv, iu) of one frame by Siddon. */
void or_project_rays(const or_geom *g, const double *angles, const int32_t *view, const int32_t *iv,
                     const int32_t *iu, int32_t nsel, const double *x, double *out)
{
    int cap = g->nx + g->ny + g->nz + 4;
#pragma omp parallel
    {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < nsel; s++) {
            double S[3], D[3];
            or_ray(g, angles[view[s]], iu[s], iv[s], S, D);
            int n = or_siddon(g, S, D, idx, len, cap);
            double acc = 0.0;
            for (int e = 0; e < n; e++) acc += len[e] * x[idx[e]];
            out[s] = acc;
        }
        free(idx);
        free(len);
    }
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (timing of the oracle itself). */
void or_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
