/*
 * TEST INFRASTRUCTURE -- reference oracle, not part of the product.
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code with the HIP path.
 *
 * Plain FP64 implementation of the CT sensing matrix A of the linear model
 * A x + e = b (paper, Sec. 2.1, eq. "tomo") and of its literal transpose A^T,
 * which every Krylov step needs (Sec. 2.2.2: the solver only touches A and
 * A^T through products).  The paper does not fix the discretisation of A; the
 * reading used here is the exact ray-driven one: one ray per detector pixel,
 * from the source point to the pixel centre, and A[i][j] = length in mm of
 * ray i inside voxel j (Siddon, Med. Phys. 12(2), 1985, merge form).
 *
 * Geometry (circular cone-beam orbit, flat panel; the reading of the
 * unstated conventions):
 *   world frame in mm, origin at the isocentre, z = rotation axis;
 *   voxel (i,j,k) occupies [lo_a + i h_a, lo_a + (i+1) h_a] on each axis with
 *   lo_a = -n_a h_a / 2;
 *   view angle th: source S = (DSO cos th, DSO sin th, 0), detector centre
 *   C = ((DSO-DSD) cos th, (DSO-DSD) sin th, 0), e_u = (-sin th, cos th, 0),
 *   e_v = (0, 0, 1);
 *   pixel (iu, iv) centre = C + ((iu+1/2) du - nu du/2) e_u
 *                             + ((iv+1/2) dv - nv dv/2) e_v.
 * Layouts: volume x[k][j][i] (i fastest), projections y[view][iv][iu].
 *
 * Every routine here is written for obviousness, not speed: each ray's chord
 * list is built by collecting every plane crossing, sorting, and classifying
 * each sub-interval by its midpoint.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;      /* voxel size [mm] */
    int32_t nu, nv;
    double du, dv;          /* detector pitch [mm] */
    double dso, dsd;        /* source-isocentre, source-detector [mm] */
    int32_t n_views;
    const double *angles;   /* [n_views] radians */
} or_geom;

/* Source and pixel centre of ray (view, iu, iv). */
static void ray_endpoints(const or_geom *g, int view, int iu, int iv,
                          double S[3], double P[3])
{
    double th = g->angles[view];
    double c = cos(th), s = sin(th);
    double uc = (iu + 0.5) * g->du - g->nu * g->du / 2.0;
    double vc = (iv + 0.5) * g->dv - g->nv * g->dv / 2.0;
    S[0] = g->dso * c;
    S[1] = g->dso * s;
    S[2] = 0.0;
    P[0] = (g->dso - g->dsd) * c + uc * (-s);
    P[1] = (g->dso - g->dsd) * s + uc * c;
    P[2] = vc;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/*
 * Chords of the segment S->P through the voxel grid.  Writes at most `cap`
 * (voxel index, length) pairs, returns the number of non-empty chords (or -1
 * if cap was too small).  `work` must hold nx+ny+nz+5 doubles.
 */
static int trace(const or_geom *g, const double S[3], const double P[3],
                 int64_t *idx, double *len, int cap, double *work)
{
    const int n[3] = {g->nx, g->ny, g->nz};
    const double h[3] = {g->vx, g->vy, g->vz};
    double d[3], lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        d[a] = P[a] - S[a];
        lo[a] = -n[a] * h[a] / 2.0;
        hi[a] = n[a] * h[a] / 2.0;
    }
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);

    /* Parameter range [amin, amax] of the segment inside the volume box. */
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double a0 = (lo[a] - S[a]) / d[a];
            double a1 = (hi[a] - S[a]) / d[a];
            amin = fmax(amin, fmin(a0, a1));
            amax = fmin(amax, fmax(a0, a1));
        } else if (!(lo[a] < S[a] && S[a] < hi[a])) {
            return 0; /* parallel to this axis and outside the slab (or on a face) */
        }
    }
    if (!(amax > amin))
        return 0;

    /* All plane crossings strictly inside (amin, amax), plus both ends. */
    int m = 0;
    work[m++] = amin;
    work[m++] = amax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0)
            continue;
        for (int p = 0; p <= n[a]; ++p) {
            double al = (lo[a] + p * h[a] - S[a]) / d[a];
            if (al > amin && al < amax)
                work[m++] = al;
        }
    }
    qsort(work, (size_t)m, sizeof(double), cmp_double);

    int cnt = 0;
    for (int q = 0; q + 1 < m; ++q) {
        double dal = work[q + 1] - work[q];
        if (!(dal > 0.0))
            continue;
        double mid = 0.5 * (work[q] + work[q + 1]);
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            double f = floor((S[a] + mid * d[a] - lo[a]) / h[a]);
            int64_t ci = (int64_t)f;
            if (ci < 0) ci = 0;
            if (ci > n[a] - 1) ci = n[a] - 1;
            c[a] = ci;
        }
        if (cnt >= cap)
            return -1;
        idx[cnt] = (c[2] * g->ny + c[1]) * g->nx + c[0];
        len[cnt] = dal * L;
        ++cnt;
    }
    return cnt;
}

static int chord_cap(const or_geom *g) { return g->nx + g->ny + g->nz + 4; }

/* ---------------------------------------------------------------------- */
/* Public entry points (called through ctypes from oracle/oracle.py).       */

int or_ray_chords(const or_geom *g, int view, int iu, int iv,
                  int64_t *idx, double *len, int cap)
{
    double S[3], P[3];
    double *work = malloc(sizeof(double) * (size_t)(chord_cap(g) + 2));
    if (!work) return -2;
    ray_endpoints(g, view, iu, iv, S, P);
    int r = trace(g, S, P, idx, len, cap, work);
    free(work);
    return r;
}

/* Chords of an arbitrary segment S->P (used by the pins with hand-made rays). */
int or_segment_chords(const or_geom *g, const double *S, const double *P,
                      int64_t *idx, double *len, int cap)
{
    double *work = malloc(sizeof(double) * (size_t)(chord_cap(g) + 2));
    if (!work) return -2;
    int r = trace(g, S, P, idx, len, cap, work);
    free(work);
    return r;
}

/* y = A x over all rays. */
int or_forward(const or_geom *g, const double *x, double *y, int nthreads)
{
    const int64_t nray = (int64_t)g->n_views * g->nv * g->nu;
    const int cap = chord_cap(g);
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(| : err)
    {
        int64_t *idx = malloc(sizeof(int64_t) * (size_t)cap);
        double *len = malloc(sizeof(double) * (size_t)cap);
        double *work = malloc(sizeof(double) * (size_t)(cap + 2));
        if (!idx || !len || !work) err |= 1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nray; ++r) {
            if (err) continue;
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            int iv = rem / g->nu, iu = rem % g->nu;
            double S[3], P[3];
            ray_endpoints(g, view, iu, iv, S, P);
            int c = trace(g, S, P, idx, len, cap, work);
            if (c < 0) { err |= 2; continue; }
            double acc = 0.0;
            for (int q = 0; q < c; ++q)
                acc += len[q] * x[idx[q]];
            y[r] = acc;
        }
        free(idx); free(len); free(work);
    }
    return err ? -1 : 0;
}

/* x = A^T y: the same enumerator, scattering len * y_i into voxel j. */
int or_back(const or_geom *g, const double *y, double *x, int nthreads)
{
    const int64_t nray = (int64_t)g->n_views * g->nv * g->nu;
    const int64_t nvox = (int64_t)g->nx * g->ny * g->nz;
    const int cap = chord_cap(g);
    int err = 0;
    memset(x, 0, sizeof(double) * (size_t)nvox);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel reduction(| : err)
    {
        int64_t *idx = malloc(sizeof(int64_t) * (size_t)cap);
        double *len = malloc(sizeof(double) * (size_t)cap);
        double *work = malloc(sizeof(double) * (size_t)(cap + 2));
        if (!idx || !len || !work) err |= 1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nray; ++r) {
            if (err) continue;
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            int iv = rem / g->nu, iu = rem % g->nu;
            double S[3], P[3];
            ray_endpoints(g, view, iu, iv, S, P);
            int c = trace(g, S, P, idx, len, cap, work);
            if (c < 0) { err |= 2; continue; }
            double yr = y[r];
            if (yr == 0.0) continue;
            for (int q = 0; q < c; ++q) {
#pragma omp atomic
                x[idx[q]] += len[q] * yr;
            }
        }
        free(idx); free(len); free(work);
    }
    return err ? -1 : 0;
}

/* y_r = (A x)_r for a list of ray ids r = (view*nv + iv)*nu + iu. */
int or_forward_rays(const or_geom *g, const double *x, const int64_t *rays,
                    int64_t n, double *out)
{
    const int cap = chord_cap(g);
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        int64_t *idx = malloc(sizeof(int64_t) * (size_t)cap);
        double *len = malloc(sizeof(double) * (size_t)cap);
        double *work = malloc(sizeof(double) * (size_t)(cap + 2));
        if (!idx || !len || !work) err |= 1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < n; ++q) {
            if (err) continue;
            int64_t r = rays[q];
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            double S[3], P[3];
            ray_endpoints(g, view, rem % g->nu, rem / g->nu, S, P);
            int c = trace(g, S, P, idx, len, cap, work);
            if (c < 0) { err |= 2; continue; }
            double acc = 0.0;
            for (int t = 0; t < c; ++t)
                acc += len[t] * x[idx[t]];
            out[q] = acc;
        }
        free(idx); free(len); free(work);
    }
    return err ? -1 : 0;
}

/*
 * (A^T y)_j for a list of voxel ids j = (k*ny + jy)*nx + i.  For each view
 * only the pixels inside the bounding rectangle of the voxel's projected
 * corners (widened by one pixel) are traced: the voxel is convex and lies in
 * front of the source, so every ray that meets it ends inside that rectangle;
 * every other ray has a zero entry in column j.
 */
int or_back_voxels(const or_geom *g, const double *y, const int64_t *vox,
                   int64_t n, double *out)
{
    const int cap = chord_cap(g);
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        int64_t *idx = malloc(sizeof(int64_t) * (size_t)cap);
        double *len = malloc(sizeof(double) * (size_t)cap);
        double *work = malloc(sizeof(double) * (size_t)(cap + 2));
        if (!idx || !len || !work) err |= 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; ++q) {
            if (err) continue;
            int64_t j = vox[q];
            int i0 = (int)(j % g->nx);
            int j0 = (int)((j / g->nx) % g->ny);
            int k0 = (int)(j / ((int64_t)g->nx * g->ny));
            double acc = 0.0;
            for (int view = 0; view < g->n_views; ++view) {
                double th = g->angles[view];
                double c = cos(th), s = sin(th);
                double S[3] = {g->dso * c, g->dso * s, 0.0};
                double Cd[3] = {(g->dso - g->dsd) * c, (g->dso - g->dsd) * s, 0.0};
                double eu[3] = {-s, c, 0.0}, nrm[3] = {c, s, 0.0};
                double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
                for (int corner = 0; corner < 8; ++corner) {
                    double X[3] = {
                        -g->nx * g->vx / 2.0 + (i0 + (corner & 1)) * g->vx,
                        -g->ny * g->vy / 2.0 + (j0 + ((corner >> 1) & 1)) * g->vy,
                        -g->nz * g->vz / 2.0 + (k0 + ((corner >> 2) & 1)) * g->vz};
                    double dx[3] = {X[0] - S[0], X[1] - S[1], X[2] - S[2]};
                    double den = dx[0] * nrm[0] + dx[1] * nrm[1];
                    double t = -g->dsd / den;
                    double Pp[3] = {S[0] + t * dx[0] - Cd[0], S[1] + t * dx[1] - Cd[1],
                                    S[2] + t * dx[2] - Cd[2]};
                    double u = Pp[0] * eu[0] + Pp[1] * eu[1];
                    double v = Pp[2];
                    double fu = u / g->du + g->nu / 2.0 - 0.5;
                    double fv = v / g->dv + g->nv / 2.0 - 0.5;
                    umin = fmin(umin, fu); umax = fmax(umax, fu);
                    vmin = fmin(vmin, fv); vmax = fmax(vmax, fv);
                }
                int ua = (int)floor(umin) - 1, ub = (int)ceil(umax) + 1;
                int va = (int)floor(vmin) - 1, vb = (int)ceil(vmax) + 1;
                if (ua < 0) ua = 0;
                if (va < 0) va = 0;
                if (ub > g->nu - 1) ub = g->nu - 1;
                if (vb > g->nv - 1) vb = g->nv - 1;
                for (int iv = va; iv <= vb; ++iv)
                    for (int iu = ua; iu <= ub; ++iu) {
                        double Sr[3], Pr[3];
                        ray_endpoints(g, view, iu, iv, Sr, Pr);
                        int cc = trace(g, Sr, Pr, idx, len, cap, work);
                        if (cc < 0) { err |= 2; continue; }
                        for (int t = 0; t < cc; ++t)
                            if (idx[t] == j)
                                acc += len[t] *
                                       y[((int64_t)view * g->nv + iv) * g->nu + iu];
                    }
            }
            out[q] = acc;
        }
        free(idx); free(len); free(work);
    }
    return err ? -1 : 0;
}

/* Total number of non-empty chords (nnz of A). */
int64_t or_count_nnz(const or_geom *g)
{
    const int64_t nray = (int64_t)g->n_views * g->nv * g->nu;
    const int cap = chord_cap(g);
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int64_t *idx = malloc(sizeof(int64_t) * (size_t)cap);
        double *len = malloc(sizeof(double) * (size_t)cap);
        double *work = malloc(sizeof(double) * (size_t)(cap + 2));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nray; ++r) {
            int view = (int)(r / ((int64_t)g->nv * g->nu));
            int rem = (int)(r % ((int64_t)g->nv * g->nu));
            double S[3], P[3];
            ray_endpoints(g, view, rem % g->nu, rem / g->nu, S, P);
            int c = trace(g, S, P, idx, len, cap, work);
            if (c > 0) total += c;
        }
        free(idx); free(len); free(work);
    }
    return total;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
