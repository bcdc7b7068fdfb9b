/*
 * FP64 CPU oracle for the shaped-stencil leapfrog acoustic scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header or table with the HIP library.
 *
 * What it computes (Peixoto & Silva, Sec. 3):
 *   wave equation u_tt - c^2 lap(u) = f  (Sec. 3.1, eq. wave_eq), with an
 *   absorbing term eta(x) u_t in a band of nb cells (Sec. 3.1, damping layer);
 *   the Laplacian is the general symmetric stencil of Sec. 3.2,
 *   eq. spacexz_derivative2, written here as a plain list of points d with
 *   weights w_d:  h^2 lap(u)(x) ~ sum_d w_d u(x + d)  (u = 0 outside the grid);
 *   the time derivative is the centred second difference of Sec. 3.2,
 *   eq. time_derivative1, and u_t in the damping term the centred first
 *   difference.  With v = (c dt / h)^2 (the squared Courant number of
 *   Sec. 3.4, eq. courant), a = 1 - eta dt/2 and b = 1/(1 + eta dt/2):
 *
 *     u^{n+1} = b [ 2 u^n - a u^{n-1} + v (W u^n) + q^n delta_{x,xs} ],
 *
 *   q^n = dt^2 s(n dt) / h^d the source term at the source node (passed in
 *   already scaled), u^{-1} = u^0 = 0 (homogeneous initial data, Sec. 3.1),
 *   trace[n][r] = u^{n+1}(x_r) (seismic traces / receiver data, Sec. 5.2).
 *
 *   Sponge profile (the paper names the classic damping layer without a
 *   profile): depth into the band along each axis delta_i = max(nb - i,
 *   i - (n_i - 1 - nb), 0) and eta = eta_max * sum_i (delta_i / nb)^2.
 *
 * Adjoint (the paper notes the stencils carry over to adjoint and gradient
 * computations, Sec. 7): the exact discrete adjoint of the recursion above for
 * J = J(traces), rho^n_r = dJ/dtrace[n][r].  With psi^k = v b lambda^k
 * (lambda the Lagrange multiplier of step k-1 -> k):
 *
 *   psi^k = b [ 2 psi^{k+1} - a psi^{k+2} + v (W psi^{k+1}) + v rho^{k-1} @ x_r ],
 *   k = nt..1, psi^{nt+1} = psi^{nt+2} = 0, and
 *   dJ/dc(x) = sum_{k=1}^{nt} (2 / c(x)) psi^k(x) (W u^{k-1})(x).
 *
 * Grids are row-major with x fastest: 2D [nz][nx], 3D [nz][ny][nx]; offsets
 * and node coordinates are given as (x, z) in 2D and (x, y, z) in 3D.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

typedef struct {
    int ndim;
    i64 n[3];       /* extent along x, y, z (y = 1 in 2D) */
    i64 npoints;
} ora_grid;

static void grid_init(ora_grid *g, int ndim, const i64 *n) {
    g->ndim = ndim;
    g->n[0] = n[0];
    if (ndim == 2) { g->n[1] = 1; g->n[2] = n[1]; }
    else { g->n[1] = n[1]; g->n[2] = n[2]; }
    g->npoints = g->n[0] * g->n[1] * g->n[2];
}

/* offset list -> (dx, dy, dz) triples */
static void expand_offsets(int ndim, int npts, const int *offs, int *o3) {
    for (int p = 0; p < npts; ++p) {
        if (ndim == 2) { o3[3*p] = offs[2*p]; o3[3*p+1] = 0; o3[3*p+2] = offs[2*p+1]; }
        else { o3[3*p] = offs[3*p]; o3[3*p+1] = offs[3*p+1]; o3[3*p+2] = offs[3*p+2]; }
    }
}

static i64 node_index(const ora_grid *g, const i64 *c) {
    if (g->ndim == 2) return c[1] * g->n[0] + c[0];
    return (c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
}

static i64 wrap(i64 i, i64 n) { i %= n; return i < 0 ? i + n : i; }

/* out = W u : plain sum over every stencil point, zero outside the grid
 * (or periodic wrap when periodic != 0). */
static void apply_stencil(const ora_grid *g, int npts, const int *o3, const double *w,
                          const double *u, double *out, int periodic) {
    const i64 nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
    for (i64 z = 0; z < nz; ++z)
        for (i64 y = 0; y < ny; ++y)
            for (i64 x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int p = 0; p < npts; ++p) {
                    i64 xx = x + o3[3*p], yy = y + o3[3*p+1], zz = z + o3[3*p+2];
                    if (periodic) {
                        xx = wrap(xx, nx); yy = wrap(yy, ny); zz = wrap(zz, nz);
                    } else if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) {
                        continue;
                    }
                    s += w[p] * u[(zz * ny + yy) * nx + xx];
                }
                out[(z * ny + y) * nx + x] = s;
            }
}

/* damping factors a = 1 - eta dt/2, b = 1/(1 + eta dt/2) for every node.
 * The band depth is measured in the coordinates of an enclosing grid: node
 * (x, y, z) of this grid is node (x, y, z) + goff of a grid of extent gext
 * (goff = 0, gext = n when the grid is the whole domain). */
static void sponge(const ora_grid *g, int nb, double eta_max, double dt, const i64 *goff,
                   const i64 *gext, double *a, double *b) {
    const i64 nx = g->n[0], ny = g->n[1], nz = g->n[2];
    for (i64 z = 0; z < nz; ++z)
        for (i64 y = 0; y < ny; ++y)
            for (i64 x = 0; x < nx; ++x) {
                double eta = 0.0;
                if (nb > 0) {
                    i64 idx[3] = {x, y, z};
                    for (int ax = 0; ax < 3; ++ax) {
                        if (g->ndim == 2 && ax == 1) continue;
                        i64 i = idx[ax] + goff[ax], n = gext[ax];
                        i64 d = nb - i;
                        i64 d2 = i - (n - 1 - nb);
                        if (d2 > d) d = d2;
                        if (d < 0) d = 0;
                        double r = (double)d / (double)nb;
                        eta += r * r;
                    }
                    eta *= eta_max;
                }
                i64 k = (z * ny + y) * nx + x;
                a[k] = 1.0 - 0.5 * eta * dt;
                b[k] = 1.0 / (1.0 + 0.5 * eta * dt);
            }
}

/*
 * Forward run.  Returns 0 on success, -1 on allocation failure, -2 on bad input.
 *   n[ndim]           grid extent (x first)
 *   offs[npts*ndim]   stencil points (x first), w[npts] their weights
 *   v[npoints]        (c dt / h)^2 per node
 *   q[nt]             source term per step (already dt^2 s / h^d), src[ndim] node
 *   rec[nrec*ndim]    receiver nodes; traces[nt*nrec] output (may be NULL)
 *   init_prev/init_cur optional u^{-1}, u^0; final_prev/final_cur optional
 *   outputs u^{nt-1}, u^{nt}; store optional (nt+1)*npoints output holding
 *   u^0 .. u^nt.
 */
int ora_forward(int ndim, const i64 *n, int npts, const int *offs, const double *w,
                const double *v, double dt, int nt, int nb, double eta_max,
                const i64 *src, const double *q, int nrec, const i64 *rec, double *traces,
                const double *init_prev, const double *init_cur,
                double *final_prev, double *final_cur, double *store, int periodic,
                const i64 *goff_in, const i64 *gext_in) {
    if (ndim != 2 && ndim != 3) return -2;
    ora_grid g; grid_init(&g, ndim, n);
    i64 goff[3] = {0, 0, 0}, gext[3] = {g.n[0], g.n[1], g.n[2]};
    if (goff_in && gext_in) {   /* given x-first with ndim entries */
        goff[0] = goff_in[0]; gext[0] = gext_in[0];
        if (ndim == 3) { goff[1] = goff_in[1]; gext[1] = gext_in[1]; goff[2] = goff_in[2]; gext[2] = gext_in[2]; }
        else { goff[2] = goff_in[1]; gext[2] = gext_in[1]; }
    }
    const i64 N = g.npoints;
    int *o3 = (int *)malloc(sizeof(int) * 3 * (size_t)(npts > 0 ? npts : 1));
    double *um = (double *)calloc((size_t)N, sizeof(double));
    double *u0 = (double *)calloc((size_t)N, sizeof(double));
    double *lu = (double *)malloc(sizeof(double) * (size_t)N);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *b = (double *)malloc(sizeof(double) * (size_t)N);
    if (!o3 || !um || !u0 || !lu || !a || !b) {
        free(o3); free(um); free(u0); free(lu); free(a); free(b); return -1;
    }
    expand_offsets(ndim, npts, offs, o3);
    sponge(&g, nb, eta_max, dt, goff, gext, a, b);
    if (init_prev) memcpy(um, init_prev, sizeof(double) * (size_t)N);
    if (init_cur) memcpy(u0, init_cur, sizeof(double) * (size_t)N);
    i64 isrc = src ? node_index(&g, src) : -1;
    if (store) memcpy(store, u0, sizeof(double) * (size_t)N);

    for (int step = 0; step < nt; ++step) {
        apply_stencil(&g, npts, o3, w, u0, lu, periodic);
        /* um <- u^{n+1} (overwrites u^{n-1}) */
#pragma omp parallel for schedule(static)
        for (i64 k = 0; k < N; ++k) {
            double f = (k == isrc && q) ? q[step] : 0.0;
            um[k] = b[k] * (2.0 * u0[k] - a[k] * um[k] + v[k] * lu[k] + f);
        }
        double *t = um; um = u0; u0 = t;   /* u0 = u^{n+1}, um = u^n */
        if (traces)
            for (int r = 0; r < nrec; ++r)
                traces[(i64)step * nrec + r] = u0[node_index(&g, rec + (i64)r * ndim)];
        if (store) memcpy(store + (i64)(step + 1) * N, u0, sizeof(double) * (size_t)N);
    }
    if (final_prev) memcpy(final_prev, um, sizeof(double) * (size_t)N);
    if (final_cur) memcpy(final_cur, u0, sizeof(double) * (size_t)N);
    free(o3); free(um); free(u0); free(lu); free(a); free(b);
    return 0;
}

/*
 * Adjoint run and gradient dJ/dc, from full forward storage.
 *   c[npoints]          velocity (only its 2/c factor is used; v is passed as is)
 *   rho[nt*nrec]        dJ/dtrace
 *   grad[npoints]       output, overwritten with dJ/dc
 *   psi_out[npoints]    optional output psi^1
 * Other arguments as in ora_forward (same source, same initial state).
 */
int ora_adjoint_gradient(int ndim, const i64 *n, int npts, const int *offs, const double *w,
                         const double *v, const double *c, double dt, int nt, int nb,
                         double eta_max, const i64 *src, const double *q,
                         int nrec, const i64 *rec, const double *rho,
                         const double *init_prev, const double *init_cur,
                         double *grad, double *psi_out) {
    if (ndim != 2 && ndim != 3) return -2;
    ora_grid g; grid_init(&g, ndim, n);
    const i64 N = g.npoints;
    double *store = (double *)malloc(sizeof(double) * (size_t)N * (size_t)(nt + 1));
    int *o3 = (int *)malloc(sizeof(int) * 3 * (size_t)(npts > 0 ? npts : 1));
    double *p1 = (double *)calloc((size_t)N, sizeof(double));   /* psi^{k+1} */
    double *p2 = (double *)calloc((size_t)N, sizeof(double));   /* psi^{k+2} */
    double *lp = (double *)malloc(sizeof(double) * (size_t)N);
    double *lu = (double *)malloc(sizeof(double) * (size_t)N);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *b = (double *)malloc(sizeof(double) * (size_t)N);
    if (!store || !o3 || !p1 || !p2 || !lp || !lu || !a || !b) {
        free(store); free(o3); free(p1); free(p2); free(lp); free(lu); free(a); free(b);
        return -1;
    }
    int rc = ora_forward(ndim, n, npts, offs, w, v, dt, nt, nb, eta_max, src, q, 0, NULL, NULL,
                         init_prev, init_cur, NULL, NULL, store, 0, NULL, NULL);
    if (rc) {
        free(store); free(o3); free(p1); free(p2); free(lp); free(lu); free(a); free(b);
        return rc;
    }
    expand_offsets(ndim, npts, offs, o3);
    {
        i64 goff[3] = {0, 0, 0}, gext[3] = {g.n[0], g.n[1], g.n[2]};
        sponge(&g, nb, eta_max, dt, goff, gext, a, b);
    }
    for (i64 k = 0; k < N; ++k) grad[k] = 0.0;

    for (int k = nt; k >= 1; --k) {
        apply_stencil(&g, npts, o3, w, p1, lp, 0);
        /* p2 <- psi^k (overwrites psi^{k+2}) */
        for (i64 i = 0; i < N; ++i)
            p2[i] = b[i] * (2.0 * p1[i] - a[i] * p2[i] + v[i] * lp[i]);
        for (int r = 0; r < nrec; ++r) {
            i64 i = node_index(&g, rec + (i64)r * ndim);
            p2[i] += b[i] * v[i] * rho[(i64)(k - 1) * nrec + r];
        }
        double *t = p1; p1 = p2; p2 = t;   /* p1 = psi^k, p2 = psi^{k+1} */
        /* gradient term pairs psi^k with W u^{k-1} */
        apply_stencil(&g, npts, o3, w, store + (i64)(k - 1) * N, lu, 0);
        for (i64 i = 0; i < N; ++i) grad[i] += 2.0 / c[i] * p1[i] * lu[i];
    }
    if (psi_out) memcpy(psi_out, p1, sizeof(double) * (size_t)N);
    free(store); free(o3); free(p1); free(p2); free(lp); free(lu); free(a); free(b);
    return 0;
}

/* Discrete energy E^{n+1/2} = sum_x [ (u1 - u0)^2 / v - u1 (W u0) ] (no damping). */
double ora_energy(int ndim, const i64 *n, int npts, const int *offs, const double *w,
                  const double *v, const double *u0, const double *u1) {
    ora_grid g; grid_init(&g, ndim, n);
    const i64 N = g.npoints;
    int *o3 = (int *)malloc(sizeof(int) * 3 * (size_t)(npts > 0 ? npts : 1));
    double *lu = (double *)malloc(sizeof(double) * (size_t)N);
    if (!o3 || !lu) { free(o3); free(lu); return NAN; }
    expand_offsets(ndim, npts, offs, o3);
    apply_stencil(&g, npts, o3, w, u0, lu, 0);
    double e = 0.0;
    for (i64 k = 0; k < N; ++k) {
        double d = u1[k] - u0[k];
        e += d * d / v[k] - u1[k] * lu[k];
    }
    free(o3); free(lu);
    return e;
}

/* W u on its own (zero outside the grid, or periodic). */
int ora_apply_stencil(int ndim, const i64 *n, int npts, const int *offs, const double *w,
                      const double *u, double *out, int periodic) {
    ora_grid g; grid_init(&g, ndim, n);
    int *o3 = (int *)malloc(sizeof(int) * 3 * (size_t)(npts > 0 ? npts : 1));
    if (!o3) return -1;
    expand_offsets(ndim, npts, offs, o3);
    apply_stencil(&g, npts, o3, w, u, out, periodic);
    free(o3);
    return 0;
}
