/*
 * FP64 CPU oracle for the finite-difference acoustic propagation path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do. It shares no code with the HIP library.
 *
 * What it computes (paper: section 2.1 eq. 1-2, section 2.2 eq. 5-12b,
 * section 2.3 eq. 13-15). The paper states the continuous equations only;
 * the discrete scheme written out here is this project's reading of them:
 *
 *   padded grid   NZ = nz + 2 nb, NX = wnx + 2 nb per shot window, zero
 *                 values outside the padded box (Dirichlet halo);
 *   free surface  (optional) the top of the model is a pressure-free
 *                 surface instead of a sponge: no sponge rows above row 0
 *                 (NZ = nz + nb), u = 0 on row 0 after every step, and the
 *                 rows above it are the odd mirror u[-m] = -u[m] (image
 *                 method);
 *   model         V = Pad(v): edge replication of the shot's window;
 *   Laplacian     L8 u = h^-2 (2 c0 u + sum_k c_k (u[i+-k][j] + u[i][j+-k])),
 *                 c = (-205/72, 8/5, -1/5, 8/315, -1/560);
 *   sponge        sigma = smax (dz^2 + dx^2), dz = distance into the sponge
 *                 / nb, smax = 3 v_ref ln(1/R) / (2 nb h);
 *                 a = 1/(1 + sigma dt/2), b = (1 - sigma dt/2) a;
 *   source        s^n = w[n] / h^2 at the source cell; a source off the grid
 *                 (fractional offsets fz, fx in [0, 1) toward +z, +x) is
 *                 spread over the four surrounding cells with bilinear
 *                 weights (1-fz)(1-fx), (1-fz) fx, fz (1-fx), fz fx;
 *   time step     u^{n+1} = a (2 u^n + V^2 dt^2 (L8 u^n + s^n)) - b u^{n-1},
 *                 u^{-1} = u^0 = 0  (eq. 1, leapfrog, damped in the sponge);
 *   receivers     d[r][n] = u^{n+1}[rz][rx]; off the grid, the bilinear
 *                 combination of the four surrounding cells (same weights);
 *   misfit        phi = 1/2 sum (d - d_obs)^2   (eq. 2).
 *
 *   Born (eq. 9-11, solved jointly as the paper notes; velocity
 *   parametrisation, exact derivative of the discrete forward map):
 *                 rho = 2 Pad(dv) / V,
 *                 du^{n+1} = a (2 du^n + V^2 dt^2 (L8 du^n + rho (L8 u^n + s^n)))
 *                            - b du^{n-1},  dd[r][n] = du^{n+1}[rz][rx].
 *
 *   Relative perturbation (eq. 12 writes the Born operator on dm / m_o):
 *                 with the grid's `relative` flag set, the operator is
 *                 J_rel = J diag(v): born_demig takes dm = dv / v and runs
 *                 the above on dv = v dm; born_mig (and so the gradient)
 *                 returns diag(v) J^T r, its exact transpose.
 *
 *   PML (optional, the grid's `pml` flag; the paper names no boundary): a
 *   perfectly matched layer in the nb padded cells instead of the sponge.
 *   Stretching each axis by s_x = 1 + d_x / s (s the Laplace variable,
 *   d_x = smax dx^2 the sponge's profile) and multiplying the stretched
 *   equation by s_x s_z gives a symmetric operator,
 *     (1/V^2)(u_tt + (d_x + d_z) u_t + d_x d_z u)
 *       - d/dx(du/dx + psi_x) - d/dz(du/dz + psi_z) = f,
 *     psi_x = (s_z / s_x - 1) du/dx:  psi_x,t + d_x psi_x = (d_z - d_x) du/dx,
 *   (psi_z alike with x and z exchanged), with f in the physical cells
 *   where d_x = d_z = 0. Discretised as the sponge scheme plus
 *     psi_x lives on the x edges (i, j+1/2), j = 0 .. NX-2, with d_x taken at
 *     the edge and d_z at row i; Dx u = (u[i][j+1] - u[i][j]) / h;
 *     psi_x^n = b_x psi_x^{n-1} + a_x Dx u^n, b_x = exp(-d_x dt),
 *     a_x = (d_z - d_x)(1 - b_x) / d_x (= d_z dt where d_x = 0), a
 *     recursive convolution; psi_z on the z edges (i+1/2, j) alike;
 *     u^{n+1} = a ((2 - d_x d_z dt^2) u^n
 *               + V^2 dt^2 (L8 u^n + s^n - Dx^T psi_x^n - Dz^T psi_z^n))
 *               - b u^{n-1},  (a, b the sponge's coefficients),
 *   where -Dx^T psi = (psi[j+1/2] - psi[j-1/2]) / h. For every time shift the
 *   operator is diag(mass) - L8 + Dx^T diag(m_x) Dx + Dz^T diag(m_z) Dz with
 *   diagonal m_x, m_z, hence symmetric: reciprocity holds exactly, and the
 *   adjoint is the same recursion (psi included) run backward in time. The
 *   imaging history becomes V^2 dt^2 (L8 u^n + s^n - D^T psi^n), and the
 *   Born source uses the same term.
 *
 *   Adjoint (eq. 13; exact transpose of the Born map):
 *                 lam^n = a (2 lam^{n+1} + V^2 dt^2 (L8 lam^{n+1} + R^T r^n))
 *                         - b lam^{n+2},  n = nt-1 .. 0, lam^{nt} = lam^{nt+1} = 0,
 *                 img = sum_shots Pad^T( (2/V) sum_n lam^n (L8 u^n + s^n) ),
 *                 where R^T adds r[r][n] at receiver cells (times the bilinear
 *                 weights off the grid) and Pad^T sums
 *                 every sponge cell onto the edge cell it replicates.
 *
 * Every function below works on one shot at a time; shots are independent
 * and run in an OpenMP loop, and per-shot images are summed in shot order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nz, nx, nb;
    double h, dt, v_ref, R;
    int free_surface;   /* 1: pressure-free top surface on physical row 0 */
    int relative;       /* 1: Born operator on dv / v (J diag(v)) */
    int pml;            /* 1: perfectly matched layer instead of the sponge */
} og_grid;

typedef struct {
    int nshots;
    const int *src_z, *src_x;
    const int *win_x0, *win_nx; /* NULL: full width */
    const int *nt;              /* NULL: nt_max for every shot */
    int nt_max;
    const int64_t *rec_ptr;
    const int *rec_z, *rec_x;
    const double *wavelet;      /* [nt_max] shared, or [nshots][nt_max] */
    int wavelet_shared;
    const double *src_fz, *src_fx; /* NULL: sources on the grid */
    const double *rec_fz, *rec_fx; /* NULL: receivers on the grid */
} og_geom;

/* 8th-order central second-derivative weights (Fornberg 1988). */
static const double C8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                             8.0 / 315.0, -1.0 / 560.0};

/* ------------------------------------------------------------------ */
/* per-shot padded domain                                              */

typedef struct {
    int NZ, NX, x0, wnx;
    int top;     /* padded rows above physical row 0 (0 with a free surface) */
    double *V;   /* padded velocity */
    double *c;   /* V^2 dt^2 */
    double *a, *b;
    /* PML only (NULL otherwise): d_x d_z dt^2 per cell; recursion
     * coefficients of the x edges (index j: edge j+1/2) and z edges (index
     * i: edge i+1/2) */
    double *fdt2, *bx, *ax, *bz, *az;
} shot_dom;

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void shot_window(const og_grid *g, const og_geom *geo, int s, int *x0, int *wnx)
{
    if (geo->win_x0) { *x0 = geo->win_x0[s]; *wnx = geo->win_nx[s]; }
    else { *x0 = 0; *wnx = g->nx; }
}

static int shot_nt(const og_geom *geo, int s) { return geo->nt ? geo->nt[s] : geo->nt_max; }

static const double *shot_wavelet(const og_geom *geo, int s)
{
    return geo->wavelet_shared ? geo->wavelet : geo->wavelet + (int64_t)s * geo->nt_max;
}

static int top_rows(const og_grid *g) { return g->free_surface ? 0 : g->nb; }

/* Pad: edge replication of the window [x0, x0+wnx) of the nz x nx model. */
static void pad_model(const og_grid *g, int x0, int wnx, const double *v, double *V)
{
    int NZ = g->nz + g->nb + top_rows(g), NX = wnx + 2 * g->nb;
    for (int i = 0; i < NZ; i++)
        for (int j = 0; j < NX; j++) {
            int pi = clampi(i - top_rows(g), 0, g->nz - 1);
            int pj = x0 + clampi(j - g->nb, 0, wnx - 1);
            V[(int64_t)i * NX + j] = v[(int64_t)pi * g->nx + pj];
        }
}

/* Pad^T: every padded cell adds onto the physical cell it was copied from. */
static void pad_adjoint_add(const og_grid *g, int x0, int wnx, const double *P, double *img)
{
    int NZ = g->nz + g->nb + top_rows(g), NX = wnx + 2 * g->nb;
    for (int i = 0; i < NZ; i++)
        for (int j = 0; j < NX; j++) {
            int pi = clampi(i - top_rows(g), 0, g->nz - 1);
            int pj = x0 + clampi(j - g->nb, 0, wnx - 1);
            img[(int64_t)pi * g->nx + pj] += P[(int64_t)i * NX + j];
        }
}

static double sponge_depth(int i, int n, int nb, int lo)
{
    /* distance (in cells, / nb) into the sponge along one axis; lo = width
     * of the sponge at the low end (nb, or 0 under a free surface) */
    int d = 0;
    if (i < lo) d = lo - i;
    if (i > n - 1 - nb) d = i - (n - 1 - nb);
    return nb > 0 ? (double)d / (double)nb : 0.0;
}

/* the same depth at a half-integer position x (an edge between cells) */
static double layer_depth(double x, int n, int nb, int lo)
{
    double d = 0.0;
    if (x < lo) d = lo - x;
    if (x > n - 1 - nb) d = x - (n - 1 - nb);
    return nb > 0 ? d / (double)nb : 0.0;
}

/* recursion coefficients of an edge: damping d along the edge's own axis,
 * e along the other; psi^n = b psi^{n-1} + a D u^n */
static void edge_coef(double d, double e, double dt, double *b, double *a)
{
    *b = exp(-d * dt);
    *a = (e - d) * (d > 0.0 ? (1.0 - *b) / d : dt);
}

static int dom_init(shot_dom *D, const og_grid *g, const og_geom *geo, int s, const double *v)
{
    shot_window(g, geo, s, &D->x0, &D->wnx);
    D->top = top_rows(g);
    D->NZ = g->nz + g->nb + D->top;
    D->NX = D->wnx + 2 * g->nb;
    int64_t n = (int64_t)D->NZ * D->NX;
    D->V = malloc(n * sizeof(double));
    D->c = malloc(n * sizeof(double));
    D->a = malloc(n * sizeof(double));
    D->b = malloc(n * sizeof(double));
    D->fdt2 = D->bx = D->ax = D->bz = D->az = NULL;
    if (!D->V || !D->c || !D->a || !D->b) return -1;
    pad_model(g, D->x0, D->wnx, v, D->V);
    double smax = g->nb > 0 ? 3.0 * g->v_ref * log(1.0 / g->R) / (2.0 * g->nb * g->h) : 0.0;
    for (int i = 0; i < D->NZ; i++)
        for (int j = 0; j < D->NX; j++) {
            int64_t k = (int64_t)i * D->NX + j;
            double dz = sponge_depth(i, D->NZ, g->nb, D->top), dx = sponge_depth(j, D->NX, g->nb, g->nb);
            double sig = smax * (dz * dz + dx * dx);
            D->a[k] = 1.0 / (1.0 + 0.5 * sig * g->dt);
            D->b[k] = (1.0 - 0.5 * sig * g->dt) / (1.0 + 0.5 * sig * g->dt);
            D->c[k] = D->V[k] * D->V[k] * g->dt * g->dt;
        }
    if (g->pml && g->nb > 0) {
        D->fdt2 = malloc(n * sizeof(double));
        D->bx = malloc(n * sizeof(double));
        D->ax = malloc(n * sizeof(double));
        D->bz = malloc(n * sizeof(double));
        D->az = malloc(n * sizeof(double));
        if (!D->fdt2 || !D->bx || !D->ax || !D->bz || !D->az) return -1;
        for (int i = 0; i < D->NZ; i++)
            for (int j = 0; j < D->NX; j++) {
                int64_t k = (int64_t)i * D->NX + j;
                double dz = smax * pow(sponge_depth(i, D->NZ, g->nb, D->top), 2);
                double dx = smax * pow(sponge_depth(j, D->NX, g->nb, g->nb), 2);
                D->fdt2[k] = dx * dz * g->dt * g->dt;
                /* x edge (i, j+1/2): d_x at the edge, d_z of row i */
                double dxe = smax * pow(layer_depth(j + 0.5, D->NX, g->nb, g->nb), 2);
                edge_coef(dxe, dz, g->dt, &D->bx[k], &D->ax[k]);
                if (j == D->NX - 1) D->ax[k] = 0.0;     /* no edge right of the box */
                /* z edge (i+1/2, j): d_z at the edge, d_x of column j */
                double dze = smax * pow(layer_depth(i + 0.5, D->NZ, g->nb, D->top), 2);
                edge_coef(dze, dx, g->dt, &D->bz[k], &D->az[k]);
                if (i == D->NZ - 1) D->az[k] = 0.0;     /* no edge below the box */
            }
    }
    return 0;
}

static void dom_free(shot_dom *D)
{
    free(D->V); free(D->c); free(D->a); free(D->b);
    free(D->fdt2); free(D->bx); free(D->ax); free(D->bz); free(D->az);
}

/* PML: advance the edge fields psi_x, psi_z of a wavefield from u (level n)
 * and add -Dx^T psi_x - Dz^T psi_z to lap. No-op without a PML. */
static void pml_terms(const shot_dom *D, double h, const double *u, double *psx, double *psz, double *lap)
{
    if (!D->fdt2) return;
    int NZ = D->NZ, NX = D->NX;
    for (int i = 0; i < NZ; i++)
        for (int j = 0; j < NX; j++) {
            int64_t k = (int64_t)i * NX + j;
            double dux = j + 1 < NX ? (u[k + 1] - u[k]) / h : 0.0;
            double duz = i + 1 < NZ ? (u[k + NX] - u[k]) / h : 0.0;
            psx[k] = D->bx[k] * psx[k] + D->ax[k] * dux;
            psz[k] = D->bz[k] * psz[k] + D->az[k] * duz;
        }
    for (int i = 0; i < NZ; i++)
        for (int j = 0; j < NX; j++) {
            int64_t k = (int64_t)i * NX + j;
            double div = psx[k] + psz[k];
            if (j > 0) div -= psx[k - 1];
            if (i > 0) div -= psz[k - NX];
            lap[k] += div / h;
        }
}

/* the leapfrog update of one cell: a ((2 - d_x d_z dt^2) u + c lap) - b u_prev */
static double leap(const shot_dom *D, int64_t k, double u, double lap, double um)
{
    double two = D->fdt2 ? 2.0 - D->fdt2[k] : 2.0;
    return D->a[k] * (two * u + D->c[k] * lap) - D->b[k] * um;
}

/* L8 u with zero values outside the NZ x NX box; with mirror != 0 the rows
 * above row 0 are the odd mirror u[-m] = -u[m] (free surface). */
static void laplacian8(const double *u, int NZ, int NX, double h, double *out, int mirror)
{
    double ih2 = 1.0 / (h * h);
    for (int i = 0; i < NZ; i++)
        for (int j = 0; j < NX; j++) {
            double acc = 2.0 * C8[0] * u[(int64_t)i * NX + j];
            for (int k = 1; k <= 4; k++) {
                if (i - k >= 0) acc += C8[k] * u[(int64_t)(i - k) * NX + j];
                else if (mirror && k - i < NZ) acc -= C8[k] * u[(int64_t)(k - i) * NX + j];
                if (i + k < NZ) acc += C8[k] * u[(int64_t)(i + k) * NX + j];
                if (j - k >= 0) acc += C8[k] * u[(int64_t)i * NX + j - k];
                if (j + k < NX) acc += C8[k] * u[(int64_t)i * NX + j + k];
            }
            out[(int64_t)i * NX + j] = acc * ih2;
        }
}

/* padded index of a physical cell (z, x) of shot s */
static int64_t cell_index(const og_grid *g, const shot_dom *D, int z, int x)
{
    return (int64_t)(z + D->top) * D->NX + (x - D->x0 + g->nb);
}

/* the pressure-free surface: row 0 held at zero */
static void pin_surface(const og_grid *g, const shot_dom *D, double *u)
{
    if (g->free_surface) memset(u, 0, (size_t)D->NX * sizeof(double));
}

/* A point (z + fz, x + fx) of shot s's physical grid: the cells it touches
 * and their bilinear weights; cells whose weight is exactly zero are left
 * out, so a point on the grid is its own cell with weight 1. */
typedef struct {
    int n;
    int64_t cell[4];
    double w[4];
} point_w;

static point_w point_weights(const og_grid *g, const shot_dom *D, int z, int x, double fz, double fx)
{
    point_w p;
    p.n = 0;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            double w = (a ? fz : 1.0 - fz) * (b ? fx : 1.0 - fx);
            if (w == 0.0) continue;
            p.cell[p.n] = cell_index(g, D, z + a, x + b);
            p.w[p.n] = w;
            p.n++;
        }
    return p;
}

static point_w src_point(const og_grid *g, const og_geom *geo, const shot_dom *D, int s)
{
    return point_weights(g, D, geo->src_z[s], geo->src_x[s], geo->src_fz ? geo->src_fz[s] : 0.0,
                         geo->src_fx ? geo->src_fx[s] : 0.0);
}

static point_w rec_point(const og_grid *g, const og_geom *geo, const shot_dom *D, int64_t r)
{
    return point_weights(g, D, geo->rec_z[r], geo->rec_x[r], geo->rec_fz ? geo->rec_fz[r] : 0.0,
                         geo->rec_fx ? geo->rec_fx[r] : 0.0);
}

/* field[cells] += w * val */
static void point_add(const point_w *p, double val, double *field)
{
    for (int k = 0; k < p->n; k++) field[p->cell[k]] += p->w[k] * val;
}

/* sum of w * field[cells] */
static double point_sample(const point_w *p, const double *field)
{
    double acc = 0.0;
    for (int k = 0; k < p->n; k++) acc += p->w[k] * field[p->cell[k]];
    return acc;
}

/* ------------------------------------------------------------------ */
/* one shot                                                            */

/* Forward modelling of shot s. d_shot is [nrec][nt]. If hist != NULL it
 * receives u^n for n = 0 .. nt ([nt+1][NZ][NX]); if lap_hist != NULL it
 * receives L8 u^n + s^n (- D^T psi^n with a PML) for n = 0 .. nt-1
 * ([nt][NZ][NX]), the term the imaging condition multiplies. */
static int forward_shot(const og_grid *g, const og_geom *geo, int s, const shot_dom *D,
                        double *d_shot, double *hist, double *lap_hist)
{
    int nt = shot_nt(geo, s);
    int64_t n = (int64_t)D->NZ * D->NX;
    double *um = calloc(n, sizeof(double)), *u0 = calloc(n, sizeof(double));
    double *up = calloc(n, sizeof(double)), *lap = malloc(n * sizeof(double));
    double *psx = calloc(n, sizeof(double)), *psz = calloc(n, sizeof(double));
    if (!um || !u0 || !up || !lap || !psx || !psz) {
        free(um); free(u0); free(up); free(lap); free(psx); free(psz);
        return -1;
    }
    const double *w = shot_wavelet(geo, s);
    point_w src = src_point(g, geo, D, s);
    int64_t r0 = geo->rec_ptr[s], nrec = geo->rec_ptr[s + 1] - r0;
    double ih2 = 1.0 / (g->h * g->h);
    for (int t = 0; t < nt; t++) {
        if (hist) memcpy(hist + (int64_t)t * n, u0, n * sizeof(double));
        laplacian8(u0, D->NZ, D->NX, g->h, lap, g->free_surface);
        point_add(&src, w[t] * ih2, lap);
        pml_terms(D, g->h, u0, psx, psz, lap);
        if (lap_hist) memcpy(lap_hist + (int64_t)t * n, lap, n * sizeof(double));
        for (int64_t k = 0; k < n; k++) up[k] = leap(D, k, u0[k], lap[k], um[k]);
        pin_surface(g, D, up);
        for (int64_t r = 0; r < nrec; r++) {
            point_w rp = rec_point(g, geo, D, r0 + r);
            d_shot[r * nt + t] = point_sample(&rp, up);
        }
        double *tmp = um; um = u0; u0 = up; up = tmp;
    }
    if (hist) memcpy(hist + (int64_t)nt * n, u0, n * sizeof(double));
    free(um); free(u0); free(up); free(lap); free(psx); free(psz);
    return 0;
}

/* Born modelling of shot s: dd_shot = J_s dv, [nrec][nt]. */
static int born_shot(const og_grid *g, const og_geom *geo, int s, const shot_dom *D,
                     const double *dv, double *dd_shot)
{
    int nt = shot_nt(geo, s);
    int64_t n = (int64_t)D->NZ * D->NX;
    double *um = calloc(n, sizeof(double)), *u0 = calloc(n, sizeof(double));
    double *up = calloc(n, sizeof(double)), *lap = malloc(n * sizeof(double));
    double *dm = calloc(n, sizeof(double)), *d0 = calloc(n, sizeof(double));
    double *dp = calloc(n, sizeof(double)), *dlap = malloc(n * sizeof(double));
    double *rho = malloc(n * sizeof(double));
    double *psx = calloc(n, sizeof(double)), *psz = calloc(n, sizeof(double));
    double *qsx = calloc(n, sizeof(double)), *qsz = calloc(n, sizeof(double));
    int ok = um && u0 && up && lap && dm && d0 && dp && dlap && rho && psx && psz && qsx && qsz;
    if (ok) {
        pad_model(g, D->x0, D->wnx, dv, rho);            /* Pad(dv) */
        for (int64_t k = 0; k < n; k++) rho[k] = 2.0 * rho[k] / D->V[k];
        const double *w = shot_wavelet(geo, s);
        point_w src = src_point(g, geo, D, s);
        int64_t r0 = geo->rec_ptr[s], nrec = geo->rec_ptr[s + 1] - r0;
        double ih2 = 1.0 / (g->h * g->h);
        for (int t = 0; t < nt; t++) {
            laplacian8(u0, D->NZ, D->NX, g->h, lap, g->free_surface);
            point_add(&src, w[t] * ih2, lap);             /* L8 u^n + s^n */
            pml_terms(D, g->h, u0, psx, psz, lap);        /* - D^T psi^n */
            laplacian8(d0, D->NZ, D->NX, g->h, dlap, g->free_surface);
            pml_terms(D, g->h, d0, qsx, qsz, dlap);
            for (int64_t k = 0; k < n; k++) {
                dp[k] = leap(D, k, d0[k], dlap[k] + rho[k] * lap[k], dm[k]);
                up[k] = leap(D, k, u0[k], lap[k], um[k]);
            }
            pin_surface(g, D, up);
            pin_surface(g, D, dp);
            for (int64_t r = 0; r < nrec; r++) {
                point_w rp = rec_point(g, geo, D, r0 + r);
                dd_shot[r * nt + t] = point_sample(&rp, dp);
            }
            double *tmp = um; um = u0; u0 = up; up = tmp;
            tmp = dm; dm = d0; d0 = dp; dp = tmp;
        }
    }
    free(um); free(u0); free(up); free(lap); free(dm); free(d0); free(dp); free(dlap); free(rho);
    free(psx); free(psz); free(qsx); free(qsz);
    return ok ? 0 : -1;
}

/* Adjoint of shot s: adds Pad^T((2/V) sum_n lam^n (L8 u^n + s^n)) to img
 * (with a PML, L8 u^n + s^n - D^T psi^n). res_shot is [nrec][nt]. If
 * lam_hist != NULL it receives lam^n for n = 0..nt-1 ([nt][NZ][NX]). */
static int adjoint_shot(const og_grid *g, const og_geom *geo, int s, const shot_dom *D,
                        const double *res_shot, double *img, double *lam_hist)
{
    int nt = shot_nt(geo, s);
    int64_t n = (int64_t)D->NZ * D->NX;
    double *lhist = malloc((size_t)(nt + 1) * n * sizeof(double));
    double *dummy = malloc(((geo->rec_ptr[s + 1] - geo->rec_ptr[s]) * (int64_t)nt + 1) * sizeof(double));
    double *l1 = calloc(n, sizeof(double)), *l2 = calloc(n, sizeof(double));
    double *l0 = calloc(n, sizeof(double)), *lap = malloc(n * sizeof(double));
    double *G = calloc(n, sizeof(double));
    double *psx = calloc(n, sizeof(double)), *psz = calloc(n, sizeof(double));
    int ok = lhist && dummy && l1 && l2 && l0 && lap && G && psx && psz;
    if (ok) ok = forward_shot(g, geo, s, D, dummy, NULL, lhist) == 0;
    if (ok) {
        int64_t r0 = geo->rec_ptr[s], nrec = geo->rec_ptr[s + 1] - r0;
        for (int t = nt - 1; t >= 0; t--) {
            laplacian8(l1, D->NZ, D->NX, g->h, lap, g->free_surface);    /* L8 lam^{n+1} */
            pml_terms(D, g->h, l1, psx, psz, lap);        /* - D^T psi~^{n+1} */
            for (int64_t r = 0; r < nrec; r++) {          /* + R^T r^n */
                point_w rp = rec_point(g, geo, D, r0 + r);
                point_add(&rp, res_shot[r * nt + t], lap);
            }
            for (int64_t k = 0; k < n; k++) l0[k] = leap(D, k, l1[k], lap[k], l2[k]);
            pin_surface(g, D, l0);
            if (lam_hist) memcpy(lam_hist + (int64_t)t * n, l0, n * sizeof(double));
            const double *lu = lhist + (int64_t)t * n;     /* L8 u^n + s^n (- D^T psi^n) */
            for (int64_t k = 0; k < n; k++) G[k] += l0[k] * lu[k];
            double *tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
        }
        for (int64_t k = 0; k < n; k++) G[k] *= 2.0 / D->V[k];
        pad_adjoint_add(g, D->x0, D->wnx, G, img);
    }
    free(lhist); free(dummy); free(l1); free(l2); free(l0); free(lap); free(G); free(psx); free(psz);
    return ok ? 0 : -1;
}

/* ------------------------------------------------------------------ */
/* public entry points (ctypes)                                        */

static int64_t shot_data_offset(const og_geom *geo, int s)
{
    int64_t off = 0;
    for (int q = 0; q < s; q++) off += (geo->rec_ptr[q + 1] - geo->rec_ptr[q]) * (int64_t)shot_nt(geo, q);
    return off;
}

int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* d = F(v), packed traces. */
int oracle_forward(const og_grid *g, const og_geom *geo, const double *v, double *d)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int s = 0; s < geo->nshots; s++) {
        shot_dom D;
        if (dom_init(&D, g, geo, s, v)) { err |= 1; dom_free(&D); continue; }
        err |= forward_shot(g, geo, s, &D, d + shot_data_offset(geo, s), NULL, NULL) ? 1 : 0;
        dom_free(&D);
    }
    return err ? -1 : 0;
}

/* dd = J dv (relative: dd = J diag(v) dm, the perturbation given as dm = dv / v). */
int oracle_born_demig(const og_grid *g, const og_geom *geo, const double *v, const double *dv, double *dd)
{
    double *abs_dv = NULL;
    if (g->relative) {
        int64_t npix = (int64_t)g->nz * g->nx;
        abs_dv = malloc((size_t)npix * sizeof(double) + 1);
        if (!abs_dv) return -1;
        for (int64_t k = 0; k < npix; k++) abs_dv[k] = v[k] * dv[k];
        dv = abs_dv;
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int s = 0; s < geo->nshots; s++) {
        shot_dom D;
        if (dom_init(&D, g, geo, s, v)) { err |= 1; dom_free(&D); continue; }
        err |= born_shot(g, geo, s, &D, dv, dd + shot_data_offset(geo, s)) ? 1 : 0;
        dom_free(&D);
    }
    free(abs_dv);
    return err ? -1 : 0;
}

/* img = J^T r (shot images summed in shot order); relative: diag(v) J^T r. */
int oracle_born_mig(const og_grid *g, const og_geom *geo, const double *v, const double *r, double *img)
{
    int64_t npix = (int64_t)g->nz * g->nx;
    double *per = calloc((size_t)geo->nshots * npix + 1, sizeof(double));
    if (!per) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int s = 0; s < geo->nshots; s++) {
        shot_dom D;
        if (dom_init(&D, g, geo, s, v)) { err |= 1; dom_free(&D); continue; }
        err |= adjoint_shot(g, geo, s, &D, r + shot_data_offset(geo, s), per + s * npix, NULL) ? 1 : 0;
        dom_free(&D);
    }
    memset(img, 0, npix * sizeof(double));
    for (int s = 0; s < geo->nshots; s++)
        for (int64_t k = 0; k < npix; k++) img[k] += per[s * npix + k];
    if (g->relative)
        for (int64_t k = 0; k < npix; k++) img[k] *= v[k];
    free(per);
    return err ? -1 : 0;
}

/* g = J^T (F(v) - d_obs), misfit = 1/2 ||F(v) - d_obs||^2; d_syn optional. */
int oracle_gradient(const og_grid *g, const og_geom *geo, const double *v, const double *d_obs,
                    double *grad, double *misfit, double *d_syn)
{
    int64_t nd = shot_data_offset(geo, geo->nshots);
    double *d = malloc((nd + 1) * sizeof(double));
    if (!d) return -1;
    int err = oracle_forward(g, geo, v, d);
    double phi = 0.0;
    for (int64_t k = 0; k < nd; k++) {
        d[k] -= d_obs[k];
        phi += 0.5 * d[k] * d[k];
    }
    if (misfit) *misfit = phi;
    if (d_syn)
        for (int64_t k = 0; k < nd; k++) d_syn[k] = d[k] + d_obs[k];
    if (!err) err = oracle_born_mig(g, geo, v, d, grad);
    free(d);
    return err;
}

/* Wavefield histories of one shot, for identity tests:
 * u_hist [nt+1][NZ][NX] receives u^0 .. u^nt; lam_hist (nullable)
 * [nt][NZ][NX] receives lam^0 .. lam^{nt-1} for the residual res_shot
 * ([nrec][nt]); a_out, b_out, c_out (nullable) receive the padded sponge
 * coefficients and V^2 dt^2. */
int oracle_shot_fields(const og_grid *g, const og_geom *geo, int s, const double *v,
                       const double *res_shot, double *u_hist, double *lam_hist,
                       double *a_out, double *b_out, double *c_out)
{
    shot_dom D;
    if (dom_init(&D, g, geo, s, v)) { dom_free(&D); return -1; }
    int nt = shot_nt(geo, s);
    int64_t n = (int64_t)D.NZ * D.NX;
    int64_t nrec = geo->rec_ptr[s + 1] - geo->rec_ptr[s];
    double *d = malloc((nrec * nt + 1) * sizeof(double));
    double *img = calloc((int64_t)g->nz * g->nx, sizeof(double));
    int err = (!d || !img) ? -1 : 0;
    if (!err) err = forward_shot(g, geo, s, &D, d, u_hist, NULL);
    if (!err && lam_hist) err = adjoint_shot(g, geo, s, &D, res_shot, img, lam_hist);
    if (a_out) memcpy(a_out, D.a, n * sizeof(double));
    if (b_out) memcpy(b_out, D.b, n * sizeof(double));
    if (c_out) memcpy(c_out, D.c, n * sizeof(double));
    free(d); free(img);
    dom_free(&D);
    return err;
}

/* Pad and Pad^T of one window, exported so that tests can check the
 * adjoint pair <Pad x, y> = <x, Pad^T y> directly. P is [nz+2nb][wnx+2nb]. */
void oracle_pad(const og_grid *g, int x0, int wnx, const double *v, double *P)
{
    pad_model(g, x0, wnx, v, P);
}

void oracle_pad_adjoint(const og_grid *g, int x0, int wnx, const double *P, double *img)
{
    memset(img, 0, (size_t)g->nz * g->nx * sizeof(double));
    pad_adjoint_add(g, x0, wnx, P, img);
}
