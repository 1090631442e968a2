/*
 * Plain FP64 CPU reference ("oracle") for the WCSPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it; the product path never calls it.
 * It shares no code with the HIP library.  Build: gcc -O2 -ffp-contract=off
 * -fopenmp (no FMA contraction, so the neighbour predicate and the cell keys
 * are the plain IEEE expressions written below).
 *
 * Every loop over targets is a gather: a target reads its neighbours and
 * writes only its own slots, and every sum runs in a fixed order (stencil
 * cells in z, y, x order; fluid slots of a cell in sorted order, then its wall
 * slots).  The result therefore does not depend on the OpenMP thread count.
 *
 * Formulation (the paper names the data structures only: a cell linked list,
 * direct search over the nearest cells and a radix sort by cell, Sec. 5):
 *   kernel      Wendland C2, support 2h:
 *               W(r) = a_d (1 - q/2)^4 (2q + 1), q = r/h,
 *               a_2 = 7/(4 pi h^2), a_3 = 21/(16 pi h^3);
 *               F(r) = (1/r) dW/dr = -5 a_d (1 - q/2)^3 / h^2, grad_i W = F r_ij.
 *   sigma0      number density of the perfect lattice: sum over k in Z^d of
 *               W(|k| dx); every particle has mass m = rho0 / sigma0.
 *   neighbours  all j != i, fluid or wall, in the 3^d cells around i with
 *               r^2 < (2h)^2, r^2 = ((dx*dx) + (dy*dy)) + (dz*dz).
 *   density     sigma_i = W(0) + sum_j W_ij;  Drho_i = sum_j m (v_i - v_j).F_ij r_ij;
 *               rho_sum = m sigma_i;  rho* = rho_i + dt Drho_i;
 *               rho_i <- rho_sum + max(0, rho* - rho_sum) rho0 / rho*;
 *               p = max(0, c0^2 (rho - rho0))  (no tension: negative pressure
 *               drives the tensile instability at fixed walls);  P = p / rho^2.
 *   force       a_i = g - sum_j m (P_i + P_j + Pi_ij) F_ij r_ij with
 *               Pi_ij = -alpha c0 h (v_ij.r_ij) / (rhobar_ij (r^2 + eps h^2))
 *               when v_ij.r_ij < 0, else 0.  A wall j mirrors the target:
 *               rho_j = rho_i, p_j = max(0, p_i + rho_i g.(x_j - x_i)), v_j = 0.
 *   step        v += dt/2 a;  x += dt v;  keys, sort, ranges (and every K steps
 *               a physical reorder of the arrays);  density;  force;
 *               v += dt/2 a;  dt <- min(C_ac h / (c0 + max|v|), C_f sqrt(h / max|a|)).
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Kernel                                                                   */
/* ------------------------------------------------------------------------ */

double or_kernel_alpha(int dim, double h)
{
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    return 21.0 / (16.0 * M_PI * h * h * h);
}

double or_W(int dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return or_kernel_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

double or_F(int dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * or_kernel_alpha(dim, h) * t * t * t / (h * h);
}

double or_sigma0(int dim, double dx, double h)
{
    int K = (int)ceil(2.0 * h / dx) + 1;
    double s = 0.0;
    int kz_lo = (dim == 3) ? -K : 0, kz_hi = (dim == 3) ? K : 0;
    for (int kz = kz_lo; kz <= kz_hi; ++kz)
        for (int ky = -K; ky <= K; ++ky)
            for (int kx = -K; kx <= K; ++kx) {
                double r2 = (double)(kx * kx + ky * ky + kz * kz) * dx * dx;
                s += or_W(dim, h, sqrt(r2));
            }
    return s;
}

int or_setup(or_params *p)
{
    if (p->dim != 2 && p->dim != 3) return -1;
    if (!(p->dx > 0.0) || !(p->h > 0.0)) return -1;
    p->cs = 2.0 * p->h;
    p->inv_cs = 1.0 / p->cs;
    p->cut2 = p->cs * p->cs;
    p->sigma0 = or_sigma0(p->dim, p->dx, p->h);
    p->mass = p->rho0 / p->sigma0;
    long total = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < p->dim) {
            p->lo[a] = p->tank_lo[a] - 3.0 * p->dx;
            double ext = (p->tank_hi[a] - p->tank_lo[a]) + 6.0 * p->dx;
            p->ncell[a] = (int)ceil(ext / p->cs);
            if (p->ncell[a] < 1) p->ncell[a] = 1;
        } else {
            p->lo[a] = 0.0;
            p->ncell[a] = 1;
        }
        total *= p->ncell[a];
    }
    if (total > 0x7fffffffL) return -2;
    p->ncells = (int)total;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cell linked list                                                         */
/* ------------------------------------------------------------------------ */

/* Cell index along one axis: floor((x - lo) * inv_cs), clamped to the grid.
 * Non-finite or out-of-grid coordinates are clamped and reported. */
static int cell_1d(double x, double lo, double inv_cs, int n, int *clamped)
{
    double t = floor((x - lo) * inv_cs);
    if (!(t >= 0.0)) { *clamped = 1; return 0; }
    if (t >= (double)n) { *clamped = 1; return n - 1; }
    return (int)t;
}

static int32_t cell_key(const or_params *p, const double *xi, int *clamped)
{
    int c[3] = {0, 0, 0};
    for (int a = 0; a < p->dim; ++a)
        c[a] = cell_1d(xi[a], p->lo[a], p->inv_cs, p->ncell[a], clamped);
    return (int32_t)(c[0] + p->ncell[0] * (c[1] + p->ncell[1] * c[2]));
}

int or_keys(const or_params *p, int n, const double *x, int32_t *key)
{
    int nclamped = 0;
#pragma omp parallel for reduction(+ : nclamped) schedule(static)
    for (int i = 0; i < n; ++i) {
        int cl = 0;
        key[i] = cell_key(p, x + (long)i * p->dim, &cl);
        nclamped += cl;
    }
    return nclamped;
}

/* Stable sort of storage indices by key, written as its definition: cells in
 * increasing key order, and inside a cell the indices in storage order.
 * start[c] = number of particles with key < c (start[ncells] = n). */
void or_sort(int n, const int32_t *key, int ncells, int32_t *perm, int32_t *start)
{
    int32_t *fill = (int32_t *)calloc((size_t)ncells + 1, sizeof(int32_t));
    for (int c = 0; c <= ncells; ++c) start[c] = 0;
    for (int i = 0; i < n; ++i) start[key[i] + 1] += 1;
    for (int c = 0; c < ncells; ++c) start[c + 1] += start[c];
    for (int c = 0; c < ncells; ++c) fill[c] = start[c];
    for (int i = 0; i < n; ++i) perm[fill[key[i]]++] = i;
    free(fill);
}

static void gather_d(double *arr, const int32_t *perm, int n, int stride)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n * stride);
    for (int k = 0; k < n; ++k)
        for (int a = 0; a < stride; ++a) tmp[(long)k * stride + a] = arr[(long)perm[k] * stride + a];
    memcpy(arr, tmp, sizeof(double) * (size_t)n * stride);
    free(tmp);
}

static void gather_i(int32_t *arr, const int32_t *perm, int n)
{
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int k = 0; k < n; ++k) tmp[k] = arr[perm[k]];
    memcpy(arr, tmp, sizeof(int32_t) * (size_t)n);
    free(tmp);
}

/* Physical reorder: every per-particle array takes the sorted order, after
 * which the sort permutation is the identity. */
void or_reorder(const or_params *p, or_state *s)
{
    int n = s->n;
    gather_d(s->x, s->perm, n, p->dim);
    gather_d(s->v, s->perm, n, p->dim);
    gather_d(s->a, s->perm, n, p->dim);
    gather_d(s->rho, s->perm, n, 1);
    gather_d(s->P, s->perm, n, 1);
    gather_i(s->id, s->perm, n);
    gather_i(s->key, s->perm, n);
    gather_i(s->count, s->perm, n);
    for (int k = 0; k < n; ++k) s->perm[k] = k;
}

/* ------------------------------------------------------------------------ */
/* Pair sweeps                                                              */
/* ------------------------------------------------------------------------ */

/* Squared distance, summed left to right without fused multiply-add, and the
 * separation vector r_ij = x_i - x_j. */
static double dist2(int dim, const double *xi, const double *xj, double *r)
{
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
        r[a] = xi[a] - xj[a];
        double sq = r[a] * r[a];
        s = (a == 0) ? sq : s + sq;
    }
    return s;
}

static void cell_coords(const or_params *p, int32_t key, int c[3])
{
    c[0] = key % p->ncell[0];
    c[1] = (key / p->ncell[0]) % p->ncell[1];
    c[2] = key / (p->ncell[0] * p->ncell[1]);
}

/* Visits every neighbour of fluid target i in the fixed order described at the
 * top of the file.  kind = 0 for fluid sources, 1 for walls. */
typedef void (*pair_fn)(void *ctx, int kind, int j, double r2, const double *r);

/* The same with the fluid positions taken from xf (the table must have been
 * built at those positions). */
static void for_neighbours_at(const or_params *p, const or_state *s, const double *xf, int i, pair_fn fn,
                              void *ctx);

static void for_neighbours(const or_params *p, const or_state *s, int i, pair_fn fn, void *ctx)
{
    for_neighbours_at(p, s, s->x, i, fn, ctx);
}

static void for_neighbours_at(const or_params *p, const or_state *s, const double *xf, int i, pair_fn fn,
                              void *ctx)
{
    int dim = p->dim;
    const double *xi = xf + (long)i * dim;
    int c[3];
    cell_coords(p, s->key[i], c);
    int dz_lo = (dim == 3) ? -1 : 0, dz_hi = (dim == 3) ? 1 : 0;
    double r[3];
    for (int dz = dz_lo; dz <= dz_hi; ++dz) {
        int cz = c[2] + dz;
        if (cz < 0 || cz >= p->ncell[2]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = c[1] + dy;
            if (cy < 0 || cy >= p->ncell[1]) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int cx = c[0] + dx;
                if (cx < 0 || cx >= p->ncell[0]) continue;
                int cell = cx + p->ncell[0] * (cy + p->ncell[1] * cz);
                for (int k = s->start[cell]; k < s->start[cell + 1]; ++k) {
                    int j = s->perm[k];
                    if (j == i) continue;
                    double r2 = dist2(dim, xi, xf + (long)j * dim, r);
                    if (r2 < p->cut2) fn(ctx, 0, j, r2, r);
                }
                for (int k = s->wstart[cell]; k < s->wstart[cell + 1]; ++k) {
                    int j = s->wperm[k];
                    double r2 = dist2(dim, xi, s->xw + (long)j * dim, r);
                    if (r2 < p->cut2) fn(ctx, 1, j, r2, r);
                }
            }
        }
    }
}

typedef struct {
    const or_params *p;
    const or_state *s;
    int i;
    double sigma, drho;
    int count;
} dens_ctx;

static void dens_pair(void *vc, int kind, int j, double r2, const double *r)
{
    dens_ctx *c = (dens_ctx *)vc;
    const or_params *p = c->p;
    int dim = p->dim;
    double rr = sqrt(r2);
    double W = or_W(dim, p->h, rr);
    double F = or_F(dim, p->h, rr);
    const double *vi = c->s->v + (long)c->i * dim;
    double vr = 0.0;
    for (int a = 0; a < dim; ++a) {
        double vj = (kind == 0) ? c->s->v[(long)j * dim + a] : 0.0;
        vr += (vi[a] - vj) * r[a];
    }
    c->sigma += W;
    c->drho += p->mass * vr * F;
    c->count += 1;
}

void or_density(const or_params *p, or_state *s, double dt)
{
    double W0 = or_W(p->dim, p->h, 0.0);
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < s->n; ++i) {
        dens_ctx c = {p, s, i, W0, 0.0, 0};
        for_neighbours(p, s, i, dens_pair, &c);
        double rho_sum = p->mass * c.sigma;
        double rho_star = s->rho[i] + dt * c.drho;
        double excess = rho_star - rho_sum;
        /* the free-surface term max(0, rho* - rho_sum) rho0/rho* is zero
         * unless the excess is positive (then rho* > rho_sum >= 0) */
        double rho = (excess > 0.0) ? rho_sum + excess * p->rho0 / rho_star : rho_sum;
        double pr = p->c0 * p->c0 * (rho - p->rho0);
        if (pr < 0.0) pr = 0.0;
        s->rho[i] = rho;
        s->P[i] = pr / (rho * rho);
        s->count[i] = c.count;
    }
}

typedef struct {
    const or_params *p;
    const or_state *s;
    int i;
    double acc[3], acc_ff[3];
} force_ctx;

static void force_pair(void *vc, int kind, int j, double r2, const double *r)
{
    force_ctx *c = (force_ctx *)vc;
    const or_params *p = c->p;
    const or_state *s = c->s;
    int dim = p->dim, i = c->i;
    double rr = sqrt(r2);
    double F = or_F(dim, p->h, rr);
    double rho_i = s->rho[i];
    double P_i = s->P[i];
    double rho_j, P_j, vr = 0.0;
    const double *vi = s->v + (long)i * dim;
    if (kind == 0) {
        rho_j = s->rho[j];
        P_j = s->P[j];
        for (int a = 0; a < dim; ++a) vr += (vi[a] - s->v[(long)j * dim + a]) * r[a];
    } else {
        /* hydrostatic mirror of the target: p_j = p_i + rho_i g.(x_j - x_i) */
        double p_i = p->c0 * p->c0 * (rho_i - p->rho0);
        if (p_i < 0.0) p_i = 0.0;
        double gx = 0.0;
        for (int a = 0; a < dim; ++a) gx += p->g[a] * (s->xw[(long)j * dim + a] - s->x[(long)i * dim + a]);
        double p_j = p_i + rho_i * gx;
        if (p_j < 0.0) p_j = 0.0;
        rho_j = rho_i;
        P_j = p_j / (rho_i * rho_i);
        for (int a = 0; a < dim; ++a) vr += vi[a] * r[a];
    }
    double visc = 0.0;
    if (vr < 0.0) {
        double rho_bar = 0.5 * (rho_i + rho_j);
        visc = -p->alpha * p->c0 * p->h * vr / (rho_bar * (r2 + p->eps * p->h * p->h));
    }
    double coef = p->mass * (P_i + P_j + visc) * F;
    for (int a = 0; a < dim; ++a) {
        c->acc[a] -= coef * r[a];
        if (kind == 0) c->acc_ff[a] -= coef * r[a];
    }
}

void or_forces(const or_params *p, or_state *s, double *a_ff)
{
    int dim = p->dim;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < s->n; ++i) {
        force_ctx c;
        c.p = p; c.s = s; c.i = i;
        for (int a = 0; a < 3; ++a) { c.acc[a] = 0.0; c.acc_ff[a] = 0.0; }
        for_neighbours(p, s, i, force_pair, &c);
        for (int a = 0; a < dim; ++a) {
            s->a[(long)i * dim + a] = p->g[a] + c.acc[a];
            if (a_ff) a_ff[(long)i * dim + a] = c.acc_ff[a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Time integration and reductions                                          */
/* ------------------------------------------------------------------------ */

void or_half1(const or_params *p, or_state *s, double dt)
{
    int dim = p->dim;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < dim; ++a) {
            long k = (long)i * dim + a;
            s->v[k] = s->v[k] + 0.5 * dt * s->a[k];
            s->x[k] = s->x[k] + dt * s->v[k];
        }
}

void or_half2(const or_params *p, or_state *s, double dt)
{
    int dim = p->dim;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < dim; ++a) {
            long k = (long)i * dim + a;
            s->v[k] = s->v[k] + 0.5 * dt * s->a[k];
        }
}

/* Diagnostics slots (per instance):
 *  0 max|v|   1 max|a|   2 fluid mass   3..5 momentum sum m v
 *  6 kinetic  7 potential (-m g.x)
 *  8 internal: m c0^2 (ln(rho/rho0) + rho0/rho - 1) for rho > rho0, else 0
 *    (du/drho = p/rho^2 for the clipped equation of state)
 *  9 |sum m a_ff| (fluid-fluid force residual of this step)
 * 10 mean(rho)/rho0 - 1   11 clamped keys (cumulative)   12 neighbour pairs (this step)
 * 13 cumulative sum of dt |sum m a_ff|   14 simulated time   15 completed steps */
void or_reduce(const or_params *p, or_state *s, const double *a_ff, int clamped, double dt_used)
{
    int dim = p->dim;
    double vmax = 0.0, amax = 0.0, mom[3] = {0, 0, 0}, ke = 0.0, pe = 0.0, ie = 0.0;
    double ff[3] = {0, 0, 0}, rsum = 0.0, pairs = 0.0;
    double m = p->mass, c2 = p->c0 * p->c0;
    for (int i = 0; i < s->n; ++i) {
        double v2 = 0.0, a2 = 0.0, gx = 0.0;
        for (int a = 0; a < dim; ++a) {
            double va = s->v[(long)i * dim + a], aa = s->a[(long)i * dim + a];
            v2 += va * va;
            a2 += aa * aa;
            gx += p->g[a] * s->x[(long)i * dim + a];
            mom[a] += m * va;
            if (a_ff) ff[a] += m * a_ff[(long)i * dim + a];
        }
        double vi = sqrt(v2), ai = sqrt(a2);
        if (vi > vmax) vmax = vi;
        if (ai > amax) amax = ai;
        double rho = s->rho[i];
        ke += 0.5 * m * v2;
        pe += -m * gx;
        if (rho > p->rho0) ie += m * c2 * (log(rho / p->rho0) + p->rho0 / rho - 1.0);
        rsum += rho;
        pairs += (double)s->count[i];
    }
    double *d = s->diag;
    d[0] = vmax;
    d[1] = amax;
    d[2] = m * (double)s->n;
    for (int a = 0; a < 3; ++a) d[3 + a] = mom[a];
    d[6] = ke;
    d[7] = pe;
    d[8] = ie;
    d[9] = sqrt(ff[0] * ff[0] + ff[1] * ff[1] + ff[2] * ff[2]);
    d[10] = (s->n > 0) ? rsum / ((double)s->n * p->rho0) - 1.0 : 0.0;
    d[11] += (double)clamped;
    d[12] = pairs;
    d[13] += dt_used * d[9];
    d[14] += dt_used;
    double dt_ac = p->cfl_ac * p->h / (p->c0 + vmax);
    double dt_f = p->cfl_f * sqrt(p->h / amax);
    s->dt[0] = (dt_ac < dt_f) ? dt_ac : dt_f;
}

/* ------------------------------------------------------------------------ */
/* Whole steps                                                              */
/* ------------------------------------------------------------------------ */

int or_bind_walls(const or_params *p, or_state *s)
{
    int cl = or_keys(p, s->nw, s->xw, s->wkey);
    or_sort(s->nw, s->wkey, p->ncells, s->wperm, s->wstart);
    return cl;
}

/* Step 0: table at x0, density with dt = 0, force, reductions (no kick). */
int or_prime(const or_params *p, or_state *s)
{
    int cl = or_keys(p, s->n, s->x, s->key);
    or_sort(s->n, s->key, p->ncells, s->perm, s->start);
    or_density(p, s, 0.0);
    double *a_ff = (double *)malloc(sizeof(double) * (size_t)(s->n > 0 ? s->n : 1) * p->dim);
    or_forces(p, s, a_ff);
    or_reduce(p, s, a_ff, cl, 0.0);
    s->diag[15] = 0.0;
    *s->step = 0;
    free(a_ff);
    return cl;
}

int or_step(const or_params *p, or_state *s, int nsteps)
{
    double *a_ff = (double *)malloc(sizeof(double) * (size_t)(s->n > 0 ? s->n : 1) * p->dim);
    int total_clamped = 0;
    for (int it = 0; it < nsteps; ++it) {
        double dt = s->dt[0];
        or_half1(p, s, dt);
        int cl = or_keys(p, s->n, s->x, s->key);
        or_sort(s->n, s->key, p->ncells, s->perm, s->start);
        if (p->reorder_every > 0 && (*s->step % p->reorder_every) == 0) or_reorder(p, s);
        or_density(p, s, dt);
        or_forces(p, s, a_ff);
        or_half2(p, s, dt);
        or_reduce(p, s, a_ff, cl, dt);
        *s->step += 1;
        s->diag[15] = (double)*s->step;
        total_clamped += cl;
    }
    free(a_ff);
    return total_clamped;
}

/* ------------------------------------------------------------------------ */
/* Dual-criteria time stepping with a Riemann-solver pressure (second       */
/* scheme).                                                                 */
/*                                                                          */
/* The library behind the paper (SPHinXsys) advances weakly compressible     */
/* flow with two time-step criteria: an advection step Dt that rebuilds the  */
/* cell table and the neighbour configuration and resets the density by      */
/* summation, and several acoustic sub-steps dt inside it that relax          */
/* pressure and density against the configuration frozen at the advection   */
/* step, with interface states from a linearised (acoustic) Riemann problem   */
/* along each pair in place of artificial viscosity (Zhang, Hu & Adams 2017;  */
/* Zhang, Rezavand & Hu 2021).  Written here from that description:           */
/*                                                                          */
/*   advection   keys, sort, ranges (reorder every K advection steps) at x;  */
/*               x_adv <- x; density by summation with the free-surface      */
/*               rule (or_density with dt = 0); Drho <- 0.                    */
/*               Dt = C_adv h / max(max|v|, U_ref), U_ref = c0 / 10;          */
/*               n = ceil(Dt / (C_ac' h / (c0 + max|v|))), dt = Dt / n, with  */
/*               max|v| taken at the end of the previous advection step.      */
/*   sub-step    rho += dt/2 Drho;  p = max(0, c0^2 (rho - rho0));  x += dt/2 v;*/
/*               a_i = g - 2 sum_j m P*_ij / (rho_i rho_j) grad_i W_ij;       */
/*               v += dt a;  x += dt/2 v;                                     */
/*               Drho_i = 2 rho_i sum_j (m / rho_j) (v_i - v*_ij).grad_i W_ij; */
/*               rho += dt/2 Drho.                                            */
/*   geometry    grad_i W_ij = F_ij r_ij and e_ij = r_ij / |r_ij| from x_adv  */
/*               (the frozen configuration), for all sub-steps.               */
/*   Riemann     along e = e_ij: U_L = -v_i.e, U_R = -v_j.e, Z = rho c0;      */
/*               beta = min(eta max(U_L - U_R, 0) / c0, 1), eta = 3;          */
/*               P* = (Z_L p_R + Z_R p_L + Z_L Z_R beta (U_L - U_R)) / (Z_L + Z_R);*/
/*               v* = (Z_L v_i + Z_R v_j) / (Z_L + Z_R) - (p_L - p_R) / (Z_L + Z_R) e.*/
/*   walls       rho_j = rho_i, p_j = max(0, p_i + rho_i g.(x_j - x_i^adv)), v_j = 0.*/
/* Each sweep computes all targets from the previous values before any is    */
/* updated (gathers into scratch, then the update).                          */
/* ------------------------------------------------------------------------ */

void or_riemann(double rho_l, double p_l, double u_l, double rho_r, double p_r, double u_r, double c0,
                double eta, double *p_star, double *u_star)
{
    double zl = rho_l * c0, zr = rho_r * c0;
    double du = u_l - u_r;
    double beta = eta * (du > 0.0 ? du : 0.0) / c0;
    if (beta > 1.0) beta = 1.0;
    double zs = zl + zr;
    *p_star = (zl * p_r + zr * p_l + zl * zr * beta * du) / zs;
    *u_star = (zl * u_l + zr * u_r + (p_l - p_r)) / zs;
}

void or_dual_plan(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d)
{
    double vmax = s->diag[0];
    double uref = p->c0 / 10.0;
    double Dt = dp->cfl_adv * p->h / (vmax > uref ? vmax : uref);
    double dac = dp->cfl_ac * p->h / (p->c0 + vmax);
    int nsub = (int)ceil(Dt / dac);
    if (nsub < 1) nsub = 1;
    d->Dt = Dt;
    d->nsub = nsub;
    d->dt = Dt / (double)nsub;
    s->dt[0] = Dt;
}

static double eos_clipped(const or_params *p, double rho)
{
    double pr = p->c0 * p->c0 * (rho - p->rho0);
    return pr < 0.0 ? 0.0 : pr;
}

void or_dual_summation(const or_params *p, or_state *s, or_dual_state *d)
{
    or_density(p, s, 0.0);
    memcpy(d->x_adv, s->x, sizeof(double) * (size_t)s->n * p->dim);
    for (int i = 0; i < s->n; ++i) d->drho[i] = 0.0;
}

void or_dual_first_half(const or_params *p, or_state *s, or_dual_state *d, double dt)
{
    int dim = p->dim;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) {
        s->rho[i] = s->rho[i] + 0.5 * dt * d->drho[i];
        d->pres[i] = eos_clipped(p, s->rho[i]);
        for (int a = 0; a < dim; ++a) {
            long k = (long)i * dim + a;
            s->x[k] = s->x[k] + 0.5 * dt * s->v[k];
        }
    }
}

typedef struct {
    const or_params *p;
    const or_dual *dp;
    const or_state *s;
    const or_dual_state *d;
    int i;
    double acc[3], acc_ff[3], drho;
} dual_ctx;

/* Interface state of pair (i, j): pressure P* and the velocity jump v_i - v*. */
static void dual_pair_state(dual_ctx *c, int kind, int j, double r2, const double *r, double *pstar,
                            double *dv, double *rho_j_out)
{
    const or_params *p = c->p;
    const or_state *s = c->s;
    const or_dual_state *d = c->d;
    int dim = p->dim, i = c->i;
    double rho_i = s->rho[i], p_i = d->pres[i];
    double rho_j, p_j, vj[3] = {0.0, 0.0, 0.0};
    if (kind == 0) {
        rho_j = s->rho[j];
        p_j = d->pres[j];
        for (int a = 0; a < dim; ++a) vj[a] = s->v[(long)j * dim + a];
    } else {
        double gx = 0.0;
        for (int a = 0; a < dim; ++a) gx += p->g[a] * (s->xw[(long)j * dim + a] - d->x_adv[(long)i * dim + a]);
        p_j = p_i + rho_i * gx;
        if (p_j < 0.0) p_j = 0.0;
        rho_j = rho_i;
    }
    double rr = sqrt(r2);
    double e[3] = {0.0, 0.0, 0.0};
    if (rr > 0.0)
        for (int a = 0; a < dim; ++a) e[a] = r[a] / rr;
    const double *vi = s->v + (long)i * dim;
    double ul = 0.0, ur = 0.0;
    for (int a = 0; a < dim; ++a) {
        ul -= vi[a] * e[a];
        ur -= vj[a] * e[a];
    }
    double ps, us;
    or_riemann(rho_i, p_i, ul, rho_j, p_j, ur, p->c0, c->dp->eta, &ps, &us);
    double zl = rho_i * p->c0, zr = rho_j * p->c0, zs = zl + zr;
    /* v_i - v* = Z_R (v_i - v_j) / (Z_L + Z_R) + (p_L - p_R) / (Z_L + Z_R) e */
    for (int a = 0; a < dim; ++a) dv[a] = zr * (vi[a] - vj[a]) / zs + (p_i - p_j) / zs * e[a];
    *pstar = ps;
    *rho_j_out = rho_j;
}

static void dual_force_pair(void *vc, int kind, int j, double r2, const double *r)
{
    dual_ctx *c = (dual_ctx *)vc;
    const or_params *p = c->p;
    int dim = p->dim;
    double ps, dv[3], rho_j;
    dual_pair_state(c, kind, j, r2, r, &ps, dv, &rho_j);
    double F = or_F(dim, p->h, sqrt(r2));
    double coef = 2.0 * p->mass * ps / (c->s->rho[c->i] * rho_j) * F;
    for (int a = 0; a < dim; ++a) {
        c->acc[a] -= coef * r[a];
        if (kind == 0) c->acc_ff[a] -= coef * r[a];
    }
}

void or_dual_pressure(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, double dt)
{
    int dim = p->dim;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < s->n; ++i) {
        dual_ctx c;
        c.p = p; c.dp = dp; c.s = s; c.d = d; c.i = i; c.drho = 0.0;
        for (int a = 0; a < 3; ++a) { c.acc[a] = 0.0; c.acc_ff[a] = 0.0; }
        for_neighbours_at(p, s, d->x_adv, i, dual_force_pair, &c);
        for (int a = 0; a < dim; ++a) {
            s->a[(long)i * dim + a] = p->g[a] + c.acc[a];
            d->a_ff[(long)i * dim + a] = c.acc_ff[a];
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < dim; ++a) {
            long k = (long)i * dim + a;
            s->v[k] = s->v[k] + dt * s->a[k];
        }
}

void or_dual_second_half(const or_params *p, or_state *s, double dt)
{
    int dim = p->dim;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < dim; ++a) {
            long k = (long)i * dim + a;
            s->x[k] = s->x[k] + 0.5 * dt * s->v[k];
        }
}

static void dual_density_pair(void *vc, int kind, int j, double r2, const double *r)
{
    dual_ctx *c = (dual_ctx *)vc;
    const or_params *p = c->p;
    int dim = p->dim;
    double ps, dv[3], rho_j;
    dual_pair_state(c, kind, j, r2, r, &ps, dv, &rho_j);
    double F = or_F(dim, p->h, sqrt(r2));
    double dot = 0.0;
    for (int a = 0; a < dim; ++a) dot += dv[a] * r[a];
    c->drho += p->mass / rho_j * dot * F;
}

void or_dual_density(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, double dt)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < s->n; ++i) {
        dual_ctx c;
        c.p = p; c.dp = dp; c.s = s; c.d = d; c.i = i; c.drho = 0.0;
        for (int a = 0; a < 3; ++a) { c.acc[a] = 0.0; c.acc_ff[a] = 0.0; }
        for_neighbours_at(p, s, d->x_adv, i, dual_density_pair, &c);
        d->drho[i] = 2.0 * s->rho[i] * c.drho;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) s->rho[i] = s->rho[i] + 0.5 * dt * d->drho[i];
}

static void dual_substep(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, double dt)
{
    or_dual_first_half(p, s, d, dt);
    or_dual_pressure(p, dp, s, d, dt);
    or_dual_second_half(p, s, dt);
    or_dual_density(p, dp, s, d, dt);
}

/* Table and summation at x0, one pressure sweep with v = 0 (for the
 * diagnostics), reductions, and the plan of the first advection step. */
int or_dual_prime(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d)
{
    int cl = or_keys(p, s->n, s->x, s->key);
    or_sort(s->n, s->key, p->ncells, s->perm, s->start);
    or_dual_summation(p, s, d);
    for (int i = 0; i < s->n; ++i) d->pres[i] = eos_clipped(p, s->rho[i]);
    or_dual_pressure(p, dp, s, d, 0.0);
    or_reduce(p, s, d->a_ff, cl, 0.0);
    s->diag[15] = 0.0;
    *s->step = 0;
    or_dual_plan(p, dp, s, d);
    return cl;
}

int or_dual_step(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, int nsteps)
{
    int total_clamped = 0;
    for (int it = 0; it < nsteps; ++it) {
        int cl = or_keys(p, s->n, s->x, s->key);
        or_sort(s->n, s->key, p->ncells, s->perm, s->start);
        if (p->reorder_every > 0 && (*s->step % p->reorder_every) == 0) or_reorder(p, s);
        or_dual_summation(p, s, d);
        double Dt = d->Dt;
        for (int k = 0; k < d->nsub; ++k) dual_substep(p, dp, s, d, d->dt);
        or_reduce(p, s, d->a_ff, cl, Dt);
        *s->step += 1;
        s->diag[15] = (double)*s->step;
        or_dual_plan(p, dp, s, d);
        total_clamped += cl;
    }
    return total_clamped;
}
