/*
 * Plain FP64 CPU reference ("oracle") for the WCSPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark call it; the product path never does.  It shares
 * no source, header, table or helper with the HIP library.
 *
 * What it computes (per independent instance, all in FP64):
 *   - the cell linked list of the paper's Sec. 5: a cell key per particle on a
 *     uniform grid of cell size 2h, a stable sort of particles by key and the
 *     start offset of every cell (cell c holds sorted slots start[c]..start[c+1]);
 *   - direct search over the 3^d nearest cells (Sec. 5) feeding a weakly
 *     compressible SPH step: summation density with a continuity fallback at
 *     the free surface, a linear equation of state, the symmetric pressure
 *     force with Monaghan's artificial viscosity, fixed wall particles with a
 *     hydrostatic pressure mirror, kick-drift-kick time integration, and the
 *     FP64 reductions that give the CFL time step and the conservation
 *     diagnostics.
 * The paper leaves the discretisation unstated; the formulation is the
 * textbook one (Monaghan 1992, 2005; Wendland 1995 for the kernel).
 *
 * Arrays are row-major with a stride of `dim` doubles per particle.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H

#include <stdint.h>

#define OR_NDIAG 16

typedef struct {
    /* set by the caller */
    int dim;                 /* 2 or 3 */
    double dx, h;            /* lattice spacing, smoothing length */
    double rho0, c0;         /* reference density, artificial sound speed */
    double alpha, eps;       /* viscosity coefficient, regulariser (x h^2) */
    double cfl_ac, cfl_f;    /* Courant numbers: acoustic and body force */
    double g[3];             /* gravity */
    double tank_lo[3], tank_hi[3];
    int reorder_every;       /* physical reorder of the arrays every K steps */
    /* filled by or_setup */
    double cs, inv_cs, cut2; /* cell size 2h, 1/cs, (2h)^2 */
    double sigma0, mass;     /* lattice number density, particle mass */
    double lo[3];            /* grid origin */
    int ncell[3];
    int ncells;
} or_params;

typedef struct {
    int n, nw;               /* fluid and wall particle counts */
    /* fluid, storage order */
    double *x, *v, *a;       /* n*dim */
    double *rho, *P;         /* n */
    int32_t *id, *key, *perm, *count;   /* n */
    int32_t *start;          /* ncells + 1 */
    /* walls (fixed) */
    const double *xw;        /* nw*dim */
    int32_t *wkey, *wperm, *wstart;     /* nw, nw, ncells + 1 */
    /* per instance */
    double *dt;              /* [1] */
    double *diag;            /* [OR_NDIAG] */
    int64_t *step;           /* [1] completed steps */
} or_state;

/* OpenMP threads the sweeps use. */
int or_num_threads(void);

/* Kernel and lattice constants. */
double or_kernel_alpha(int dim, double h);
double or_W(int dim, double h, double r);
double or_F(int dim, double h, double r);
double or_sigma0(int dim, double dx, double h);
int or_setup(or_params *p);

/* Stages. */
int or_keys(const or_params *p, int n, const double *x, int32_t *key);
void or_sort(int n, const int32_t *key, int ncells, int32_t *perm, int32_t *start);
void or_reorder(const or_params *p, or_state *s);
void or_density(const or_params *p, or_state *s, double dt);
void or_forces(const or_params *p, or_state *s, double *a_ff /* n*dim or NULL */);
void or_half1(const or_params *p, or_state *s, double dt);
void or_half2(const or_params *p, or_state *s, double dt);
void or_reduce(const or_params *p, or_state *s, const double *a_ff, int clamped, double dt_used);

/* Second scheme: dual-criteria time stepping with a Riemann-solver pressure
 * (definitions in sph_oracle.c). */
typedef struct {
    double cfl_adv;          /* advection Courant number (0.25) */
    double cfl_ac;           /* acoustic Courant number (0.6) */
    double eta;              /* dissipation limiter slope (3) */
} or_dual;

typedef struct {
    double *x_adv;           /* n*dim positions of the frozen configuration */
    double *drho;            /* n continuity rate of the last second half */
    double *pres;            /* n pressure of the current sub-step */
    double *a_ff;            /* n*dim fluid-fluid part of the last pressure sweep */
    double Dt, dt;           /* advection step and its sub-step */
    int nsub;                /* sub-steps per advection step */
} or_dual_state;

void or_riemann(double rho_l, double p_l, double u_l, double rho_r, double p_r, double u_r, double c0,
                double eta, double *p_star, double *u_star);
void or_dual_plan(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d);
void or_dual_summation(const or_params *p, or_state *s, or_dual_state *d);
void or_dual_first_half(const or_params *p, or_state *s, or_dual_state *d, double dt);
void or_dual_pressure(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, double dt);
void or_dual_second_half(const or_params *p, or_state *s, double dt);
void or_dual_density(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, double dt);
int or_dual_prime(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d);
int or_dual_step(const or_params *p, const or_dual *dp, or_state *s, or_dual_state *d, int nsteps);

/* Whole steps. */
int or_bind_walls(const or_params *p, or_state *s);
int or_prime(const or_params *p, or_state *s);
int or_step(const or_params *p, or_state *s, int nsteps);

#endif
