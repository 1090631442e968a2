/*
 * sph.h -- C ABI of the MI355X (gfx950) WCSPH hot path.
 *
 * The library runs one time step of a weakly compressible SPH dam break, or
 * many independent ones batched into the same launches, on one GPU:
 *
 *   cell keys -> stable radix sort of particles by cell -> cell start table
 *   (the cell linked list, direct search over the nearest cells and radix
 *   sort of the paper's Sec. 5) -> density summation sweep -> pressure and
 *   viscous force sweep -> kick-drift-kick ("two half") time integration and
 *   the FP64 reductions that give the CFL time step and the conservation
 *   diagnostics.
 *
 * Formulation, per fluid particle i over neighbours j (fluid or fixed wall
 * particles within 2h, found in the 3^d cells around i; the paper leaves the
 * discretisation unstated, the one below is the textbook WCSPH):
 *   W(r) = a_d (1-q/2)^4 (2q+1), q = r/h (Wendland C2), grad_i W = F(r) r_ij,
 *   F(r) = -5 a_d (1-q/2)^3 / h^2, a_2 = 7/(4 pi h^2), a_3 = 21/(16 pi h^3);
 *   sigma0 = sum over the lattice Z^d dx of W, m = rho0 / sigma0;
 *   rho_sum = m (W(0) + sum_j W_ij),  rho* = rho + dt sum_j m v_ij.F r_ij,
 *   rho <- rho_sum + max(0, rho* - rho_sum) rho0 / rho*,
 *   p = max(0, c0^2 (rho - rho0)), P = p / rho^2;
 *   a_i = g - sum_j m (P_i + P_j + Pi_ij) F_ij r_ij, Pi_ij the Monaghan
 *   artificial viscosity -alpha c0 h v_ij.r_ij / (rhobar (r^2 + eps h^2)) on
 *   approach; a wall j carries rho_j = rho_i, v_j = 0 and the hydrostatic
 *   mirror p_j = max(0, p_i + rho_i g.(x_j - x_i));
 *   step: v += dt/2 a; x += dt v; cells; sweeps; v += dt/2 a;
 *   dt <- min(C_ac h / (c0 + max|v|), C_f sqrt(h / max|a|)) per instance.
 *
 * Conventions
 *   - Every call returns an sph_status; no exception crosses the ABI.  A
 *     failed call leaves a message in sph_last_error() (per host thread).
 *   - Device pointers are caller-owned (allocated by the caller, e.g. torch).
 *     The library allocates no device memory: scratch lives in the caller's
 *     workspace of sph_workspace_size() bytes, or, for small cases bound with
 *     sph_bind_static, in a static device array of the library.  Pointers
 *     passed to sph_bind must stay valid until sph_destroy or the next bind.
 *   - Stage calls are stream-ordered and asynchronous; argument errors are
 *     reported synchronously; device-side conditions set sticky flags read by
 *     sph_poll_errors.  One context per stream / host thread at a time.
 *   - Per-particle arrays are structure-of-arrays, component-major: component
 *     a of particle i of an array with n particles sits at [a * n + i].
 *     Instances are concatenated in order (instance b's fluid particles occupy
 *     storage slots [fluid_offset(b), fluid_offset(b+1)), likewise walls).
 *   - Units are SI.  Indices are int32.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_E_ARG = -1,          /* invalid argument (checked on the host) */
    SPH_E_STATE = -2,        /* call out of order (e.g. step before bind/prime) */
    SPH_E_HIP = -3,          /* a HIP runtime call failed */
    SPH_E_CAPACITY = -4,     /* a size exceeds what the library supports */
    SPH_E_UNSUPPORTED = -5   /* option not available */
} sph_status;

typedef enum {
    SPH_SCHEME_WCSPH = 0,    /* the step described at the top of this file */
    SPH_SCHEME_DUAL = 1      /* dual-criteria time stepping with an acoustic
                                Riemann-solver pressure (below) */
} sph_scheme;

typedef enum {
    SPH_KEYS_ROW_MAJOR = 0,  /* cell key cx + ncx (cy + ncy cz) */
    SPH_KEYS_MORTON_TILES = 1 /* tiles of 8^d cells in row-major order, the
                                cells of a tile in Morton (Z) order; the key
                                range is padded to whole tiles */
} sph_key_order;

typedef enum {
    SPH_FP64 = 0,            /* all arithmetic in FP64 */
    SPH_MIXED = 1            /* pair sweeps on 32-bit fixed-point offsets from
                                the cell centres: FP32 force and continuity
                                sums, the summation density in FP64 from exact
                                pair differences; FP64 state, integration and
                                reductions */
} sph_precision;

/* Per-instance diagnostics, SPH_NDIAG doubles per instance, written by the
 * reductions after every step (and by sph_prime):
 *  0 max|v|   1 max|a|   2 fluid mass   3..5 momentum sum m v
 *  6 kinetic energy   7 potential energy -sum m g.x
 *  8 internal energy sum m c0^2 (ln(rho/rho0) + rho0/rho - 1) over rho > rho0
 *  9 |sum m a_ff|, the fluid-fluid force residual of the step (0 exactly)
 * 10 mean(rho)/rho0 - 1   11 clamped cell keys (cumulative)
 * 12 neighbour pairs of the step (sum of counts)
 * 13 cumulative sum of dt |sum m a_ff|   14 simulated time   15 steps done */
#define SPH_NDIAG 16

/* Sticky device flags returned by sph_poll_errors. */
#define SPH_FLAG_CLAMPED   1u   /* a particle left the grid; its key was clamped */
#define SPH_FLAG_NONFINITE 2u   /* a reduction saw a non-finite max|v| or max|a| */
#define SPH_FLAG_CAPACITY  4u   /* a neighbour list overflowed (handled, slower) */

/* Where the step runs.  SPH_POLICY_DEVICE: the HIP kernels on the current
 * GPU (buffers are device memory).  SPH_POLICY_HOST: the same per-particle and
 * per-pair bodies on the host's threads over host memory, the host execution
 * policy of the paper's single-source kernels (Sec. 4); FP64, the WCSPH
 * scheme without a skin, row-major keys; sph_prime and sph_step_batched only
 * (the stage calls, timing and sph_bind_static return SPH_E_UNSUPPORTED); no
 * workspace (sph_workspace_size gives 0); threads: the environment variable
 * SPH_HOST_THREADS, else the hardware concurrency.  Never chosen by the
 * library on its own: a device context never falls back to the host. */
typedef enum {
    SPH_POLICY_DEVICE = 0,
    SPH_POLICY_HOST = 1
} sph_policy;

typedef struct {
    int32_t n_fluid;         /* fluid particles of this instance (>= 0) */
    int32_t n_wall;          /* fixed wall particles of this instance (>= 0) */
    double tank_lo[3];       /* lower corner of the tank interior (unused axes 0) */
    double tank_hi[3];       /* upper corner of the tank interior */
    double c0;               /* artificial sound speed of this instance */
} sph_instance_desc;

typedef struct {
    int32_t dim;             /* 2 or 3; gravity acts along the last axis */
    int32_t precision;       /* sph_precision */
    int32_t n_instances;     /* >= 1 */
    int32_t reorder_every;   /* K: physical reorder of the arrays by cell every K
                                steps (0 = never); the cell table itself is
                                rebuilt every step (with a skin: on a rebuild
                                at least K steps after the last reorder) */
    double dx;               /* lattice spacing of the initial particles */
    double h;                /* smoothing length; support 2h, cell size 2h + skin */
    double rho0;             /* reference density */
    double alpha;            /* artificial viscosity coefficient */
    double eps;              /* viscosity regulariser (times h^2) */
    double cfl_ac;           /* acoustic/advective Courant number */
    double cfl_f;            /* body-force Courant number */
    double g[3];             /* gravity */
    const sph_instance_desc *inst;   /* n_instances entries (copied) */
    int32_t block_threads;   /* threads per sweep block: 0 (default 256), 64, 128, 256 */
    int32_t use_graph;       /* sph_step_batched replays captured HIP graphs */
    int32_t list_cap;        /* neighbour list per target built by the density
                                sweep and walked by both sweeps: 0 = default
                                (96 in 3D, 40 in 2D entries, times
                                ((2h + skin) / 2h)^dim), > 0 = capacity,
                                -1 = no list (both sweeps traverse the stencil).
                                A target with more neighbours than the capacity
                                traverses the stencil instead (same results)
                                and sets SPH_FLAG_CAPACITY.  With a list, each
                                instance set must hold fewer than 2^25 fluid
                                and 2^25 wall particles (else SPH_E_CAPACITY
                                from sph_create). */
    int32_t prefetch;        /* candidate records in flight per thread in the
                                density sweep: 0 = default (8), 4 or 8 */
    int32_t scheme;          /* sph_scheme.  SPH_SCHEME_DUAL needs SPH_FP64;
                                cfl_ac is then the Courant number of the
                                acoustic sub-steps (0.6 in the published
                                scheme), alpha, eps and cfl_f are unused */
    int32_t key_order;       /* sph_key_order of the cell keys (the order of
                                the particle sort and of cell_start) */
    double cfl_adv;          /* SPH_SCHEME_DUAL: advection Courant number (0.25) */
    double eta;              /* SPH_SCHEME_DUAL: slope of the Riemann dissipation
                                limiter (3) */
    double skin;             /* Verlet skin (0 <= skin <= 2h; 0 = none): cells of
                                2h + skin, lists of the neighbours within
                                2h + skin, both reused by sph_step_batched
                                until the particles may have moved skin / 2
                                (below) */
    int32_t build;           /* neighbour-list build: 0 = default (cell pairs
                                in 3D, one lane per target in 2D), 1 = one
                                lane per target, 2 = cell pairs (the sources of
                                a cell's stencil held by the lanes of a wave,
                                the cell's targets taken one at a time;
                                row-major keys and list_cap <= 255, else one
                                lane per target).  All give the same results */
    int32_t policy;          /* sph_policy: where the step runs (below) */
} sph_params;

typedef struct {
    /* fluid, storage order, N = sum of n_fluid */
    double *x;               /* [dim*N] positions */
    double *v;               /* [dim*N] velocities */
    double *a;               /* [dim*N] accelerations */
    double *rho;             /* [N] densities */
    int32_t *id;             /* [N] particle ids, reordered with the data */
    int32_t *key;            /* [N] cell key of each particle (out) */
    int32_t *perm;           /* [N] sorted slot k -> storage index (out) */
    int32_t *count;          /* [N] neighbour count of each particle (out) */
    /* walls, fixed; Nw = sum of n_wall */
    const double *xw;        /* [dim*Nw] wall particle centres (read at bind) */
    int32_t *wall_perm;      /* [Nw] wall sorted slot -> wall index (out, at bind) */
    /* cell tables over all instances, C = sum of cells (sph_get_info) */
    int32_t *cell_start;     /* [C+1] fluid: cell c holds sorted slots
                                cell_start[c] .. cell_start[c+1]-1 */
    int32_t *wall_start;     /* [C+1] walls, same convention (out, at bind) */
    /* per instance */
    double *dt;              /* [B] time step of the next step */
    double *diag;            /* [B*SPH_NDIAG] */
    /* scratch */
    void *workspace;         /* sph_workspace_size() bytes, 256-byte aligned */
} sph_buffers;

typedef struct {
    int64_t n_fluid;         /* N */
    int64_t n_wall;          /* Nw */
    int64_t n_cells;         /* C */
    size_t workspace_bytes;
    double sigma0;           /* lattice number density (1/m^d) */
    double mass;             /* particle mass rho0/sigma0 */
    double cell_size;        /* 2h + skin */
    int64_t steps_done;      /* steps since sph_prime */
    int64_t substeps_done;   /* SPH_SCHEME_DUAL: acoustic sub-steps since
                                sph_prime (per step, the largest count over
                                the instances); counted on the device, so
                                sph_get_info then waits for the device */
} sph_info;

typedef struct sph_ctx sph_ctx;

/* Message of the last failed call on this host thread ("" if none). */
const char *sph_last_error(void);

/* Validate and copy the parameters; derive sigma0, the particle mass, the cell
 * grid of every instance (origin tank_lo - 3 dx, ceil((tank extent + 6 dx) /
 * (2h + skin)) cells per axis; keys row-major, x fastest, or in tiled Morton
 * order per key_order) and the workspace layout.  No device memory is
 * touched.  On success *out owns a context to be released by sph_destroy.
 * (The paper, Sec. 5 "Cell linked-list, direct search and sorting": cells
 * for the neighbour search; Sec. 6: the dam-break workloads.) */
sph_status sph_create(const sph_params *p, sph_ctx **out);

/* Release the context and anything the library owns (host objects, graphs,
 * events); caller memory is never freed.  NULL is accepted. */
void sph_destroy(sph_ctx *ctx);

/* Sizes derived by sph_create. */
sph_status sph_get_info(const sph_ctx *ctx, sph_info *info);

/* Grid of instance b: origin lo[3], cells per axis ncell[3] and the offset of
 * its first cell in the global cell numbering (its keys are local + base). */
sph_status sph_get_grid(const sph_ctx *ctx, int32_t b, double lo[3], int32_t ncell[3],
                        int32_t *cell_base);

/* Workspace bytes the caller must allocate and pass in sph_buffers. */
sph_status sph_workspace_size(const sph_ctx *ctx, size_t *bytes);

/* Attach caller buffers (all device pointers) and build the static wall cell
 * table: wall keys, the stable sort of walls by cell (wall_perm), wall_start
 * and the sorted wall records.  Synchronises `stream` before returning.
 * (Sec. 4 "Implementing SYCL kernels in SPHinXsys": the kernel-shell layer
 * hands the kernels their data as raw pointers, usable as arrays; here the
 * caller's raw device arrays.) */
sph_status sph_bind(sph_ctx *ctx, const sph_buffers *b, void *stream);

/* Bytes of the library-owned workspace behind sph_bind_static (per device). */
#define SPH_STATIC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_bind
 * with the library's own workspace, a static device array of
 * SPH_STATIC_SCRATCH_BYTES bytes that every device using the library holds
 * until the process ends, in place of b->workspace (ignored; may be NULL).
 * The caller still passes every input and output buffer.  Calls no
 * allocating routine.  Fails with SPH_E_CAPACITY, before touching the device,
 * when sph_workspace_size() exceeds SPH_STATIC_SCRATCH_BYTES (about 100 k
 * particles of the small cases).  All contexts bound this way on one device
 * share that array: binding another context overwrites the state of the
 * previous one, and contexts used at the same time on one device race.
 * Everything a step needs to start from zero is cleared by the bind and the
 * prime, as for a caller workspace.  Synchronises `stream` before returning. */
sph_status sph_bind_static(sph_ctx *ctx, const sph_buffers *b, void *stream);

/* Step 0: cell table at the current positions, density with dt = 0 (so
 * rho <- rho_sum + max(0, rho - rho_sum) rho0/rho), forces, reductions.  Gives
 * a^0, dt^0 and diag; resets diag and the step counter.  (Sec. 4 and 5: the
 * stages of a step without its first half.) */
sph_status sph_prime(sph_ctx *ctx, void *stream);

/* Cell keys from the current positions (and the per-cell counts the sort
 * consumes).  Must be followed by sph_sort before the next sph_build_cells.
 * (Sec. 5: the cell linked list built concurrently on the device; the paper
 * inserts with atomics, here integer counts per cell then a scan, so that the
 * order inside a cell does not depend on scheduling.) */
sph_status sph_build_cells(sph_ctx *ctx, void *stream);

/* Stable radix sort of storage indices by key (perm), cell_start, and the
 * sorted sweep records.  reorder != 0 also gathers x, v, rho and id into
 * sorted order (perm becomes the identity, key the sorted keys).  (Sec. 5:
 * particles sorted on the device with a radix sort rather than a quick sort;
 * Sec. 6: the re-sort period of the benchmarks.) */
sph_status sph_sort(sph_ctx *ctx, int32_t reorder, void *stream);

/* Density sweep: rho (storage order), neighbour counts, P.  Uses dt[].
 * (Sec. 5: direct search, kernel values computed for the particles of the
 * nearest cells; Sec. 4: a particle_for over the fluid particles.  The
 * per-target neighbour list it also builds is this library's, see
 * list_cap.) */
sph_status sph_density(sph_ctx *ctx, void *stream);

/* Force sweep: a (storage order).  Does not kick.  Reads the densities and
 * pressures that sph_density writes into the sweep records, so it follows
 * sph_density (sph_sort leaves those record fields zero).  (Sec. 5: the
 * pairs of the nearest cells; Sec. 4: a particle_for.) */
sph_status sph_forces(sph_ctx *ctx, void *stream);

/* half = 1: v += dt/2 a, x += dt v, then cell keys as sph_build_cells.
 * half = 2: v += dt/2 a, then the reductions (dt[], diag[]).  (Sec. 4: the
 * per-particle updates are a particle_for, the time step and the diagnostics
 * a particle_reduce.) */
sph_status sph_integrate(sph_ctx *ctx, int32_t half, void *stream);

/* n_steps full steps of every instance: half 1 + keys, sort (with the reorder
 * on steps where steps_done % K == 0), density, force fused with half 2,
 * reductions.  dt stays on the device; asynchronous.  (Sec. 4 and 5 for the
 * stages; the instances batched into the same launches are this library's.)
 *
 * With SPH_SCHEME_DUAL a step is one advection step of every instance.  The
 * plan stays on the device: an advection step enqueues
 * ceil(11 cfl_adv / cfl_ac) sub-step slots (the most sub-steps the plan below
 * can ask for: n peaks at max|v| = c0 / 10), and each instance runs the first
 * n of them; no host synchronisation, so use_graph replays whole advection
 * steps too.  The scheme (the library
 * behind the paper, SPHinXsys; Zhang, Hu & Adams 2017 and Zhang, Rezavand &
 * Hu 2021 for the published method):
 *   advection  keys, sort, ranges (reorder every K advection steps) and the
 *              sweep records at x, which stay frozen for the sub-steps;
 *              density by summation as in sph_prime; Drho <- 0;
 *              Dt = cfl_adv h / max(max|v|, c0 / 10),
 *              n = ceil(Dt / (cfl_ac h / (c0 + max|v|))), dt = Dt / n, with
 *              max|v| from the previous reductions (dt[] holds Dt);
 *   sub-step   rho += dt/2 Drho; p = max(0, c0^2 (rho - rho0)); x += dt/2 v;
 *              a_i = g - 2 m sum_j P*_ij / (rho_i rho_j) grad_i W_ij; v += dt a;
 *              x += dt/2 v;
 *              Drho_i = 2 rho_i m sum_j (v_i - v*_ij).grad_i W_ij / rho_j;
 *              rho += dt/2 Drho;  with grad_i W_ij = F_ij r_ij and
 *              e = r_ij / |r_ij| from the frozen configuration;
 *   Riemann    U_L = -v_i.e, U_R = -v_j.e, Z = rho c0,
 *              beta = min(eta max(U_L - U_R, 0) / c0, 1),
 *              P* = (Z_L p_R + Z_R p_L + Z_L Z_R beta (U_L - U_R)) / (Z_L + Z_R),
 *              v* = (Z_L v_i + Z_R v_j) / (Z_L + Z_R) - (p_L - p_R) / (Z_L + Z_R) e;
 *   walls      rho_j = rho_i, v_j = 0, p_j = max(0, p_i + rho_i g.(x_j - x_i));
 *   then the reductions (diag as above, a and the force residual from the
 *   last sub-step) and the plan of the next advection step.
 * The stage calls (sph_build_cells ... sph_integrate) are for
 * SPH_SCHEME_WCSPH only and return SPH_E_UNSUPPORTED otherwise. */
sph_status sph_step_batched(sph_ctx *ctx, int32_t n_steps, void *stream);

/* Verlet skin (skin > 0; an extension of the cell linked list and direct
 * search of the paper's Sec. 5, after Verlet 1967): a build sorts the
 * particles into cells of 2h + skin and lists, per particle, the neighbours
 * closer than 2h + skin; every step walks those lists, skipping entries at 2h
 * or beyond, so each step sees exactly the pairs closer than 2h, as without a
 * skin (sums in list order).  The reductions that end a step bound the next
 * drift of every particle by dt (max|v| + dt max|a| / 2) per instance and add
 * the largest bound to the total since the last build; the next step rebuilds
 * when twice that total reaches skin (1 - 1e-4), all on the device, so
 * sph_step_batched stays asynchronous and graph replays stay valid.  Between
 * builds key[], perm[], cell_start[] and the neighbour list are those of the
 * last build; count[] is recounted every step.  The stage calls return
 * SPH_E_UNSUPPORTED when a skin is set.
 * With SPH_SCHEME_DUAL the sub-steps keep the pairs of their advection step,
 * so the test is exact instead: at the end of an advection step the largest
 * distance of a particle from its position at the last build, D, is taken
 * on the device, and the next advection step rebuilds when 2 D reaches
 * skin (1 - 1e-4).  The workspace then holds x at the last build
 * (dim*N doubles more). */

/* SPH_SCHEME_DUAL: the acoustic sub-step count of the next advection step of
 * each instance (n[0..B-1]).  Synchronises `stream`. */
sph_status sph_substeps(sph_ctx *ctx, int32_t *n, void *stream);

/* Number of cell-table builds (each with its neighbour lists) since
 * sph_prime, the prime's own included: steps_done + 1 without a skin.
 * Synchronises `stream` when a skin is set. */
sph_status sph_cell_builds(sph_ctx *ctx, int64_t *n, void *stream);

/* Synchronise `stream`, return the sticky device flags and clear them. */
sph_status sph_poll_errors(sph_ctx *ctx, uint32_t *flags, void *stream);

/* Per-stage GPU time.  enable != 0 records HIP events around every stage of
 * later steps (eager launches only).  sph_stage_times copies the accumulated
 * milliseconds and launch counts of up to `n` stages (names from
 * sph_stage_name) and, if reset != 0, clears them.  Synchronises `stream`. */
sph_status sph_set_timing(sph_ctx *ctx, int32_t enable);
/* The same for the stages whose bit (1 << stage index) is set in mask
 * (0 = off): fewer events, less overhead in the timed steps. */
sph_status sph_set_timing_mask(sph_ctx *ctx, uint32_t mask);
sph_status sph_stage_times(sph_ctx *ctx, double *ms, int64_t *launches, int32_t n,
                           int32_t reset, void *stream);
const char *sph_stage_name(int32_t stage);
int32_t sph_stage_count(void);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
