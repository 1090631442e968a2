// Host-side launchers of the libsph kernels (internal to the library).
#pragma once

#include "sph_device.h"

namespace sphx {

// ---- scan and sort (sph_sort.hip) ---------------------------------------
int scan_tiles(int64_t n);
int64_t scan_max_elems();
int radix_tiles(int64_t n);
int radix_passes(int64_t ncells);
// gate: null, or a device int; every kernel of the call returns at once
// when *gate == 0 (a step that reuses its cell table).
hipError_t launch_exclusive_scan(int *in, int *out, int64_t n, int *part, int zero_in,
                                 hipStream_t s, const int *gate = nullptr);
hipError_t launch_radix_sort(const int *keys, int64_t n, int64_t ncells, int *skey, int *perm,
                             int *k0, int *v0, int *k1, int *v1, int *hist, int *part,
                             hipStream_t s, const int *gate = nullptr);

// ---- physics (sph_kernels.hip, sph_sweeps.hip) ----------------------------
struct Dev {
    // caller buffers
    double *x, *v, *a, *rho;
    int *id, *key, *perm, *count;
    const double *xw;
    int *wall_perm, *cell_start, *wall_start;
    double *dt, *diag;
    // workspace
    int *skey, *rk0, *rv0, *rk1, *rv1, *hist, *part;
    int *cnt;                 // [C+1] per-cell counts (zero between steps)
    void *rec;                // [2N] sorted fluid sweep records (two 4-vectors each)
    void *wpos;               // [Nw] sorted wall records
    void *cpos, *wcpos;       // FP32 cell-offset copies for candidate tests (FP64 path)
    int *wkey, *wskey;        // wall keys (storage, sorted)
    double *scratch;          // reorder gather buffer
    double *partials;         // [nchunks * kNPart]
    Chunk *rmap;              // first reduction level: block -> (instance, rows of partials, output row)
    double *subpart;          // [nrblocks * kNPart] its sums
    int nrblocks;
    Chunk *fmap, *wmap;
    InstDev *inst;
    unsigned *flags;
    int *clampc;              // [B] clamped keys of the current step
    int nfchunks, nwchunks;
    int block;                // threads per chunk
    uint4 *nlist;             // [list_cap/4 * N] neighbour list in quads, slot-major
    int *lcount;              // [N] hits per sorted target (may exceed list_cap)
    int list_cap;             // 0: sweeps traverse the stencil (no list)
    int prefetch;             // candidate records in flight per thread (4 or 8)
    bool cell_pair;           // list build as cell pairs where it applies
    // dual scheme
    double *drho;             // [N] continuity rate of the last density relaxation
    int *nsub;                // [B] acoustic sub-steps of the next advection step
    double *dtsub;            // [B] their size
    int *nsub_max;            // [1] max over instances
    unsigned long long *subs_total;   // [1] sub-steps of the advection steps since the prime
    // Verlet skin (null / unused without one): gate[0] rebuild the cell table
    // and the list this step, gate[1] reorder this step, gate[2] steps since
    // the last reorder, gate[3] reduction blocks done, gate[4] builds since
    // the prime; disp[0] displacement bound since the last build, disp[1] the
    // largest bound of the next drift over the instances (as ordered bits)
    int *gate;
    double *disp;
    double *xb;               // [dim*N] positions at the last build (dual scheme with a skin)
};

hipError_t launch_fill_i32(int *p, int64_t n, int val, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double val, hipStream_t s);

// Keys (optionally after the half-1 kick and drift) and per-cell counts; with
// a skin only on build steps (gate[0] != 0).
hipError_t launch_keys(const SimConst &sc, const Dev &d, int kick, hipStream_t s);
// Wall keys and counts (bind time).
hipError_t launch_wall_keys(const SimConst &sc, const Dev &d, hipStream_t s);
// Sorted wall records (bind time).
hipError_t launch_wall_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s);
// Gather x, v, rho, id into sorted order; perm <- identity; key <- sorted keys.
hipError_t launch_reorder(const SimConst &sc, const Dev &d, hipStream_t s);
// Sorted sweep records from the storage-order state.  With a skin, on a step
// that reuses its cell table (gate[0] == 0) and kick_on != 0, the half-1 kick
// and drift happen here (launch_keys then returns at once).
hipError_t launch_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s, int kick_on = 0);
// Density sweep (sph_sweeps.hip).  use_dt = 0 for the prime (dt = 0).  With
// list_cap > 0 it also writes the per-step neighbour list.
hipError_t launch_density(const SimConst &sc, const Dev &d, int mixed, int use_dt, hipStream_t s);
// Candidate tests and neighbour lists (before launch_density, which then
// walks them); with a skin only on build steps.
hipError_t launch_build(const SimConst &sc, const Dev &d, int mixed, hipStream_t s);
// Force sweep.  fused != 0: also v += dt/2 a and all per-chunk partials.
// list != 0: walk the neighbour list written by this step's density sweep.
hipError_t launch_force(const SimConst &sc, const Dev &d, int mixed, int fused, int list, hipStream_t s);
// Staged half 2: v += dt/2 a (kick_on != 0) and the partials the force sweep
// does not write.
hipError_t launch_half2(const SimConst &sc, const Dev &d, hipStream_t s, int kick_on);
// Dual-criteria scheme (sph_sweeps.hip): the four kernels of acoustic
// sub-step `sub` of the current advection step; instances with fewer
// sub-steps skip it.  list != 0: the sweeps walk the neighbour list of the
// advection step's summation.
hipError_t launch_dual_substep(const SimConst &sc, const Dev &d, int sub, int list, hipStream_t s, int part);
// Dual scheme with a skin: the largest displacement since the last build
// decides the gates of the next advection step; x is saved at each build.
hipError_t launch_skin_displacement(const SimConst &sc, const Dev &d, hipStream_t s);
hipError_t launch_save_build_positions(const SimConst &sc, const Dev &d, hipStream_t s);
// Per-instance reductions of the partials -> dt, diag, flags.
hipError_t launch_final_reduce(const SimConst &sc, const Dev &d, int prime, hipStream_t s);
hipError_t launch_count_substeps(const Dev &d, hipStream_t s);

}  // namespace sphx
