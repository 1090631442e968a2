// Device-side types and helpers shared by the HIP kernels of libsph.
//
// Particle data on the GPU:
//   storage order  the caller's FP64 state (x, v, a, rho, id) in
//                  component-major SoA; it is physically reordered by cell
//                  every K steps, so between reorders it stays nearly sorted;
//   sorted order   per-step sweep records built right after the sort, one
//                  aligned 64-byte (FP64) or 32-byte (mixed) record per
//                  particle holding position (FP64, or 32-bit fixed-point
//                  offset from the centre of the particle's cell), velocity,
//                  and the (rho, P) pair written by the density sweep.
// Work is split into chunks of at most one block of consecutive particles of
// one instance, so every block knows its instance and reductions never mix
// instances.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphx {

constexpr int kMaxBlock = 256;
constexpr int kReduceRows = 1024;     // chunk rows per block of the first reduction level
constexpr int kNPart = 16;            // per-chunk partial sums (see k_final_reduce)

struct __align__(16) dvec2 { double x, y; };
struct __align__(32) dvec4 { double x, y, z, w; };
struct __align__(8) fvec2 { float x, y; };
struct __align__(16) fvec4 { float x, y, z, w; };

struct Chunk {
    int inst;                          // instance of the chunk
    int begin;                         // first particle (global index)
    int end;                           // one past the last
    int id;                            // chunk number in particle order (partials slot)
};

// Workgroups are dispatched to the XCDs round robin (block b runs on XCD
// b % kXcds).  Chunk maps are laid out so that the blocks of one XCD take
// consecutive chunks: each XCD then sweeps one contiguous slab of cells and
// the stencil data shared by neighbouring chunks stays in that XCD's L2.
constexpr int kXcds = 8;

struct InstDev {
    double lo[3];                      // grid origin
    int ncell[3];                      // cells per axis (1 on unused axes)
    int cell_base;                     // first global cell of the instance
    int fluid_off, n_fluid;
    int wall_off, n_wall;
    int chunk_begin, chunk_end;        // fluid chunks of the instance
    int sub_begin, sub_end;            // its rows of the first reduction level
    double c0;
};

struct SimConst {
    int dim, n_inst, N, Nw, C;
    int scheme;                        // 0 WCSPH step, 1 dual-criteria Riemann scheme
    double h, inv_h, cs, inv_cs, cut2;  // cell size 2h + skin; cut2 = (2h)^2, the pair cutoff
    double rho0, mass, sigma0, alpha, eps_h2, cfl_ac, cfl_f;
    double kW, kF, W0;                 // W = kW t^4 (2q+1), F = kF t^3, t = 1 - q/2
    double g[3];
    double cfl_adv, cfl_sub, eta;      // dual scheme: advection and acoustic Courant numbers, limiter
    int nsub_bound;                    // dual scheme: most acoustic sub-steps a plan can ask for
    double bcut2;                      // (2h + skin)^2: radius of the cell stencil and the list build
    double skin;                       // Verlet skin (0: cells and lists rebuilt every step)
    int reorder_every;                 // with a skin: reorder at a rebuild this many steps after the last
    int key_order;                     // 0 row-major cells, 1 8^d tiles with Morton order inside
    int64_t wrec_off;                  // bytes from the fluid sweep records to the wall records
                                       // padded to the same size (list walks; < 2^32 with lists)
    float fh, finv_h, fcs, fcut2, fkW, fkF, feps_h2, fbcut2;
    float fg[3], pad2;
    // Mixed path: lengths in units of the cell size cs.  A sweep record holds
    // the position as 32-bit fixed-point offsets from the centre of the
    // particle's cell, q = round((x - centre) 2^31 / cs), so that a pair
    // vector is an exact integer difference (kQUnit below).
    float ucut2, ubcut2, uinv_h, ueps_h2;   // (2h/cs)^2, ((2h + skin)/cs)^2 = 1, cs/h, eps h^2/cs^2
    float ug[3], uvisc_scale;                // g cs; alpha h / cs (times c0 per instance)
    double qcut2, qbcut2, qinv_h;            // the same in fixed-point units (2^-31 cs) for the
                                             // exact pair tests: (2h/cs)^2 2^62, 2^62, 2^-31 cs/h
};

// Fixed-point unit of the mixed path's positions: 2^-31 of a cell.
constexpr float kQUnit = 0x1p-31f;
constexpr double kQScale = 0x1p31;

// Record types per (dimension, precision): v4 halves of a fluid sweep record,
// v2 for (rho, P), wpos_t for a wall record.
template <int DIM, bool MIXED> struct Rec;
template <> struct Rec<2, false> { using v4 = dvec4; using v2 = dvec2; using wpos_t = dvec2; using real = double; };
template <> struct Rec<3, false> { using v4 = dvec4; using v2 = dvec2; using wpos_t = dvec4; using real = double; };
template <> struct Rec<2, true>  { using v4 = fvec4; using v2 = fvec2; using wpos_t = fvec4; using real = float; };
template <> struct Rec<3, true>  { using v4 = fvec4; using v2 = fvec2; using wpos_t = fvec4; using real = float; };

// ---- cell keys ----------------------------------------------------------------
//
// Local key of cell (cx, cy, cz) of an instance.  key_order 0: row-major,
// x fastest.  key_order 1: the grid is cut into tiles of 8^d cells, taken in
// row-major order, and the cells of a tile follow the Morton (Z) curve (bits of
// x, y, z interleaved), so that particles close in space are close in the
// sorted order in every direction.  Tiles past the grid's edge are padded:
// their cells stay empty.

__host__ __device__ __forceinline__ int spread_bits(int v, int dim)      // 3 bits -> every dim-th bit
{
    return dim == 3 ? ((v & 1) | ((v & 2) << 2) | ((v & 4) << 4))
                    : ((v & 1) | ((v & 2) << 1) | ((v & 4) << 2));
}

__host__ __device__ __forceinline__ int gather_bits(int m, int dim)      // inverse of spread_bits
{
    return dim == 3 ? ((m & 1) | ((m >> 2) & 2) | ((m >> 4) & 4))
                    : ((m & 1) | ((m >> 1) & 2) | ((m >> 2) & 4));
}

__host__ __device__ __forceinline__ int cell_key(const SimConst &sc, const InstDev &I, int cx, int cy, int cz)
{
    if (sc.key_order == 0) return cx + I.ncell[0] * (cy + I.ncell[1] * cz);
    const int ntx = (I.ncell[0] + 7) >> 3, nty = (I.ncell[1] + 7) >> 3;
    const int tile = (cx >> 3) + ntx * ((cy >> 3) + nty * (cz >> 3));
    const int m = spread_bits(cx & 7, sc.dim) | (spread_bits(cy & 7, sc.dim) << 1) |
                  (sc.dim == 3 ? spread_bits(cz & 7, 3) << 2 : 0);
    return (tile << (3 * sc.dim)) | m;
}

__host__ __device__ __forceinline__ void cell_coords(const SimConst &sc, const InstDev &I, int lk, int &cx, int &cy,
                                            int &cz)
{
    if (sc.key_order == 0) {
        cx = lk % I.ncell[0];
        const int t = lk / I.ncell[0];
        cy = t % I.ncell[1];
        cz = t / I.ncell[1];
        return;
    }
    const int ntx = (I.ncell[0] + 7) >> 3, nty = (I.ncell[1] + 7) >> 3;
    const int sh = 3 * sc.dim;
    const int tile = lk >> sh, m = lk & ((1 << sh) - 1);
    const int tx = tile % ntx, t2 = tile / ntx;
    cx = (tx << 3) | gather_bits(m, sc.dim);
    cy = ((t2 % nty) << 3) | gather_bits(m >> 1, sc.dim);
    cz = sc.dim == 3 ? (((t2 / nty) << 3) | gather_bits(m >> 2, 3)) : 0;
}

// ---- wave64 primitives ------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane (v_mbcnt).
__device__ __forceinline__ int mbcnt(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive block scan of one int per thread (blockDim.x <= 1024, multiple of
// 64).  `lds` must hold blockDim.x/64 + 1 ints.  Returns the prefix; *total is
// the block sum.  Contains barriers: every thread of the block must call it.
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int *total)
{
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int t = (lane < nw) ? lds[lane] : 0;
        int ti = wave_inclusive_scan(t);
        if (lane < nw) lds[lane] = ti - t;
        if (lane == nw - 1) lds[nw] = ti;
    }
    __syncthreads();
    int res = inc - v + lds[wid];
    *total = lds[nw];
    __syncthreads();
    return res;
}

// Deterministic sum over a wave (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace sphx
