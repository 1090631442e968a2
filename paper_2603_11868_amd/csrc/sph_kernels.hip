// Physics kernels of libsph: keys, reorder, sweep records, the density and
// force sweeps (direct search over the 3^d nearest cells, Sec. 5 of the
// paper), half-step integration and the FP64 reductions.
//
// Every per-particle kernel runs over a chunk map: block b handles particles
// [map[b].begin, map[b].end) of instance map[b].inst, consecutive in storage
// order (streaming kernels) or in sorted order (sweeps).  Sorted order keeps
// the instances in the same ranges as storage order because the global cell
// key is the instance's cell base plus its local key.
#include "sph_launch.h"

namespace sphx {

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int *p, int64_t n, int val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_fill_f64(double *p, int64_t n, double val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

static int fill_grid(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_i32(int *p, int64_t n, int val, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<fill_grid(n), 256, 0, s>>>(p, n, val);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double val, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_f64<<<fill_grid(n), 256, 0, s>>>(p, n, val);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------

// floor((x - lo) * inv_cs) clamped to [0, n); subtract then multiply, no FMA.
__device__ __forceinline__ int cell_1d(double x, double lo, double inv_cs, int n, int &clamped)
{
#pragma clang fp contract(off)
    const double t = floor((x - lo) * inv_cs);
    if (!(t >= 0.0)) { clamped = 1; return 0; }
    if (t >= (double)n) { clamped = 1; return n - 1; }
    return (int)t;
}

// Half-step kick and drift, rounded like the plain expressions (no FMA).
__device__ __forceinline__ void kick_drift(double &x, double &v, double a, double dt)
{
#pragma clang fp contract(off)
    v = v + 0.5 * dt * a;
    x = x + dt * v;
}

__device__ __forceinline__ double kick(double v, double a, double dt)
{
#pragma clang fp contract(off)
    return v + 0.5 * dt * a;
}

// cnt[key] += 1 for every valid lane, one atomic per distinct key of the wave.
__device__ __forceinline__ void aggregated_count(int *cnt, int key, bool valid)
{
    uint64_t rem = __ballot(valid);
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int lk = __shfl(key, leader, 64);
        const uint64_t m = __ballot(valid && key == lk);
        if (lane_id() == leader) atomicAdd(&cnt[lk], (int)__popcll(m));
        rem &= ~m;
    }
}

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_keys(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    double *__restrict__ x, double *__restrict__ v, const double *__restrict__ a,
    const double *__restrict__ dt, int kick_on, int n, int *__restrict__ key,
    int *__restrict__ cnt, int *__restrict__ clampc, unsigned *__restrict__ flags)
{
    const Chunk ch = map[blockIdx.x];
    const int i = ch.begin + threadIdx.x;
    const bool act = i < ch.end;
    int k = 0;
    int clamped = 0;
    if (act) {
        const InstDev &I = inst[ch.inst];
        double xi[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) xi[c] = x[(int64_t)c * n + i];
        if (kick_on) {
            const double dtb = dt[ch.inst];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                double vc = v[(int64_t)c * n + i];
                kick_drift(xi[c], vc, a[(int64_t)c * n + i], dtb);
                v[(int64_t)c * n + i] = vc;
                x[(int64_t)c * n + i] = xi[c];
            }
        }
        int cc[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < DIM; ++c) cc[c] = cell_1d(xi[c], I.lo[c], sc.inv_cs, I.ncell[c], clamped);
        k = I.cell_base + cc[0] + I.ncell[0] * (cc[1] + I.ncell[1] * cc[2]);
        key[i] = k;
    }
    aggregated_count(cnt, k, act);
    const uint64_t cm = __ballot(act && clamped);
    if (cm && lane_id() == 0) {
        atomicAdd(&clampc[ch.inst], (int)__popcll(cm));
        atomicOr(flags, 1u);
    }
}

hipError_t launch_keys(const SimConst &sc, const Dev &d, int kick_on, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2)
        k_keys<2><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.x, d.v, d.a, d.dt, kick_on,
                                                  sc.N, d.key, d.cnt, d.clampc, d.flags);
    else
        k_keys<3><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.x, d.v, d.a, d.dt, kick_on,
                                                  sc.N, d.key, d.cnt, d.clampc, d.flags);
    return hipGetLastError();
}

hipError_t launch_wall_keys(const SimConst &sc, const Dev &d, hipStream_t s)
{
    if (d.nwchunks <= 0) return hipSuccess;
    // walls are read only: kick is off, so x and v are never written
    double *xw = const_cast<double *>(d.xw);
    if (sc.dim == 2)
        k_keys<2><<<d.nwchunks, d.block, 0, s>>>(sc, d.wmap, d.inst, xw, nullptr, nullptr, d.dt, 0,
                                                  sc.Nw, d.wkey, d.cnt, d.clampc, d.flags);
    else
        k_keys<3><<<d.nwchunks, d.block, 0, s>>>(sc, d.wmap, d.inst, xw, nullptr, nullptr, d.dt, 0,
                                                  sc.Nw, d.wkey, d.cnt, d.clampc, d.flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reorder and sweep records
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_reorder_gather(
    const Chunk *__restrict__ map, const int *__restrict__ perm, const double *__restrict__ x,
    const double *__restrict__ v, const double *__restrict__ rho, const int *__restrict__ id,
    double *__restrict__ scr, int n)
{
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const int i = perm[k];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        scr[(int64_t)c * n + k] = x[(int64_t)c * n + i];
        scr[(int64_t)(DIM + c) * n + k] = v[(int64_t)c * n + i];
    }
    scr[(int64_t)(2 * DIM) * n + k] = rho[i];
    reinterpret_cast<int *>(scr + (int64_t)(2 * DIM + 1) * n)[k] = id[i];
}

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_reorder_copy(
    const Chunk *__restrict__ map, const double *__restrict__ scr, const int *__restrict__ skey,
    double *__restrict__ x, double *__restrict__ v, double *__restrict__ rho,
    int *__restrict__ id, int *__restrict__ perm, int *__restrict__ key, int n)
{
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        x[(int64_t)c * n + k] = scr[(int64_t)c * n + k];
        v[(int64_t)c * n + k] = scr[(int64_t)(DIM + c) * n + k];
    }
    rho[k] = scr[(int64_t)(2 * DIM) * n + k];
    id[k] = reinterpret_cast<const int *>(scr + (int64_t)(2 * DIM + 1) * n)[k];
    perm[k] = k;
    key[k] = skey[k];
}

hipError_t launch_reorder(const SimConst &sc, const Dev &d, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) {
        k_reorder_gather<2><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.perm, d.x, d.v, d.rho, d.id, d.scratch, sc.N);
        k_reorder_copy<2><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.scratch, d.skey, d.x, d.v, d.rho, d.id, d.perm, d.key, sc.N);
    } else {
        k_reorder_gather<3><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.perm, d.x, d.v, d.rho, d.id, d.scratch, sc.N);
        k_reorder_copy<3><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.scratch, d.skey, d.x, d.v, d.rho, d.id, d.perm, d.key, sc.N);
    }
    return hipGetLastError();
}

template <int DIM, bool MIXED>
__device__ __forceinline__ typename Rec<DIM, MIXED>::pos_t make_pos(const double *xi, const InstDev &I,
                                                                    int local_key, double cs)
{
    typename Rec<DIM, MIXED>::pos_t p;
    if constexpr (MIXED) {
        const int cx = local_key % I.ncell[0];
        const int t = local_key / I.ncell[0];
        const int cy = t % I.ncell[1];
        const int cz = t / I.ncell[1];
        p.x = (float)(xi[0] - (I.lo[0] + cx * cs));
        p.y = (float)(xi[1] - (I.lo[1] + cy * cs));
        if constexpr (DIM == 3) {
            p.z = (float)(xi[2] - (I.lo[2] + cz * cs));
            p.w = 0.0f;
        }
        (void)cz;
    } else {
        p.x = xi[0];
        p.y = xi[1];
        if constexpr (DIM == 3) {
            p.z = xi[2];
            p.w = 0.0;
        }
    }
    return p;
}

template <int DIM, bool MIXED>
__global__ __launch_bounds__(kMaxBlock) void k_pack(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const double *__restrict__ x, const double *__restrict__ v, const int *__restrict__ perm,
    const int *__restrict__ skey, int n, typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    typename Rec<DIM, MIXED>::vel_t *__restrict__ vel)
{
    using R = Rec<DIM, MIXED>;
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const InstDev &I = inst[ch.inst];
    const int i = perm[k];
    double xi[DIM];
    typename R::vel_t vv;
#pragma unroll
    for (int c = 0; c < DIM; ++c) xi[c] = x[(int64_t)c * n + i];
    vv.x = (typename R::real)v[i];
    vv.y = (typename R::real)v[(int64_t)n + i];
    if constexpr (DIM == 3) {
        vv.z = (typename R::real)v[(int64_t)2 * n + i];
        vv.w = 0;
    }
    pos[k] = make_pos<DIM, MIXED>(xi, I, skey[k] - I.cell_base, sc.cs);
    vel[k] = vv;
}

template <int DIM, bool MIXED>
__global__ __launch_bounds__(kMaxBlock) void k_wall_pack(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const double *__restrict__ xw, const int *__restrict__ wperm, const int *__restrict__ wskey,
    int nw, typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos)
{
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const InstDev &I = inst[ch.inst];
    const int j = wperm[k];
    double xj[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) xj[c] = xw[(int64_t)c * nw + j];
    wpos[k] = make_pos<DIM, MIXED>(xj, I, wskey[k] - I.cell_base, sc.cs);
}

template <int DIM, bool MIXED>
static void pack_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_pack<DIM, MIXED><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.x, d.v, d.perm, d.skey, sc.N,
        static_cast<typename R::pos_t *>(d.pos), static_cast<typename R::vel_t *>(d.vel));
}

hipError_t launch_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) pack_dispatch<2, true>(sc, d, s); else pack_dispatch<2, false>(sc, d, s); }
    else { if (mixed) pack_dispatch<3, true>(sc, d, s); else pack_dispatch<3, false>(sc, d, s); }
    return hipGetLastError();
}

template <int DIM, bool MIXED>
static void wall_pack_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_wall_pack<DIM, MIXED><<<d.nwchunks, d.block, 0, s>>>(
        sc, d.wmap, d.inst, d.xw, d.wall_perm, d.wskey, sc.Nw,
        static_cast<typename R::pos_t *>(d.wpos));
}

hipError_t launch_wall_pack(const SimConst &sc, const Dev &d, int mixed, hipStream_t s)
{
    if (d.nwchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) wall_pack_dispatch<2, true>(sc, d, s); else wall_pack_dispatch<2, false>(sc, d, s); }
    else { if (mixed) wall_pack_dispatch<3, true>(sc, d, s); else wall_pack_dispatch<3, false>(sc, d, s); }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// neighbour traversal
// ---------------------------------------------------------------------------

// r^2 summed left to right without FMA: the predicate r^2 < (2h)^2 of the FP64
// path then matches a plain IEEE evaluation bit for bit.
__device__ __forceinline__ double dist2(double rx, double ry)
{
#pragma clang fp contract(off)
    return rx * rx + ry * ry;
}
__device__ __forceinline__ double dist2(double rx, double ry, double rz)
{
#pragma clang fp contract(off)
    return rx * rx + ry * ry + rz * rz;
}
__device__ __forceinline__ float dist2(float rx, float ry) { return rx * rx + ry * ry; }
__device__ __forceinline__ float dist2(float rx, float ry, float rz) { return rx * rx + ry * ry + rz * rz; }

// Offsets of a target inside its own cell, per axis (in [0, cs) up to rounding).
template <int DIM, bool MIXED>
__device__ __forceinline__ void cell_offsets(const SimConst &sc, const InstDev &I, int cx, int cy, int cz,
                                             const typename Rec<DIM, MIXED>::pos_t &pi,
                                             typename Rec<DIM, MIXED>::real *o)
{
    if constexpr (MIXED) {
        o[0] = pi.x;
        o[1] = pi.y;
        if constexpr (DIM == 3) o[2] = pi.z;
        else o[2] = 0.0f;
    } else {
        o[0] = pi.x - (I.lo[0] + cx * sc.cs);
        o[1] = pi.y - (I.lo[1] + cy * sc.cs);
        if constexpr (DIM == 3) o[2] = pi.z - (I.lo[2] + cz * sc.cs);
        else o[2] = 0.0;
    }
}

// Stencil row (dy, dz) of a target with in-cell offsets o: false when every
// point of the row is at least 2h away, else the x range of cells that can
// hold a neighbour.  cut2m is (2h)^2 enlarged by a margin far above the
// rounding of o, so a skipped cell never holds a particle that passes the
// r^2 < (2h)^2 predicate: the neighbour set is unchanged.
template <class real>
__device__ __forceinline__ bool row_cells(const real *o, real cs, real cut2m, int dy, int dz, int cx,
                                          int ncx, int &xlo, int &xhi)
{
    real d2 = 0;
    if (dy < 0) d2 += o[1] * o[1];
    else if (dy > 0) { const real t = cs - o[1]; d2 += t * t; }
    if (dz < 0) d2 += o[2] * o[2];
    else if (dz > 0) { const real t = cs - o[2]; d2 += t * t; }
    if (d2 >= cut2m) return false;
    xlo = (cx > 0 && o[0] * o[0] + d2 < cut2m) ? cx - 1 : cx;
    const real t = cs - o[0];
    xhi = (cx < ncx - 1 && t * t + d2 < cut2m) ? cx + 1 : cx;
    return true;
}

// Calls fn(wall, s, r[], r2) for every neighbour of sorted target k (fluid
// slots of a stencil row first, then its wall slots; rows in z, y order).
// In the mixed path the pair vector is rebuilt from the FP32 offsets and the
// exact cell distance: r = (o_i - o_j) - (c_j - c_i) cs.
template <int DIM, bool MIXED, class Fn>
__device__ __forceinline__ void for_neighbours(const SimConst &sc, const InstDev &I, int lk, int k,
                                               const typename Rec<DIM, MIXED>::pos_t &pi,
                                               const int *__restrict__ cstart,
                                               const int *__restrict__ wstart,
                                               const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
                                               const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
                                               Fn &&fn)
{
    using real = typename Rec<DIM, MIXED>::real;
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    const int cx = lk % ncx;
    const int tq = lk / ncx;
    const int cy = tq % ncy;
    const int cz = tq / ncy;
    const int dz_lo = (DIM == 3 && cz > 0) ? -1 : 0;
    const int dz_hi = (DIM == 3 && cz < ncz - 1) ? 1 : 0;
    const real cs = MIXED ? (real)sc.fcs : (real)sc.cs;
    const real cut2m = MIXED ? (real)sc.fcut2 * (real)(1.0 + 1e-5) : (real)(sc.cut2 * (1.0 + 1e-9));
    real o[3];
    cell_offsets<DIM, MIXED>(sc, I, cx, cy, cz, pi, o);
    for (int dz = dz_lo; dz <= dz_hi; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = cy + dy;
            if (yy < 0 || yy >= ncy) continue;
            int xlo, xhi;
            if (!row_cells(o, cs, cut2m, dy, dz, cx, ncx, xlo, xhi)) continue;
            const int row = I.cell_base + (yy + ncy * (cz + dz)) * ncx;
            real ty = 0, tz = 0;
            if constexpr (MIXED) {
                ty = pi.y - (real)dy * cs;
                if constexpr (DIM == 3) tz = pi.z - (real)dz * cs;
            }
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int *__restrict__ st = pass == 0 ? cstart : wstart;
                const typename Rec<DIM, MIXED>::pos_t *__restrict__ src = pass == 0 ? pos : wpos;
                const int s0 = st[row + xlo];
                const int s1 = st[row + xhi + 1];
                int b1 = s1, b2 = s1;
                if constexpr (MIXED) {
                    if (xlo + 1 <= xhi) b1 = st[row + xlo + 1];
                    if (xlo + 2 <= xhi) b2 = st[row + xlo + 2];
                }
                for (int s = s0; s < s1; ++s) {
                    if (pass == 0 && s == k) continue;
                    const auto pj = src[s];
                    real r[3];
                    if constexpr (MIXED) {
                        const int ox = xlo - cx + (s >= b1) + (s >= b2);
                        r[0] = (pi.x - (real)ox * cs) - pj.x;
                        r[1] = ty - pj.y;
                        if constexpr (DIM == 3) r[2] = tz - pj.z;
                    } else {
                        r[0] = pi.x - pj.x;
                        r[1] = pi.y - pj.y;
                        if constexpr (DIM == 3) r[2] = pi.z - pj.z;
                    }
                    real r2;
                    if constexpr (DIM == 3) r2 = dist2(r[0], r[1], r[2]);
                    else r2 = dist2(r[0], r[1]);
                    if (r2 < (MIXED ? (real)sc.fcut2 : (real)sc.cut2)) fn(pass == 1, s, r, r2);
                }
            }
        }
    }
}

template <class real>
__device__ __forceinline__ void kernel_WF(real r2, real inv_h, real kW, real kF, real &W, real &F)
{
    const real rr = sqrt(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    const real t3 = t * t * t;
    W = kW * t3 * t * ((real)2 * q + (real)1);
    F = kF * t3;
}

template <class real>
__device__ __forceinline__ void kernel_F(real r2, real inv_h, real kF, real &F)
{
    const real rr = sqrt(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    F = kF * t * t * t;
}

__device__ __forceinline__ int wave_max_int(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Queue entries: source slot (26 bits), stencil cell code (5 bits), wall flag.
constexpr int kQueueSlotBits = 26;
constexpr unsigned kQueueSlotMask = (1u << kQueueSlotBits) - 1u;

// Neighbour traversal with per-lane compaction.  Phase 1 tests candidates in
// wave-uniform loops (lanes past the end of their own range are predicated
// off) and appends every hit to the lane's queue in LDS; whenever a lane's
// queue is full, and once at the end, the wave drains all queues together,
// so the pair arithmetic runs on dense work instead of on every candidate
// where any lane of the wave has a hit.  Hits are drained in the order they
// were found, so the sums run in the same order as the direct traversal.
template <int DIM, bool MIXED, int Q, class Fn>
__device__ __forceinline__ void for_neighbours_queued(
    const SimConst &sc, const InstDev &I, bool act, int lk, int k,
    const typename Rec<DIM, MIXED>::pos_t &pi, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos, unsigned (*__restrict__ q)[kMaxBlock],
    Fn &&fn)
{
    using real = typename Rec<DIM, MIXED>::real;
    const int tid = threadIdx.x;
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    int cx = 0, cy = 0, cz = 0;
    if (act) {
        cx = lk % ncx;
        const int tq = lk / ncx;
        cy = tq % ncy;
        cz = tq / ncy;
    }
    const real cs = MIXED ? (real)sc.fcs : (real)sc.cs;
    const real cut2 = MIXED ? (real)sc.fcut2 : (real)sc.cut2;
    const real cut2m = MIXED ? (real)sc.fcut2 * (real)(1.0 + 1e-5) : (real)(sc.cut2 * (1.0 + 1e-9));
    real o[3] = {0, 0, 0};
    if (act) cell_offsets<DIM, MIXED>(sc, I, cx, cy, cz, pi, o);
    int len = 0;

    auto pair_vector = [&](const typename Rec<DIM, MIXED>::pos_t &pj, int code, real *r) __attribute__((always_inline)) {
        if constexpr (MIXED) {
            const int ox = code % 3 - 1, oy = (code / 3) % 3 - 1, oz = code / 9 - 1;
            r[0] = (pi.x - (real)ox * cs) - pj.x;
            r[1] = (pi.y - (real)oy * cs) - pj.y;
            if constexpr (DIM == 3) r[2] = (pi.z - (real)oz * cs) - pj.z;
        } else {
            (void)code;
            r[0] = pi.x - pj.x;
            r[1] = pi.y - pj.y;
            if constexpr (DIM == 3) r[2] = pi.z - pj.z;
        }
    };
    auto drain = [&]() __attribute__((always_inline)) {
        const int m = wave_max_int(len);
        for (int t = 0; t < m; ++t) {
            if (t < len) {
                const unsigned e = q[t][tid];
                const bool wall = (e >> 31) != 0u;
                const int s = (int)(e & kQueueSlotMask);
                const int code = (int)((e >> kQueueSlotBits) & 31u);
                const auto pj = wall ? wpos[s] : pos[s];
                real r[3];
                pair_vector(pj, code, r);
                real r2;
                if constexpr (DIM == 3) r2 = dist2(r[0], r[1], r[2]);
                else r2 = dist2(r[0], r[1]);
                fn(wall, s, r, r2);
            }
        }
        len = 0;
    };

    const int dz_first = DIM == 3 ? -1 : 0, dz_last = DIM == 3 ? 1 : 0;
    for (int dz = dz_first; dz <= dz_last; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = cy + dy, zz = cz + dz;
            int xlo = cx, xhi = cx;
            const bool row_ok = act && yy >= 0 && yy < ncy && zz >= 0 && zz < ncz &&
                                row_cells(o, cs, cut2m, dy, dz, cx, ncx, xlo, xhi);
            const int row = I.cell_base + (yy + ncy * zz) * ncx;
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int *__restrict__ st = pass == 0 ? cstart : wstart;
                const typename Rec<DIM, MIXED>::pos_t *__restrict__ src = pass == 0 ? pos : wpos;
                int s0 = 0, s1 = 0, b1 = 0, b2 = 0;
                if (row_ok) {
                    s0 = st[row + xlo];
                    s1 = st[row + xhi + 1];
                    b1 = xlo + 1 <= xhi ? st[row + xlo + 1] : s1;
                    b2 = xlo + 2 <= xhi ? st[row + xlo + 2] : s1;
                }
                const int n = s1 - s0;
                const int nmax = wave_max_int(n);
                const unsigned wall_bit = pass == 1 ? 0x80000000u : 0u;
                const int code_base = ((dz + 1) * 3 + (dy + 1)) * 3 + (xlo - cx + 1);
                for (int t = 0; t < nmax; ++t) {
                    const int s = s0 + t;
                    if (t < n && !(pass == 0 && s == k)) {
                        const auto pj = src[s];
                        const int xi = (s >= b1) + (s >= b2);      // cell within the row
                        const int code = code_base + xi;
                        real r[3];
                        pair_vector(pj, code, r);
                        real r2;
                        if constexpr (DIM == 3) r2 = dist2(r[0], r[1], r[2]);
                        else r2 = dist2(r[0], r[1]);
                        if (r2 < cut2) {
                            q[len][tid] = wall_bit | ((unsigned)code << kQueueSlotBits) | (unsigned)s;
                            ++len;
                        }
                    }
                    if (__ballot(len == Q)) drain();
                }
            }
        }
    }
    drain();
}

// Traversal dispatch: Q == 0 is the plain direct search, Q > 0 the queued one.
template <int DIM, bool MIXED, int Q, class Fn>
__device__ __forceinline__ void traverse(const SimConst &sc, const InstDev &I, bool act, int lk, int k,
                                         const typename Rec<DIM, MIXED>::pos_t &pi,
                                         const int *__restrict__ cstart, const int *__restrict__ wstart,
                                         const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
                                         const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
                                         unsigned (*__restrict__ q)[kMaxBlock], Fn &&fn)
{
    if constexpr (Q == 0) {
        (void)q;
        if (act) for_neighbours<DIM, MIXED>(sc, I, lk, k, pi, cstart, wstart, pos, wpos, fn);
    } else {
        for_neighbours_queued<DIM, MIXED, Q>(sc, I, act, lk, k, pi, cstart, wstart, pos, wpos, q, fn);
    }
}

// ---------------------------------------------------------------------------
// density sweep
// ---------------------------------------------------------------------------

template <int DIM, bool MIXED, int Q>
__global__ __launch_bounds__(kMaxBlock) void k_density(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    const typename Rec<DIM, MIXED>::vel_t *__restrict__ vel,
    const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos, double *__restrict__ rho,
    int *__restrict__ count, typename Rec<DIM, MIXED>::rp_t *__restrict__ rp,
    const double *__restrict__ dt, int use_dt)
{
    using R = Rec<DIM, MIXED>;
    using real = typename R::real;
    __shared__ unsigned q[Q > 0 ? Q : 1][kMaxBlock];
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    if (Q == 0 && !act) return;
    const InstDev &I = inst[ch.inst];
    const int kk = act ? k : ch.begin;
    const int lk = skey[kk] - I.cell_base;
    const typename R::pos_t pi = pos[kk];
    const typename R::vel_t vi = vel[kk];
    const real inv_h = MIXED ? (real)sc.finv_h : (real)sc.inv_h;
    const real kW = MIXED ? (real)sc.fkW : (real)sc.kW;
    const real kF = MIXED ? (real)sc.fkF : (real)sc.kF;
    real sigma = MIXED ? (real)0 : (real)sc.W0;
    real drho = 0;
    int cnt = 0;
    traverse<DIM, MIXED, Q>(sc, I, act, lk, k, pi, cstart, wstart, pos, wpos, q,
        [&](bool wall, int s, const real *r, real r2) __attribute__((always_inline)) {
            real W, F;
            kernel_WF(r2, inv_h, kW, kF, W, F);
            real vr;
            if (wall) {
                vr = vi.x * r[0] + vi.y * r[1];
                if constexpr (DIM == 3) vr += vi.z * r[2];
            } else {
                const typename R::vel_t vj = vel[s];
                vr = (vi.x - vj.x) * r[0] + (vi.y - vj.y) * r[1];
                if constexpr (DIM == 3) vr += (vi.z - vj.z) * r[2];
            }
            sigma += W;
            drho += vr * F;
            ++cnt;
        });
    if (!act) return;
    const int i = perm[k];
    const double sig = MIXED ? sc.W0 + (double)sigma : (double)sigma;
    const double rho_sum = sc.mass * sig;
    const double dtb = use_dt ? dt[ch.inst] : 0.0;
    const double rho_star = rho[i] + dtb * (sc.mass * (double)drho);
    const double excess = rho_star - rho_sum;
    const double rn = excess > 0.0 ? rho_sum + excess * sc.rho0 / rho_star : rho_sum;
    double p = I.c0 * I.c0 * (rn - sc.rho0);
    if (p < 0.0) p = 0.0;
    const double P = p / (rn * rn);
    rho[i] = rn;
    count[i] = cnt;
    typename R::rp_t out;
    out.x = (real)rn;
    out.y = (real)P;
    rp[k] = out;
}

template <int DIM, bool MIXED, int Q>
static void density_dispatch(const SimConst &sc, const Dev &d, int use_dt, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_density<DIM, MIXED, Q><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start,
        static_cast<const typename R::pos_t *>(d.pos), static_cast<const typename R::vel_t *>(d.vel),
        static_cast<const typename R::pos_t *>(d.wpos), d.rho, d.count,
        static_cast<typename R::rp_t *>(d.rp), d.dt, use_dt);
}

template <int DIM, bool MIXED>
static void density_q(const SimConst &sc, const Dev &d, int use_dt, hipStream_t s)
{
    if (d.queue_cap == 0) density_dispatch<DIM, MIXED, 0>(sc, d, use_dt, s);
    else if (d.queue_cap == 16) density_dispatch<DIM, MIXED, 16>(sc, d, use_dt, s);
    else density_dispatch<DIM, MIXED, 32>(sc, d, use_dt, s);
}

hipError_t launch_density(const SimConst &sc, const Dev &d, int mixed, int use_dt, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) density_q<2, true>(sc, d, use_dt, s); else density_q<2, false>(sc, d, use_dt, s); }
    else { if (mixed) density_q<3, true>(sc, d, use_dt, s); else density_q<3, false>(sc, d, use_dt, s); }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// block partial sums (deterministic: fixed lanes, fixed butterfly, fixed wave order)
// ---------------------------------------------------------------------------

// slots: 0 max|v| 1 max|a| 2..4 sum m v 5 kinetic 6 potential 7 internal
//        8..10 sum m a_ff 11 sum rho 12 pairs 13 non-finite count
enum { P_VMAX = 0, P_AMAX = 1, P_MOM = 2, P_KE = 5, P_PE = 6, P_IE = 7, P_FF = 8,
       P_RHO = 11, P_PAIRS = 12, P_BAD = 13 };

__device__ __forceinline__ bool is_max_slot(int s) { return s == P_VMAX || s == P_AMAX; }

// Reduce vals[lo..hi) over the block and write them to out[lo..hi).
template <int LO, int HI>
__device__ __forceinline__ void block_partials(double (&vals)[kNPart], double *__restrict__ out)
{
    __shared__ double sh[kMaxBlock / 64][kNPart];
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int s = LO; s < HI; ++s) {
        const double r = is_max_slot(s) ? wave_max(vals[s]) : wave_sum(vals[s]);
        if (lane_id() == 0) sh[w][s] = r;
    }
    __syncthreads();
    const int s = threadIdx.x + LO;
    if (s < HI) {
        double r = sh[0][s];
        for (int q = 1; q < nw; ++q) r = is_max_slot(s) ? fmax(r, sh[q][s]) : r + sh[q][s];
        out[s] = r;
    }
}

// Contributions of one particle to the step diagnostics (FP64).
template <int DIM>
__device__ __forceinline__ void state_partials(const SimConst &sc, const InstDev &I, const double *vn,
                                               const double *an, const double *xi, double rhoi,
                                               double (&vals)[kNPart])
{
    double v2 = 0, a2 = 0, gx = 0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        v2 += vn[c] * vn[c];
        a2 += an[c] * an[c];
        gx += sc.g[c] * xi[c];
        vals[P_MOM + c] = sc.mass * vn[c];
    }
    const double vm = sqrt(v2), am = sqrt(a2);
    vals[P_VMAX] = vm;
    vals[P_AMAX] = am;
    vals[P_KE] = 0.5 * sc.mass * v2;
    vals[P_PE] = -sc.mass * gx;
    vals[P_IE] = rhoi > sc.rho0
                     ? sc.mass * I.c0 * I.c0 * (log(rhoi / sc.rho0) + sc.rho0 / rhoi - 1.0)
                     : 0.0;
    vals[P_RHO] = rhoi;
    vals[P_BAD] = (isfinite(vm) && isfinite(am)) ? 0.0 : 1.0;
}

// ---------------------------------------------------------------------------
// force sweep (+ half 2 and partials when fused)
// ---------------------------------------------------------------------------

template <int DIM, bool MIXED, bool FUSED, int Q>
__global__ __launch_bounds__(kMaxBlock) void k_force(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    const typename Rec<DIM, MIXED>::vel_t *__restrict__ vel,
    const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
    const typename Rec<DIM, MIXED>::rp_t *__restrict__ rp, double *__restrict__ a,
    double *__restrict__ v, const double *__restrict__ x, const double *__restrict__ rho,
    const double *__restrict__ dt, double *__restrict__ partials, int n)
{
    using R = Rec<DIM, MIXED>;
    using real = typename R::real;
    __shared__ unsigned q[Q > 0 ? Q : 1][kMaxBlock];
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    const InstDev &I = inst[ch.inst];
    const int kk = act ? k : ch.begin;
    const int lk = skey[kk] - I.cell_base;
    const typename R::pos_t pi = pos[kk];
    const typename R::vel_t vi = vel[kk];
    const typename R::rp_t rpi = rp[kk];
    const real rho_i = rpi.x, P_i = rpi.y;
    const real p_i = P_i * rho_i * rho_i;
    const real inv_rho_i2 = (real)1 / (rho_i * rho_i);
    const real inv_h = MIXED ? (real)sc.finv_h : (real)sc.inv_h;
    const real kF = MIXED ? (real)sc.fkF : (real)sc.kF;
    const real visc_a = (real)(sc.alpha * I.c0 * sc.h);
    const real eps_h2 = MIXED ? (real)sc.feps_h2 : (real)sc.eps_h2;
    const real gx = MIXED ? (real)sc.fg[0] : (real)sc.g[0];
    const real gy = MIXED ? (real)sc.fg[1] : (real)sc.g[1];
    const real gz = MIXED ? (real)sc.fg[2] : (real)sc.g[2];
    real acc[3] = {0, 0, 0}, aff[3] = {0, 0, 0};
    int cnt = 0;
    traverse<DIM, MIXED, Q>(sc, I, act, lk, k, pi, cstart, wstart, pos, wpos, q,
        [&](bool wall, int s, const real *r, real r2) __attribute__((always_inline)) {
            real F;
            kernel_F(r2, inv_h, kF, F);
            real P_j, rho_j, vr;
            if (wall) {
                real gr = gx * r[0] + gy * r[1];
                if constexpr (DIM == 3) gr += gz * r[2];
                real p_j = p_i - rho_i * gr;       // p_i + rho_i g.(x_j - x_i)
                if (p_j < (real)0) p_j = (real)0;
                P_j = p_j * inv_rho_i2;
                rho_j = rho_i;
                vr = vi.x * r[0] + vi.y * r[1];
                if constexpr (DIM == 3) vr += vi.z * r[2];
            } else {
                const typename R::rp_t rpj = rp[s];
                const typename R::vel_t vj = vel[s];
                rho_j = rpj.x;
                P_j = rpj.y;
                vr = (vi.x - vj.x) * r[0] + (vi.y - vj.y) * r[1];
                if constexpr (DIM == 3) vr += (vi.z - vj.z) * r[2];
            }
            real visc = 0;
            if (vr < (real)0)
                visc = -visc_a * vr / ((real)0.5 * (rho_i + rho_j) * (r2 + eps_h2));
            const real coef = (P_i + P_j + visc) * F;
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[c] -= coef * r[c];
            if (!wall) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) aff[c] -= coef * r[c];
            }
            ++cnt;
        });
    double vals[kNPart];
#pragma unroll
    for (int qq = 0; qq < kNPart; ++qq) vals[qq] = 0.0;
    if (act) {
        const int i = perm[k];
        double an[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            an[c] = sc.g[c] + sc.mass * (double)acc[c];
            a[(int64_t)c * n + i] = an[c];
            vals[P_FF + c] = sc.mass * (sc.mass * (double)aff[c]);
        }
        vals[P_PAIRS] = (double)cnt;
        if constexpr (FUSED) {
            const double dtb = dt[ch.inst];
            double vn[DIM], xi[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                vn[c] = kick(v[(int64_t)c * n + i], an[c], dtb);
                v[(int64_t)c * n + i] = vn[c];
                xi[c] = x[(int64_t)c * n + i];
            }
            state_partials<DIM>(sc, I, vn, an, xi, rho[i], vals);
        }
    }
    double *out = partials + (int64_t)ch.id * kNPart;
    if constexpr (FUSED) block_partials<0, P_BAD + 1>(vals, out);
    else block_partials<P_FF, P_PAIRS + 1>(vals, out);
}

template <int DIM, bool MIXED, bool FUSED, int Q>
static void force_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_force<DIM, MIXED, FUSED, Q><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start,
        static_cast<const typename R::pos_t *>(d.pos), static_cast<const typename R::vel_t *>(d.vel),
        static_cast<const typename R::pos_t *>(d.wpos), static_cast<const typename R::rp_t *>(d.rp),
        d.a, d.v, d.x, d.rho, d.dt, d.partials, sc.N);
}

template <int DIM, bool MIXED, bool FUSED>
static void force_q(const SimConst &sc, const Dev &d, hipStream_t s)
{
    if (d.queue_cap == 0) force_dispatch<DIM, MIXED, FUSED, 0>(sc, d, s);
    else if (d.queue_cap == 16) force_dispatch<DIM, MIXED, FUSED, 16>(sc, d, s);
    else force_dispatch<DIM, MIXED, FUSED, 32>(sc, d, s);
}

hipError_t launch_force(const SimConst &sc, const Dev &d, int mixed, int fused, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) {
        if (mixed) { if (fused) force_q<2, true, true>(sc, d, s); else force_q<2, true, false>(sc, d, s); }
        else { if (fused) force_q<2, false, true>(sc, d, s); else force_q<2, false, false>(sc, d, s); }
    } else {
        if (mixed) { if (fused) force_q<3, true, true>(sc, d, s); else force_q<3, true, false>(sc, d, s); }
        else { if (fused) force_q<3, false, true>(sc, d, s); else force_q<3, false, false>(sc, d, s); }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// neighbour-list sweeps
//
// The density sweep tests the candidates once and writes each target's hits
// (encoded like the queue entries: slot, stencil cell code, wall bit) to a
// slot-major list nlist[m * N + k]; its own pair loop and the whole force
// sweep then walk that list, so the force sweep tests no candidates at all and
// both pair loops read the list with coalesced loads.  Candidate records are
// fetched U at a time so that U loads per lane are in flight together.  A
// target with more than `cap` neighbours walks the stencil again instead
// (same order, same results) and raises SPH_FLAG_CAPACITY.
// ---------------------------------------------------------------------------

template <int DIM, bool MIXED>
struct PairGeom {
    using real = typename Rec<DIM, MIXED>::real;
    using pos_t = typename Rec<DIM, MIXED>::pos_t;
    // r = x_i - x_j from the target record and a source record of stencil cell `code`
    __device__ __forceinline__ static void vec(const pos_t &pi, const pos_t &pj, int code, real cs, real *r)
    {
        if constexpr (MIXED) {
            const int ox = code % 3 - 1, oy = (code / 3) % 3 - 1, oz = code / 9 - 1;
            r[0] = (pi.x - (real)ox * cs) - pj.x;
            r[1] = (pi.y - (real)oy * cs) - pj.y;
            if constexpr (DIM == 3) r[2] = (pi.z - (real)oz * cs) - pj.z;
            (void)oz;
        } else {
            (void)code;
            (void)cs;
            r[0] = pi.x - pj.x;
            r[1] = pi.y - pj.y;
            if constexpr (DIM == 3) r[2] = pi.z - pj.z;
        }
    }
    __device__ __forceinline__ static real r2(const real *r)
    {
        if constexpr (DIM == 3) return dist2(r[0], r[1], r[2]);
        else return dist2(r[0], r[1]);
    }
};

// Phase 1: candidate tests of target k, hits appended to its list.  Returns
// the number of hits (possibly above cap; only the first cap are stored).
template <int DIM, bool MIXED, int U>
__device__ __forceinline__ int build_list(const SimConst &sc, const InstDev &I, int lk, int k,
                                          const typename Rec<DIM, MIXED>::pos_t &pi,
                                          const int *__restrict__ cstart, const int *__restrict__ wstart,
                                          const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
                                          const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
                                          uint4 *__restrict__ nlist, int cap, int n)
{
    using G = PairGeom<DIM, MIXED>;
    using real = typename G::real;
    using pos_t = typename G::pos_t;
    const int ncx = I.ncell[0], ncy = I.ncell[1], ncz = I.ncell[2];
    const int cx = lk % ncx;
    const int tq = lk / ncx;
    const int cy = tq % ncy;
    const int cz = tq / ncy;
    const real cs = MIXED ? (real)sc.fcs : (real)sc.cs;
    const real cut2 = MIXED ? (real)sc.fcut2 : (real)sc.cut2;
    const real cut2m = MIXED ? (real)sc.fcut2 * (real)(1.0 + 1e-5) : (real)(sc.cut2 * (1.0 + 1e-9));
    real o[3];
    cell_offsets<DIM, MIXED>(sc, I, cx, cy, cz, pi, o);
    int m = 0;
    uint4 buf = make_uint4(0u, 0u, 0u, 0u);
    const int dz_lo = (DIM == 3 && cz > 0) ? -1 : 0;
    const int dz_hi = (DIM == 3 && cz < ncz - 1) ? 1 : 0;
    for (int dz = dz_lo; dz <= dz_hi; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = cy + dy;
            if (yy < 0 || yy >= ncy) continue;
            int xlo, xhi;
            if (!row_cells(o, cs, cut2m, dy, dz, cx, ncx, xlo, xhi)) continue;
            const int row = I.cell_base + (yy + ncy * (cz + dz)) * ncx;
            const int code_base = ((dz + 1) * 3 + (dy + 1)) * 3 + (xlo - cx + 1);
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                const int *__restrict__ st = pass == 0 ? cstart : wstart;
                const pos_t *__restrict__ src = pass == 0 ? pos : wpos;
                const unsigned wall_bit = pass == 1 ? 0x80000000u : 0u;
                const int s0 = st[row + xlo];
                const int s1 = st[row + xhi + 1];
                int b1 = s1, b2 = s1;
                if constexpr (MIXED) {
                    if (xlo + 1 <= xhi) b1 = st[row + xlo + 1];
                    if (xlo + 2 <= xhi) b2 = st[row + xlo + 2];
                }
                for (int t0 = s0; t0 < s1; t0 += U) {
                    pos_t pj[U];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (t0 + u < s1) pj[u] = src[t0 + u];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int s = t0 + u;
                        if (s < s1 && !(pass == 0 && s == k)) {
                            const int code = code_base + (s >= b1) + (s >= b2);
                            real r[3];
                            G::vec(pi, pj[u], code, cs, r);
                            if (G::r2(r) < cut2) {
                                if (m < cap) {
                                    const unsigned e = wall_bit | ((unsigned)code << kQueueSlotBits) | (unsigned)s;
                                    const int j = m & 3;
                                    buf.x = j == 0 ? e : buf.x;
                                    buf.y = j == 1 ? e : buf.y;
                                    buf.z = j == 2 ? e : buf.z;
                                    buf.w = j == 3 ? e : buf.w;
                                    if (j == 3) nlist[(int64_t)(m >> 2) * n + k] = buf;
                                }
                                ++m;
                            }
                        }
                    }
                }
            }
        }
    }
    if ((m & 3) != 0 && m <= cap) nlist[(int64_t)(m >> 2) * n + k] = buf;   // last partial quad
    return m;
}

// Phase 2: calls fn(wall, s, r, r2) for the first m (<= cap) list entries of
// target k.  Entries are stored as quads (uint4) slot-major: quad q of target
// k is nlist[q * N + k], so a wave reads 1 KiB contiguous per quad.  The
// records of U entries are fetched before any of them is used.
template <int DIM, bool MIXED, int U, class Fn>
__device__ __forceinline__ void walk_list(const SimConst &sc, int k, int m,
                                          const typename Rec<DIM, MIXED>::pos_t &pi,
                                          const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
                                          const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
                                          const uint4 *__restrict__ nlist, int n, Fn &&fn)
{
    static_assert(U == 2 || U == 4, "entries are fetched in quads");
    using G = PairGeom<DIM, MIXED>;
    using real = typename G::real;
    using pos_t = typename G::pos_t;
    const real cs = MIXED ? (real)sc.fcs : (real)sc.cs;
    for (int q0 = 0; q0 < m; q0 += 4) {
        const uint4 quad = nlist[(int64_t)(q0 >> 2) * n + k];
        const unsigned eq[4] = {quad.x, quad.y, quad.z, quad.w};
#pragma unroll
        for (int h = 0; h < 4; h += U) {
            pos_t pj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + h + u < m) {
                    const unsigned e = eq[h + u];
                    const pos_t *__restrict__ src = (e >> 31) ? wpos : pos;
                    pj[u] = src[e & kQueueSlotMask];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (q0 + h + u < m) {
                    const unsigned e = eq[h + u];
                    const bool wall = (e >> 31) != 0u;
                    const int s = (int)(e & kQueueSlotMask);
                    const int code = (int)((e >> kQueueSlotBits) & 31u);
                    real r[3];
                    G::vec(pi, pj[u], code, cs, r);
                    fn(wall, s, r, G::r2(r));
                }
            }
        }
    }
}

template <int DIM, bool MIXED, int U>
__global__ __launch_bounds__(kMaxBlock) void k_density_list(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    const typename Rec<DIM, MIXED>::vel_t *__restrict__ vel,
    const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos, double *__restrict__ rho,
    int *__restrict__ count, typename Rec<DIM, MIXED>::rp_t *__restrict__ rp,
    const double *__restrict__ dt, int use_dt, uint4 *__restrict__ nlist,
    int *__restrict__ lcount, int cap, int n, unsigned *__restrict__ flags)
{
    using R = Rec<DIM, MIXED>;
    using real = typename R::real;
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    if (k >= ch.end) return;
    const InstDev &I = inst[ch.inst];
    const int lk = skey[k] - I.cell_base;
    const typename R::pos_t pi = pos[k];
    const typename R::vel_t vi = vel[k];
    const real inv_h = MIXED ? (real)sc.finv_h : (real)sc.inv_h;
    const real kW = MIXED ? (real)sc.fkW : (real)sc.kW;
    const real kF = MIXED ? (real)sc.fkF : (real)sc.kF;
    real sigma = MIXED ? (real)0 : (real)sc.W0;
    real drho = 0;
    int cnt = 0;
    auto pair = [&](bool wall, int s, const real *r, real r2) __attribute__((always_inline)) {
        real W, F;
        kernel_WF(r2, inv_h, kW, kF, W, F);
        real vr;
        if (wall) {
            vr = vi.x * r[0] + vi.y * r[1];
            if constexpr (DIM == 3) vr += vi.z * r[2];
        } else {
            const typename R::vel_t vj = vel[s];
            vr = (vi.x - vj.x) * r[0] + (vi.y - vj.y) * r[1];
            if constexpr (DIM == 3) vr += (vi.z - vj.z) * r[2];
        }
        sigma += W;
        drho += vr * F;
        ++cnt;
    };
    const int m = build_list<DIM, MIXED, 4>(sc, I, lk, k, pi, cstart, wstart, pos, wpos, nlist, cap, n);
    if (m <= cap) {
        walk_list<DIM, MIXED, U>(sc, k, m, pi, pos, wpos, nlist, n, pair);
    } else {
        atomicOr(flags, 4u);
        for_neighbours<DIM, MIXED>(sc, I, lk, k, pi, cstart, wstart, pos, wpos, pair);
    }
    lcount[k] = m;
    const int i = perm[k];
    const double sig = MIXED ? sc.W0 + (double)sigma : (double)sigma;
    const double rho_sum = sc.mass * sig;
    const double dtb = use_dt ? dt[ch.inst] : 0.0;
    const double rho_star = rho[i] + dtb * (sc.mass * (double)drho);
    const double excess = rho_star - rho_sum;
    const double rn = excess > 0.0 ? rho_sum + excess * sc.rho0 / rho_star : rho_sum;
    double p = I.c0 * I.c0 * (rn - sc.rho0);
    if (p < 0.0) p = 0.0;
    const double P = p / (rn * rn);
    rho[i] = rn;
    count[i] = cnt;
    typename R::rp_t out;
    out.x = (real)rn;
    out.y = (real)P;
    rp[k] = out;
}

template <int DIM, bool MIXED, bool FUSED, int U>
__global__ __launch_bounds__(kMaxBlock) void k_force_list(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    const int *__restrict__ skey, const int *__restrict__ perm, const int *__restrict__ cstart,
    const int *__restrict__ wstart, const typename Rec<DIM, MIXED>::pos_t *__restrict__ pos,
    const typename Rec<DIM, MIXED>::vel_t *__restrict__ vel,
    const typename Rec<DIM, MIXED>::pos_t *__restrict__ wpos,
    const typename Rec<DIM, MIXED>::rp_t *__restrict__ rp, double *__restrict__ a,
    double *__restrict__ v, const double *__restrict__ x, const double *__restrict__ rho,
    const double *__restrict__ dt, double *__restrict__ partials, int n,
    const uint4 *__restrict__ nlist, const int *__restrict__ lcount, int cap)
{
    using R = Rec<DIM, MIXED>;
    using real = typename R::real;
    const Chunk ch = map[blockIdx.x];
    const int k = ch.begin + threadIdx.x;
    const bool act = k < ch.end;
    const InstDev &I = inst[ch.inst];
    const int kk = act ? k : ch.begin;
    const typename R::pos_t pi = pos[kk];
    const typename R::vel_t vi = vel[kk];
    const typename R::rp_t rpi = rp[kk];
    const real rho_i = rpi.x, P_i = rpi.y;
    const real p_i = P_i * rho_i * rho_i;
    const real inv_rho_i2 = (real)1 / (rho_i * rho_i);
    const real inv_h = MIXED ? (real)sc.finv_h : (real)sc.inv_h;
    const real kF = MIXED ? (real)sc.fkF : (real)sc.kF;
    const real visc_a = (real)(sc.alpha * I.c0 * sc.h);
    const real eps_h2 = MIXED ? (real)sc.feps_h2 : (real)sc.eps_h2;
    const real gx = MIXED ? (real)sc.fg[0] : (real)sc.g[0];
    const real gy = MIXED ? (real)sc.fg[1] : (real)sc.g[1];
    const real gz = MIXED ? (real)sc.fg[2] : (real)sc.g[2];
    real acc[3] = {0, 0, 0}, aff[3] = {0, 0, 0};
    int cnt = 0;
    auto pair = [&](bool wall, int s, const real *r, real r2) __attribute__((always_inline)) {
        real F;
        kernel_F(r2, inv_h, kF, F);
        real P_j, rho_j, vr;
        if (wall) {
            real gr = gx * r[0] + gy * r[1];
            if constexpr (DIM == 3) gr += gz * r[2];
            real p_j = p_i - rho_i * gr;       // p_i + rho_i g.(x_j - x_i)
            if (p_j < (real)0) p_j = (real)0;
            P_j = p_j * inv_rho_i2;
            rho_j = rho_i;
            vr = vi.x * r[0] + vi.y * r[1];
            if constexpr (DIM == 3) vr += vi.z * r[2];
        } else {
            const typename R::rp_t rpj = rp[s];
            const typename R::vel_t vj = vel[s];
            rho_j = rpj.x;
            P_j = rpj.y;
            vr = (vi.x - vj.x) * r[0] + (vi.y - vj.y) * r[1];
            if constexpr (DIM == 3) vr += (vi.z - vj.z) * r[2];
        }
        real visc = 0;
        if (vr < (real)0)
            visc = -visc_a * vr / ((real)0.5 * (rho_i + rho_j) * (r2 + eps_h2));
        const real coef = (P_i + P_j + visc) * F;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] -= coef * r[c];
        if (!wall) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) aff[c] -= coef * r[c];
        }
        ++cnt;
    };
    if (act) {
        const int m = lcount[k];
        if (m <= cap) {
            walk_list<DIM, MIXED, U>(sc, k, m, pi, pos, wpos, nlist, n, pair);
        } else {
            const int lk = skey[k] - I.cell_base;
            for_neighbours<DIM, MIXED>(sc, I, lk, k, pi, cstart, wstart, pos, wpos, pair);
        }
    }
    double vals[kNPart];
#pragma unroll
    for (int qq = 0; qq < kNPart; ++qq) vals[qq] = 0.0;
    if (act) {
        const int i = perm[k];
        double an[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            an[c] = sc.g[c] + sc.mass * (double)acc[c];
            a[(int64_t)c * n + i] = an[c];
            vals[P_FF + c] = sc.mass * (sc.mass * (double)aff[c]);
        }
        vals[P_PAIRS] = (double)cnt;
        if constexpr (FUSED) {
            const double dtb = dt[ch.inst];
            double vn[DIM], xi[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                vn[c] = kick(v[(int64_t)c * n + i], an[c], dtb);
                v[(int64_t)c * n + i] = vn[c];
                xi[c] = x[(int64_t)c * n + i];
            }
            state_partials<DIM>(sc, I, vn, an, xi, rho[i], vals);
        }
    }
    double *out = partials + (int64_t)ch.id * kNPart;
    if constexpr (FUSED) block_partials<0, P_BAD + 1>(vals, out);
    else block_partials<P_FF, P_PAIRS + 1>(vals, out);
}

template <int DIM, bool MIXED>
static void density_list_dispatch(const SimConst &sc, const Dev &d, int use_dt, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    k_density_list<DIM, MIXED, 4><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start,
        static_cast<const typename R::pos_t *>(d.pos), static_cast<const typename R::vel_t *>(d.vel),
        static_cast<const typename R::pos_t *>(d.wpos), d.rho, d.count,
        static_cast<typename R::rp_t *>(d.rp), d.dt, use_dt, d.nlist, d.lcount, d.list_cap, sc.N,
        d.flags);
}

hipError_t launch_density_list(const SimConst &sc, const Dev &d, int mixed, int use_dt, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) { if (mixed) density_list_dispatch<2, true>(sc, d, use_dt, s); else density_list_dispatch<2, false>(sc, d, use_dt, s); }
    else { if (mixed) density_list_dispatch<3, true>(sc, d, use_dt, s); else density_list_dispatch<3, false>(sc, d, use_dt, s); }
    return hipGetLastError();
}

template <int DIM, bool MIXED, bool FUSED>
static void force_list_dispatch(const SimConst &sc, const Dev &d, hipStream_t s)
{
    using R = Rec<DIM, MIXED>;
    constexpr int U = MIXED ? 4 : 2;
    k_force_list<DIM, MIXED, FUSED, U><<<d.nfchunks, d.block, 0, s>>>(
        sc, d.fmap, d.inst, d.skey, d.perm, d.cell_start, d.wall_start,
        static_cast<const typename R::pos_t *>(d.pos), static_cast<const typename R::vel_t *>(d.vel),
        static_cast<const typename R::pos_t *>(d.wpos), static_cast<const typename R::rp_t *>(d.rp),
        d.a, d.v, d.x, d.rho, d.dt, d.partials, sc.N, d.nlist, d.lcount, d.list_cap);
}

hipError_t launch_force_list(const SimConst &sc, const Dev &d, int mixed, int fused, hipStream_t s)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2) {
        if (mixed) { if (fused) force_list_dispatch<2, true, true>(sc, d, s); else force_list_dispatch<2, true, false>(sc, d, s); }
        else { if (fused) force_list_dispatch<2, false, true>(sc, d, s); else force_list_dispatch<2, false, false>(sc, d, s); }
    } else {
        if (mixed) { if (fused) force_list_dispatch<3, true, true>(sc, d, s); else force_list_dispatch<3, true, false>(sc, d, s); }
        else { if (fused) force_list_dispatch<3, false, true>(sc, d, s); else force_list_dispatch<3, false, false>(sc, d, s); }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// staged half 2
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_half2(
    SimConst sc, const Chunk *__restrict__ map, const InstDev *__restrict__ inst,
    double *__restrict__ v, const double *__restrict__ a, const double *__restrict__ x,
    const double *__restrict__ rho, const double *__restrict__ dt, double *__restrict__ partials,
    int n, int kick_on)
{
    const Chunk ch = map[blockIdx.x];
    const int i = ch.begin + threadIdx.x;
    double vals[kNPart];
#pragma unroll
    for (int q = 0; q < kNPart; ++q) vals[q] = 0.0;
    if (i < ch.end) {
        const InstDev &I = inst[ch.inst];
        const double dtb = kick_on ? dt[ch.inst] : 0.0;
        double vn[DIM], an[DIM], xi[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            an[c] = a[(int64_t)c * n + i];
            vn[c] = v[(int64_t)c * n + i];
            if (kick_on) {
                vn[c] = kick(vn[c], an[c], dtb);
                v[(int64_t)c * n + i] = vn[c];
            }
            xi[c] = x[(int64_t)c * n + i];
        }
        state_partials<DIM>(sc, I, vn, an, xi, rho[i], vals);
    }
    double *out = partials + (int64_t)ch.id * kNPart;
    block_partials<0, P_FF>(vals, out);
    // slots after the force sweep's share
    block_partials<P_RHO, P_RHO + 1>(vals, out);
    block_partials<P_BAD, P_BAD + 1>(vals, out);
}

hipError_t launch_half2(const SimConst &sc, const Dev &d, hipStream_t s, int kick_on)
{
    if (d.nfchunks <= 0) return hipSuccess;
    if (sc.dim == 2)
        k_half2<2><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.v, d.a, d.x, d.rho, d.dt, d.partials, sc.N, kick_on);
    else
        k_half2<3><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.v, d.a, d.x, d.rho, d.dt, d.partials, sc.N, kick_on);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-instance reductions -> dt, diag
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_final_reduce(SimConst sc, const InstDev *__restrict__ inst,
                                                      const double *__restrict__ partials,
                                                      double *__restrict__ dt,
                                                      double *__restrict__ diag,
                                                      int *__restrict__ clampc,
                                                      unsigned *__restrict__ flags, int prime)
{
    const int b = blockIdx.x;
    const InstDev &I = inst[b];
    double acc[kNPart];
#pragma unroll
    for (int q = 0; q < kNPart; ++q) acc[q] = 0.0;
    for (int c = I.chunk_begin + threadIdx.x; c < I.chunk_end; c += blockDim.x) {
        const double *p = partials + (int64_t)c * kNPart;
#pragma unroll
        for (int q = 0; q < kNPart; ++q) acc[q] = is_max_slot(q) ? fmax(acc[q], p[q]) : acc[q] + p[q];
    }
    __shared__ double tot[kNPart];
    block_partials<0, kNPart>(acc, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        double *d = diag + (int64_t)b * 16;
        const double dt_used = prime ? 0.0 : dt[b];
        const double vmax = tot[P_VMAX], amax = tot[P_AMAX];
        d[0] = vmax;
        d[1] = amax;
        d[2] = sc.mass * (double)I.n_fluid;
        for (int c = 0; c < 3; ++c) d[3 + c] = tot[P_MOM + c];
        d[6] = tot[P_KE];
        d[7] = tot[P_PE];
        d[8] = tot[P_IE];
        const double ff = sqrt(tot[P_FF] * tot[P_FF] + tot[P_FF + 1] * tot[P_FF + 1] +
                               tot[P_FF + 2] * tot[P_FF + 2]);
        d[9] = ff;
        d[10] = I.n_fluid > 0 ? tot[P_RHO] / ((double)I.n_fluid * sc.rho0) - 1.0 : 0.0;
        d[11] += (double)clampc[b];
        clampc[b] = 0;
        d[12] = tot[P_PAIRS];
        d[13] += dt_used * ff;
        d[14] += dt_used;
        d[15] = prime ? 0.0 : d[15] + 1.0;
        const double dt_ac = sc.cfl_ac * sc.h / (I.c0 + vmax);
        const double dt_f = sc.cfl_f * sqrt(sc.h / amax);
        dt[b] = dt_ac < dt_f ? dt_ac : dt_f;
        if (tot[P_BAD] > 0.0) atomicOr(flags, 2u);
    }
}

hipError_t launch_final_reduce(const SimConst &sc, const Dev &d, int prime, hipStream_t s)
{
    if (sc.n_inst <= 0) return hipSuccess;
    k_final_reduce<<<sc.n_inst, 256, 0, s>>>(sc, d.inst, d.partials, d.dt, d.diag, d.clampc, d.flags, prime);
    return hipGetLastError();
}

}  // namespace sphx
