// Streaming kernels of libsph: fills, cell keys (with the half-1 kick and
// drift), the reorder of the state by cell, the staged half 2 and the FP64
// per-instance reductions.  The pair sweeps are in sph_sweeps.hip.
//
// Every per-particle kernel runs over a chunk map: block b handles particles
// [map[b].begin, map[b].end) of instance map[b].inst, consecutive in storage
// order (streaming kernels) or in sorted order (sweeps).  Sorted order keeps
// the instances in the same ranges as storage order because the global cell
// key is the instance's cell base plus its local key.
#include "sph_step_common.h"

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
    int *__restrict__ cnt, int *__restrict__ clampc, unsigned *__restrict__ flags,
    const int *__restrict__ gate)
{
    // a step that reuses its cell table kicks and drifts in k_pack instead
    if (gate != nullptr && *gate == 0) return;
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
        k = I.cell_base + cell_key(sc, I, cc[0], cc[1], cc[2]);
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
                                                  sc.N, d.key, d.cnt, d.clampc, d.flags, d.gate);
    else
        k_keys<3><<<d.nfchunks, d.block, 0, s>>>(sc, d.fmap, d.inst, d.x, d.v, d.a, d.dt, kick_on,
                                                  sc.N, d.key, d.cnt, d.clampc, d.flags, d.gate);
    return hipGetLastError();
}

hipError_t launch_wall_keys(const SimConst &sc, const Dev &d, hipStream_t s)
{
    if (d.nwchunks <= 0) return hipSuccess;
    // walls are read only: kick is off, so x and v are never written
    double *xw = const_cast<double *>(d.xw);
    if (sc.dim == 2)
        k_keys<2><<<d.nwchunks, d.block, 0, s>>>(sc, d.wmap, d.inst, xw, nullptr, nullptr, d.dt, 0,
                                                  sc.Nw, d.wkey, d.cnt, d.clampc, d.flags, nullptr);
    else
        k_keys<3><<<d.nwchunks, d.block, 0, s>>>(sc, d.wmap, d.inst, xw, nullptr, nullptr, d.dt, 0,
                                                  sc.Nw, d.wkey, d.cnt, d.clampc, d.flags, nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reorder and sweep records
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(kMaxBlock) void k_reorder_gather(
    const Chunk *__restrict__ map, const int *__restrict__ perm, const double *__restrict__ x,
    const double *__restrict__ v, const double *__restrict__ rho, const int *__restrict__ id,
    double *__restrict__ scr, int n, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
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
    int *__restrict__ id, int *__restrict__ perm, int *__restrict__ key, int n, const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
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
    // with a skin the reduction of the previous step decides (gate[1])
    const int *g = d.gate ? d.gate + 1 : nullptr;
    if (sc.dim == 2) {
        k_reorder_gather<2><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.perm, d.x, d.v, d.rho, d.id, d.scratch, sc.N, g);
        k_reorder_copy<2><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.scratch, d.skey, d.x, d.v, d.rho, d.id, d.perm, d.key, sc.N, g);
    } else {
        k_reorder_gather<3><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.perm, d.x, d.v, d.rho, d.id, d.scratch, sc.N, g);
        k_reorder_copy<3><<<d.nfchunks, d.block, 0, s>>>(d.fmap, d.scratch, d.skey, d.x, d.v, d.rho, d.id, d.perm, d.key, sc.N, g);
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

constexpr int kReduceBlock = 256;      // second level: one block per instance over its first-level rows

// Verlet skin: called once per instance (thread 0 of its reduction block)
// with the step dt_n it planned and the max|v|, max|a| the next drift starts
// from.  That drift moves a particle by dt_n (|v| + dt_n |a| / 2) at most.
// The last instance to arrive plans the next step: while twice the summed
// bounds since the last build stay below the skin, every pair closer than 2h
// was closer than 2h + skin at the build, so the cell table and the lists of
// that build still hold all of them; otherwise the next step rebuilds both.
// Gates of the next step from its rebuild decision: reorder on a rebuild at
// least reorder_every steps after the last reorder; count the builds.
__device__ void skin_gates(const SimConst &sc, int *__restrict__ gate, bool rebuild)
{
    const bool built = gate[0] != 0;
    const bool reordered = gate[1] != 0;
    const int since = reordered ? 1 : gate[2] + (gate[2] < (1 << 30) ? 1 : 0);
    gate[0] = rebuild ? 1 : 0;
    gate[1] = (rebuild && sc.reorder_every > 0 && since >= sc.reorder_every) ? 1 : 0;
    gate[2] = since;
    gate[3] = 0;
    if (built) gate[4] += 1;
}

__device__ void skin_plan(const SimConst &sc, int *__restrict__ gate, double *__restrict__ disp,
                          double dt_n, double vmax, double amax)
{
    double bound = dt_n * (vmax + 0.5 * dt_n * amax);
    if (!(bound >= 0.0 && bound < 1e300)) bound = 1e300;     // non-finite state: rebuild
    auto *bits = reinterpret_cast<unsigned long long *>(disp + 1);
    atomicMax(bits, (unsigned long long)__double_as_longlong(bound));
    __threadfence();
    if (atomicAdd(&gate[3], 1) != sc.n_inst - 1) return;
    __threadfence();
    const double next = __longlong_as_double((long long)atomicExch(bits, 0ull));
    const double since_build = (gate[0] != 0 ? 0.0 : disp[0]) + next;
    // margin: far above the rounding of positions and of FP32 pair distances
    const bool rebuild = !(2.0 * since_build < sc.skin * (1.0 - 1e-4));
    disp[0] = rebuild ? 0.0 : since_build;
    skin_gates(sc, gate, rebuild);
}

// Dual scheme with a skin.  The acoustic sub-steps keep the pairs of their
// advection step, so the list of a build serves an advection step as long as
// no particle has moved skin / 2 or more since that build (no pair closer
// than 2h can then have been 2h + skin or further apart).  The test takes the
// exact displacements at the end of an advection step, which are those at
// the start of the next; disp[1] holds the largest squared one as ordered bits.
__global__ __launch_bounds__(256) void k_skin_displacement(SimConst sc, const double *__restrict__ x,
                                                           const double *__restrict__ xb,
                                                           int *__restrict__ gate, double *__restrict__ disp)
{
    const int64_t n = sc.N;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d2 = 0.0;
        for (int c = 0; c < sc.dim; ++c) {
            const double e = x[c * n + i] - xb[c * n + i];
            d2 += e * e;
        }
        if (!(d2 <= 1e300)) d2 = 1e300;                       // non-finite position: rebuild
        m = d2 > m ? d2 : m;
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    auto *bits = reinterpret_cast<unsigned long long *>(disp + 1);
    atomicMax(bits, (unsigned long long)__double_as_longlong(red[0]));
    __threadfence();
    if (atomicAdd(&gate[3], 1) != (int)gridDim.x - 1) return;
    __threadfence();
    const double D = sqrt(__longlong_as_double((long long)atomicExch(bits, 0ull)));
    skin_gates(sc, gate, !(2.0 * D < sc.skin * (1.0 - 1e-4)));
}

// Positions at a build (runs when gate[0] != 0).
__global__ void k_save_build_positions(double *__restrict__ xb, const double *__restrict__ x, int64_t n,
                                       const int *__restrict__ gate)
{
    if (*gate == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        xb[i] = x[i];
}

hipError_t launch_skin_displacement(const SimConst &sc, const Dev &d, hipStream_t s)
{
    k_skin_displacement<<<fill_grid(sc.N), 256, 0, s>>>(sc, d.x, d.xb, d.gate, d.disp);
    return hipGetLastError();
}

hipError_t launch_save_build_positions(const SimConst &sc, const Dev &d, hipStream_t s)
{
    const int64_t n = (int64_t)sc.dim * sc.N;
    if (n <= 0) return hipSuccess;
    k_save_build_positions<<<fill_grid(n), 256, 0, s>>>(d.xb, d.x, n, d.gate);
    return hipGetLastError();
}

// First level: the chunk rows [begin, end) of one instance, summed (maxima for
// the max slots) into output row id.
__global__ __launch_bounds__(256) void k_reduce_rows(const Chunk *__restrict__ rmap,
                                                     const double *__restrict__ partials,
                                                     double *__restrict__ subpart)
{
    const Chunk rb = rmap[blockIdx.x];
    constexpr int R = 256 / kNPart;
    const int q = threadIdx.x % kNPart;
    const int r0 = threadIdx.x / kNPart;
    const bool mx = is_max_slot(q);
    double acc = 0.0;                      // the max slots hold non-negative values
#pragma unroll 8
    for (int c = rb.begin + r0; c < rb.end; c += R) {
        const double x = partials[(int64_t)c * kNPart + q];
        acc = mx ? fmax(acc, x) : acc + x;
    }
    __shared__ double rows[R][kNPart];
    rows[r0][q] = acc;
    __syncthreads();
    if (threadIdx.x < kNPart) {
        double t = rows[0][q];
        for (int r = 1; r < R; ++r) t = mx ? fmax(t, rows[r][q]) : t + rows[r][q];
        subpart[(int64_t)rb.id * kNPart + q] = t;
    }
}

__global__ __launch_bounds__(kReduceBlock) void k_final_reduce(
    SimConst sc, const InstDev *__restrict__ inst, const double *__restrict__ partials,
    double *__restrict__ dt, double *__restrict__ diag, int *__restrict__ clampc,
    unsigned *__restrict__ flags, int prime, int *__restrict__ nsub, double *__restrict__ dtsub,
    int *__restrict__ nsub_max, int *__restrict__ gate, double *__restrict__ disp)
{
    const int b = blockIdx.x;
    const InstDev &I = inst[b];
    // thread t sums slot t % 16 over rows t / 16, t / 16 + R, ...: a wave reads
    // four whole 128-byte rows per load instead of 64 scattered ones
    constexpr int R = kReduceBlock / kNPart;
    const int q = threadIdx.x % kNPart;
    const int r0 = threadIdx.x / kNPart;
    const bool mx = is_max_slot(q);
    double acc = 0.0;                      // the max slots hold non-negative values
    for (int c = I.sub_begin + r0; c < I.sub_end; c += R) {
        const double x = partials[(int64_t)c * kNPart + q];
        acc = mx ? fmax(acc, x) : acc + x;
    }
    __shared__ double rows[R][kNPart];
    __shared__ double tot[kNPart];
    rows[r0][q] = acc;
    __syncthreads();
    if (threadIdx.x < kNPart) {
        double t = rows[0][q];
        for (int r = 1; r < R; ++r) t = mx ? fmax(t, rows[r][q]) : t + rows[r][q];
        tot[q] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *d = diag + (int64_t)b * 16;
        const double dt_used = prime ? 0.0 : dt[b];
        const double vmax = tot[P_VMAX], amax = tot[P_AMAX];
        fill_diag(sc, I, tot, dt_used, clampc[b], prime, d);
        clampc[b] = 0;
        if (sc.scheme == 1) {
            // dual-criteria plan of the next advection step: Dt from the
            // flow speed (floored at c0 / 10), equal acoustic sub-steps
            const double uref = I.c0 / 10.0;
            const double Dt = sc.cfl_adv * sc.h / (vmax > uref ? vmax : uref);
            const double dac = sc.cfl_sub * sc.h / (I.c0 + vmax);
            // ceil(Dt / dac) <= nsub_bound for every finite max|v| (see
            // sph_create); a non-finite one plans one sub-step and is flagged
            const double q = ceil(Dt / dac);
            const int ns = !(q >= 1.0) ? 1 : (q > (double)sc.nsub_bound ? sc.nsub_bound : (int)q);
            dt[b] = Dt;
            nsub[b] = ns;
            dtsub[b] = Dt / (double)ns;
            atomicMax(nsub_max, ns);
        } else {
            dt[b] = cfl_dt(sc, I.c0, vmax, amax);
            if (gate) skin_plan(sc, gate, disp, dt[b], vmax, amax);
        }
        if (tot[P_BAD] > 0.0) atomicOr(flags, 2u);
    }
}

// Dual scheme: add the planned sub-steps of the advection step about to run
// (the largest count over the instances) to the running total.
__global__ void k_count_substeps(const int *__restrict__ nsub_max, unsigned long long *__restrict__ total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *total += (unsigned long long)*nsub_max;
}

hipError_t launch_count_substeps(const Dev &d, hipStream_t s)
{
    k_count_substeps<<<1, 64, 0, s>>>(d.nsub_max, d.subs_total);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const SimConst &sc, const Dev &d, int prime, hipStream_t s)
{
    if (sc.n_inst <= 0) return hipSuccess;
    if (d.nrblocks > 0) k_reduce_rows<<<d.nrblocks, 256, 0, s>>>(d.rmap, d.partials, d.subpart);
    k_final_reduce<<<sc.n_inst, kReduceBlock, 0, s>>>(sc, d.inst, d.subpart, d.dt, d.diag, d.clampc, d.flags, prime,
                                                      d.nsub, d.dtsub, d.nsub_max, d.gate, d.disp);
    return hipGetLastError();
}

}  // namespace sphx
