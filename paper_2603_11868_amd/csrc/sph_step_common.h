// Device helpers shared by the streaming kernels and the pair sweeps.
#pragma once

#include "sph_launch.h"
#include "sph_bodies.h"

namespace sphx {

// |r| from an FP64 r^2 for the mixed path's density summation: the FP32
// reciprocal square root refined by one Newton step in FP64 (relative error
// about 2e-14, far below what the summation needs).
__device__ __forceinline__ double root_seeded(double r2)
{
    const double y = (double)__builtin_amdgcn_rsqf((float)r2);
    const double g = r2 * y;
    const double e = fma(-g, 0.5 * y, 0.5);
    return r2 > 0.0 ? fma(g, e, g) : 0.0;
}

// Wendland C2 in FP64 from an FP64 r^2 (lengths in any unit: inv_h = 1 / h in
// that unit), with F rounded to FP32 (mixed path: W enters the summation
// density, F only the continuity term).
__device__ __forceinline__ void kernel_WF_exact(double r2, double inv_h, double kW, double kF, double &W, float &F)
{
    const double rr = root_seeded(r2);
    const double q = rr * inv_h;
    const double t = 1.0 - 0.5 * q;
    const double t3 = t * t * t;
    W = kW * t3 * t * (2.0 * q + 1.0);
    F = (float)(kF * t3);
}

// ---- block partial sums (deterministic: fixed lanes, fixed butterfly, fixed wave order)

// Reduce vals[LO..HI) over the block (at most MAXW waves) and write them to
// out[LO..HI).
template <int LO, int HI, int MAXW = kMaxBlock / 64>
__device__ __forceinline__ void block_partials(double (&vals)[kNPart], double *__restrict__ out)
{
    __shared__ double sh[MAXW][kNPart];
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

}  // namespace sphx
