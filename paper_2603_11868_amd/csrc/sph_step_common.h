// Device helpers shared by the streaming kernels and the pair sweeps.
#pragma once

#include "sph_launch.h"

namespace sphx {

// Half-step kick and drift, rounded like the plain expressions (no FMA).
__device__ __forceinline__ void kick_drift(double &x, double &v, double a, double dt)
{
#pragma clang fp contract(off)
    v = v + 0.5 * dt * a;
    x = x + dt * v;
}


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

// Half-step kick, rounded like the plain expression (no FMA).
__device__ __forceinline__ double kick(double v, double a, double dt)
{
#pragma clang fp contract(off)
    return v + 0.5 * dt * a;
}

// |r| from r^2 and reciprocals in the pair loops.  FP64: the hardware
// estimates refined by Newton (Goldschmidt) steps to within about 1 ulp, with
// none of the range scaling a general square root or IEEE division needs
// (r^2 here is 0 or a normal number below (2h)^2; divisors are densities and
// sums of positive terms).  FP32: the hardware square root and reciprocal
// (1 ulp), which the mixed path's tolerance covers.
__device__ __forceinline__ double root(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    double g = r2 * y, hh = 0.5 * y;
    const double e = fma(-g, hh, 0.5);
    g = fma(g, e, g);
    hh = fma(hh, e, hh);
    double d = fma(-g, g, r2);
    g = fma(d, hh, g);
    d = fma(-g, g, r2);
    g = fma(d, hh, g);
    return r2 > 0.0 ? g : 0.0;
}
__device__ __forceinline__ float root(float r2) { return __builtin_amdgcn_sqrtf(r2); }

__device__ __forceinline__ double recip(double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float recip(float b) { return __builtin_amdgcn_rcpf(b); }

// Wendland C2: W = kW t^4 (2q + 1), F = (1/r) dW/dr = kF t^3, t = 1 - q/2.
template <class real>
__device__ __forceinline__ void kernel_WF(real r2, real inv_h, real kW, real kF, real &W, real &F)
{
    const real rr = root(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    const real t3 = t * t * t;
    W = kW * t3 * t * ((real)2 * q + (real)1);
    F = kF * t3;
}

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

template <class real>
__device__ __forceinline__ void kernel_F(real r2, real inv_h, real kF, real &F)
{
    const real rr = root(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    F = kF * t * t * t;
}

// ---- block partial sums (deterministic: fixed lanes, fixed butterfly, fixed wave order)

// slots: 0 max|v| 1 max|a| 2..4 sum m v 5 kinetic 6 potential 7 internal
//        8..10 sum m a_ff 11 sum rho 12 pairs 13 non-finite count
enum { P_VMAX = 0, P_AMAX = 1, P_MOM = 2, P_KE = 5, P_PE = 6, P_IE = 7, P_FF = 8,
       P_RHO = 11, P_PAIRS = 12, P_BAD = 13 };

__device__ __forceinline__ bool is_max_slot(int s) { return s == P_VMAX || s == P_AMAX; }

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

}  // namespace sphx
