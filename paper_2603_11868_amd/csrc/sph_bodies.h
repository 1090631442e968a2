// Per-particle and per-pair bodies of the WCSPH step, shared by the GPU
// kernels and the host executor (sph_host.hip): the cell key of a position,
// the half kick and drift, the Wendland kernel, the density pair and the
// density update (summation with the free-surface rule, EOS), the force pair
// (pressure, Monaghan viscosity, wall mirror), the diagnostics of a particle
// and the CFL time step.  The paper runs one kernel source under several
// execution policies (Sec. 4, and the single-source goal of its conclusion);
// here one definition of each body serves both executors.
//
// The only split between the two compilations is the square root and the
// reciprocal of the FP64 pair loops: on the GPU the hardware estimates refined
// by Newton steps (about 1 ulp), on the host the correctly rounded operations.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sph_device.h"

#define SPHX_HD __host__ __device__ __forceinline__

namespace sphx {

// ---- arithmetic helpers ------------------------------------------------------

// |r| from r^2 and reciprocals in the pair loops.  FP64 on the GPU: the
// hardware estimates refined by Newton (Goldschmidt) steps to within about
// 1 ulp, with none of the range scaling a general square root or IEEE
// division needs (r^2 here is 0 or a normal number below (2h)^2; divisors are
// densities and sums of positive terms).  FP32 (GPU only): the hardware square
// root and reciprocal (1 ulp), which the mixed path's tolerance covers.
SPHX_HD double root(double r2)
{
#if defined(__HIP_DEVICE_COMPILE__)
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
#else
    return sqrt(r2);
#endif
}

SPHX_HD double recip(double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    return fma(y, e, y);
#else
    return 1.0 / b;
#endif
}

SPHX_HD float root(float r2)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(r2);
#else
    return sqrtf(r2);
#endif
}

SPHX_HD float recip(float b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(b);
#else
    return 1.0f / b;
#endif
}

// r^2 summed left to right without FMA: the predicate r^2 < (2h)^2 of the FP64
// path then matches a plain IEEE evaluation bit for bit.
SPHX_HD double dist2(double rx, double ry)
{
#pragma clang fp contract(off)
    return rx * rx + ry * ry;
}
SPHX_HD double dist2(double rx, double ry, double rz)
{
#pragma clang fp contract(off)
    return rx * rx + ry * ry + rz * rz;
}
SPHX_HD float dist2(float rx, float ry) { return rx * rx + ry * ry; }
SPHX_HD float dist2(float rx, float ry, float rz) { return rx * rx + ry * ry + rz * rz; }

// ---- integration -------------------------------------------------------------

// Half-step kick and drift, rounded like the plain expressions (no FMA).
SPHX_HD void kick_drift(double &x, double &v, double a, double dt)
{
#pragma clang fp contract(off)
    v = v + 0.5 * dt * a;
    x = x + dt * v;
}

// Half-step kick, rounded like the plain expression (no FMA).
SPHX_HD double kick(double v, double a, double dt)
{
#pragma clang fp contract(off)
    return v + 0.5 * dt * a;
}

// ---- cells -------------------------------------------------------------------

// floor((x - lo) * inv_cs) clamped to [0, n); subtract then multiply, no FMA.
SPHX_HD int cell_1d(double x, double lo, double inv_cs, int n, int &clamped)
{
#pragma clang fp contract(off)
    const double t = floor((x - lo) * inv_cs);
    if (!(t >= 0.0)) { clamped = 1; return 0; }
    if (t >= (double)n) { clamped = 1; return n - 1; }
    return (int)t;
}

// ---- kernel ------------------------------------------------------------------

// Wendland C2: W = kW t^4 (2q + 1), F = (1/r) dW/dr = kF t^3, t = 1 - q/2.
template <class real>
SPHX_HD void kernel_WF(real r2, real inv_h, real kW, real kF, real &W, real &F)
{
    const real rr = root(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    const real t3 = t * t * t;
    W = kW * t3 * t * ((real)2 * q + (real)1);
    F = kF * t3;
}

template <class real>
SPHX_HD void kernel_F(real r2, real inv_h, real kF, real &F)
{
    const real rr = root(r2);
    const real q = rr * inv_h;
    const real t = (real)1 - (real)0.5 * q;
    F = kF * t * t * t;
}

// ---- density -----------------------------------------------------------------

// One pair of the density sweep: the kernel value enters the summation, the
// divergence term v_ij . F r_ij the continuity sum.
template <int DIM, class real>
SPHX_HD void density_pair(const real *r, real r2, const real *vi, const real *vj, real inv_h, real kW,
                          real kF, double &sigma, real &drho, int &cnt)
{
    real W, F;
    kernel_WF(r2, inv_h, kW, kF, W, F);
    real vr = (vi[0] - vj[0]) * r[0] + (vi[1] - vj[1]) * r[1];
    if constexpr (DIM == 3) vr += (vi[2] - vj[2]) * r[2];
    sigma += W;
    drho += vr * F;
    ++cnt;
}

// Density of a particle after the sweep: summation density rho_sum = m sigma
// (sigma with W(0)), continuity update rho* = rho + dt m drho, and the
// free-surface rule rho = rho_sum + max(0, rho* - rho_sum) rho0 / rho*; then
// p = max(0, c0^2 (rho - rho0)) and P = p / rho^2.  m_drho: m times the
// continuity sum.
SPHX_HD void density_update(double rho_old, double sigma, double m_drho, double dt, double mass, double rho0,
                            double c0, double &rn, double &P)
{
    const double rho_sum = mass * sigma;
    const double rho_star = rho_old + dt * m_drho;
    const double excess = rho_star - rho_sum;
    rn = excess > 0.0 ? rho_sum + excess * rho0 / rho_star : rho_sum;
    double p = c0 * c0 * (rn - rho0);
    if (p < 0.0) p = 0.0;
    P = p / (rn * rn);
}

// ---- force -------------------------------------------------------------------

// One pair of the force sweep, branch-free over fluid and wall sources (lanes
// of a wave mix them): the wall mirror pressure is computed for every pair and
// selected.  A wall source carries zero velocity, rho_j = rho_i and
// p_j = max(0, p_i + rho_i g.(x_j - x_i)).  acc and aff (fluid sources only)
// accumulate -sum (P_i + P_j + Pi_ij) F r.  Target values: vi, rho_i, P_i,
// p_i = P_i rho_i^2, inv_rho_i2 = 1 / rho_i^2; sweep constants (lengths in the
// units of r): inv_h, kF, visc_a = alpha c0 h, eps_h2, g.
template <int DIM, class real>
SPHX_HD void force_pair(bool wall, const real *r, real r2, const real *vi, const real *vj, real rho_i, real P_i,
                        real p_i, real inv_rho_i2, real rho_rec, real P_rec, real inv_h, real kF, real visc_a,
                        real eps_h2, real gx, real gy, real gz, real *acc, real *aff, int &cnt)
{
    real F;
    kernel_F(r2, inv_h, kF, F);
    real vr = (vi[0] - vj[0]) * r[0] + (vi[1] - vj[1]) * r[1];
    if constexpr (DIM == 3) vr += (vi[2] - vj[2]) * r[2];
    real gr = gx * r[0] + gy * r[1];
    if constexpr (DIM == 3) gr += gz * r[2];
    real p_m = p_i - rho_i * gr;           // wall mirror: p_i + rho_i g.(x_j - x_i)
    p_m = p_m < (real)0 ? (real)0 : p_m;
    const real rho_j = wall ? rho_i : rho_rec;
    const real P_j = wall ? p_m * inv_rho_i2 : P_rec;
    real visc = 0;
    if constexpr (sizeof(real) == sizeof(float)) {
        // FP32 (the mixed GPU path): branch-free, vr clamped to <= 0 (a
        // receding pair then adds a signed zero to P_i + P_j >= +0, which
        // leaves the sum as it is); the lanes of a wave mix approaching and
        // receding pairs, and the hardware reciprocal is one instruction
        const real den = (real)0.5 * (rho_i + rho_j) * (r2 + eps_h2);
        visc = -visc_a * (vr < (real)0 ? vr : (real)0) * recip(den);
    } else if (vr < (real)0) {
        const real den = (real)0.5 * (rho_i + rho_j) * (r2 + eps_h2);
        visc = -visc_a * vr * recip(den);
    }
    const real coef = (P_i + P_j + visc) * F;
    const real coef_ff = wall ? (real)0 : coef;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        acc[c] -= coef * r[c];
        aff[c] -= coef_ff * r[c];
    }
    ++cnt;
}

// ---- diagnostics and time step -----------------------------------------------

// slots: 0 max|v| 1 max|a| 2..4 sum m v 5 kinetic 6 potential 7 internal
//        8..10 sum m a_ff 11 sum rho 12 pairs 13 non-finite count
enum { P_VMAX = 0, P_AMAX = 1, P_MOM = 2, P_KE = 5, P_PE = 6, P_IE = 7, P_FF = 8,
       P_RHO = 11, P_PAIRS = 12, P_BAD = 13 };

SPHX_HD bool is_max_slot(int s) { return s == P_VMAX || s == P_AMAX; }

// Contributions of one particle to the step diagnostics (FP64).
template <int DIM>
SPHX_HD void state_partials(const SimConst &sc, const InstDev &I, const double *vn, const double *an,
                            const double *xi, double rhoi, double (&vals)[kNPart])
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

// The next step's dt of an instance from its max|v| and max|a|:
// min(C_ac h / (c0 + max|v|), C_f sqrt(h / max|a|)).
SPHX_HD double cfl_dt(const SimConst &sc, double c0, double vmax, double amax)
{
    const double dt_ac = sc.cfl_ac * sc.h / (c0 + vmax);
    const double dt_f = sc.cfl_f * sqrt(sc.h / amax);
    return dt_ac < dt_f ? dt_ac : dt_f;
}

// The per-instance diagnostics (16 doubles) from the summed slots tot of the
// step; dt_used: the dt of the step (0 for the prime).
SPHX_HD void fill_diag(const SimConst &sc, const InstDev &I, const double *tot, double dt_used, int clamped,
                       int prime, double *d)
{
    d[0] = tot[P_VMAX];
    d[1] = tot[P_AMAX];
    d[2] = sc.mass * (double)I.n_fluid;
    for (int c = 0; c < 3; ++c) d[3 + c] = tot[P_MOM + c];
    d[6] = tot[P_KE];
    d[7] = tot[P_PE];
    d[8] = tot[P_IE];
    const double ff = sqrt(tot[P_FF] * tot[P_FF] + tot[P_FF + 1] * tot[P_FF + 1] + tot[P_FF + 2] * tot[P_FF + 2]);
    d[9] = ff;
    d[10] = I.n_fluid > 0 ? tot[P_RHO] / ((double)I.n_fluid * sc.rho0) - 1.0 : 0.0;
    d[11] += (double)clamped;
    d[12] = tot[P_PAIRS];
    d[13] += dt_used * ff;
    d[14] += dt_used;
    d[15] = prime ? 0.0 : d[15] + 1.0;
}

}  // namespace sphx
