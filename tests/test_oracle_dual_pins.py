"""Pins of the second scheme of the FP64 CPU reference: dual-criteria time
stepping with an acoustic Riemann-solver pressure.

As for the first scheme, every test checks the reference against something
other than itself: the characteristic relations of the acoustic Riemann
problem, symmetries, exact rest states, conservation, a hydrostatic column
and a shallow-water bound.  None of these needs a GPU.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import dambreak
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C0 = 40.0


# ---------------------------------------------------------------------------
# the Riemann solver
# ---------------------------------------------------------------------------

def test_riemann_equal_states():
    ps, us = O.riemann(1010.0, 3.0e4, 0.7, 1010.0, 3.0e4, 0.7, C0)
    assert ps == pytest.approx(3.0e4, rel=1e-15)
    assert us == pytest.approx(0.7, rel=1e-15)


@pytest.mark.parametrize("rl,pl,ul,rr,pr,ur", [
    (1000.0, 2.0e4, 10.0, 1020.0, 1.0e4, -5.0),   # strong compression: limiter saturated
    (990.0, 0.0, 0.5, 1005.0, 5.0e4, -40.0),
])
def test_riemann_full_dissipation_satisfies_both_characteristics(rl, pl, ul, rr, pr, ur):
    # with beta = 1 the star state lies on the left-going and right-going
    # acoustic characteristics: p* - p_L = -Z_L (u* - u_L), p* - p_R = Z_R (u* - u_R)
    assert 3.0 * (ul - ur) / C0 >= 1.0
    ps, us = O.riemann(rl, pl, ul, rr, pr, ur, C0)
    zl, zr = rl * C0, rr * C0
    assert ps - pl == pytest.approx(-zl * (us - ul), rel=1e-12)
    assert ps - pr == pytest.approx(zr * (us - ur), rel=1e-12)


def test_riemann_limiter_scales_the_dissipation():
    rl, pl, rr, pr = 1000.0, 2.0e4, 1000.0, 2.4e4
    z = 1000.0 * C0
    base = (z * pr + z * pl) / (2 * z)
    # expansion: no dissipation, the impedance-weighted pressure
    ps, _ = O.riemann(rl, pl, -1.0, rr, pr, 1.0, C0)
    assert ps == pytest.approx(base, rel=1e-15)
    # weak compression du: beta = 3 du / c0, so P* - base = Z beta du / 2
    du = 0.5
    ps, _ = O.riemann(rl, pl, du, rr, pr, 0.0, C0)
    assert ps - base == pytest.approx(z * (3 * du / C0) * du / 2, rel=1e-12)


def test_riemann_mirror_symmetry():
    # the same pair seen from the other particle: the axis flips, so the left
    # and right states swap and both normal velocities change sign
    a = (1003.0, 1.2e4, 0.8)
    b = (996.0, 0.9e4, -0.3)
    p1, u1 = O.riemann(*a, *b, C0)
    p2, u2 = O.riemann(b[0], b[1], -b[2], a[0], a[1], -a[2], C0)
    assert p1 == pytest.approx(p2, rel=1e-14)
    assert u1 == pytest.approx(-u2, rel=1e-14)


def test_riemann_galilean_invariance_of_pressure():
    p1, u1 = O.riemann(1001.0, 5e3, 0.4, 999.0, 6e3, -0.2, C0)
    p2, u2 = O.riemann(1001.0, 5e3, 2.4, 999.0, 6e3, 1.8, C0)
    assert p1 == pytest.approx(p2, rel=1e-14)
    assert u2 - u1 == pytest.approx(2.0, rel=1e-12)


# ---------------------------------------------------------------------------
# the scheme
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_block_at_rest_without_gravity_stays_at_rest(dim):
    # on a perfect lattice the free-surface summation gives rho0 everywhere
    # (to rounding), so p = 0, every interface state vanishes and nothing moves
    case = dambreak.make_case("tiny_2d" if dim == 2 else "tiny_3d")
    inst = case.instances[0]
    dx = case.dx
    fluid = (np.round(inst.fluid / dx - 0.5) + 0.5) * dx          # jitter removed
    r = O.OracleSim(dim, dx, case.h, inst.tank_lo, inst.tank_hi, fluid, inst.wall, inst.c0,
                    g=(0.0,) * dim, reorder_every=0)
    r.dual_prime()
    x0 = r.x.copy()
    r.dual_step(5)
    assert np.abs(r.v).max() < 1e-9
    assert np.abs(r.x - x0).max() < 1e-12
    assert np.abs(r.rho - 1000.0).max() < 1e-9


def test_plan_of_the_advection_step():
    case = dambreak.make_case("c1_2d")
    r = O.OracleSim.from_case(case)
    r.dual_prime()
    c0, h = case.instances[0].c0, case.h
    Dt, n, dt = r.dual_plan()
    assert Dt == pytest.approx(O.DUAL_CFL_ADV * h / (c0 / 10), rel=1e-15)
    assert n == math.ceil(Dt / (O.DUAL_CFL_AC * h / c0))
    assert n * dt == pytest.approx(Dt, rel=1e-15)
    r.dual_step(3)
    vmax = r.diag[0]
    Dt, n, dt = r.dual_plan()
    assert Dt == pytest.approx(O.DUAL_CFL_ADV * h / max(vmax, c0 / 10), rel=1e-15)
    assert dt <= O.DUAL_CFL_AC * h / (c0 + vmax) * (1 + 1e-12)
    assert r.diag[14] > 0 and r.diag[15] == 3


def test_fluid_fluid_momentum_is_conserved_and_mass_exact():
    case = dambreak.make_case("c1_2d")
    r = O.OracleSim.from_case(case)
    r.dual_prime()
    r.dual_step(20)
    scale = r.mass * r.n * np.abs(r.a).max()
    assert r.diag[9] < 1e-12 * scale
    assert r.diag[2] == r.mass * r.n


def test_linear_pressure_field_gradient():
    # equal densities and no relative motion: P* is the mean pressure and the
    # pressure sweep gives -grad(p)/rho up to the lattice discretisation error
    dim, n, dx = 2, 30, 0.02
    x = (np.stack(np.meshgrid(np.arange(n), np.arange(n), indexing="ij"), -1)
                            .reshape(-1, 2) + 0.5) * dx
    r = O.OracleSim(dim, dx, 1.3 * dx, (0.0, 0.0), (n * dx, n * dx), x, np.zeros((0, 2)), 20.0,
                    g=(0.0, 0.0), reorder_every=0)
    r.keys(); r.sort()
    r.dual_stage("summation")
    kappa, rho = 1000.0, 1000.0
    r.rho[:] = rho
    r.pres[:] = 2000.0 + kappa * x[:, 1]
    r.dual_stage("pressure", 0.0)
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 4) & (idx < n - 4), axis=1)
    ay = r.a[interior, 1]
    assert np.allclose(ay, ay.mean(), rtol=1e-9)
    assert abs(ay.mean() / (-kappa / rho) - 1.0) < 0.05
    assert np.abs(r.a[interior, 0]).max() < 1e-9


def _lattice_sim(dim, n, dx, v=None):
    axes = [np.arange(n)] * dim
    x = (np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, dim) + 0.5) * dx
    r = O.OracleSim(dim, dx, 1.3 * dx, (0.0,) * dim, (n * dx,) * dim, x, np.zeros((0, dim)), 20.0,
                    g=(0.0,) * dim, reorder_every=0, v=v)
    r.keys(); r.sort()
    r.dual_stage("summation")
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 3) & (idx < n - 3), axis=1)
    return r, x, interior


@pytest.mark.parametrize("dim", [2, 3])
def test_dual_continuity_of_linear_compression(dim):
    # v = -beta (x - c) at uniform density and pressure: the velocity jump is
    # v_i - v* = (v_i - v_j) / 2, so Drho_i = sum_j m (v_i - v_j).grad W_ij,
    # which is rho0 d beta (div v = -d beta) up to the lattice error
    n, dx, beta = (24, 0.01, 2.0) if dim == 2 else (12, 0.01, 2.0)
    axes = [np.arange(n)] * dim
    x = (np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, dim) + 0.5) * dx
    r, x, interior = _lattice_sim(dim, n, dx, v=-beta * (x - x.mean(0)))
    r.rho[:] = 1000.0
    r.pres[:] = 5000.0
    r.dual_stage("density", 0.0)
    ratio = r.drho[interior] / (1000.0 * dim * beta)
    assert np.all(np.abs(ratio - 1.0) < 0.05), (ratio.min(), ratio.max())


@pytest.mark.parametrize("dim", [2, 3])
def test_dual_continuity_pressure_term(dim):
    # at rest with p = kappa y^2 and uniform density the velocity jump is the
    # acoustic term (p_i - p_j) / (Z_i + Z_j) e, so
    # Drho_i = sum_j (m / rho) (p_i - p_j) F_ij |r_ij| / c0; the odd part of
    # p_i - p_j = 2 y_i r_y - r_y^2 cancels on the lattice, leaving
    # -(kappa / c0) int F(r) r r_y^2 dV = -(kappa / c0) (S_d / d) int_0^2h F r^(d+2) dr
    # (S_2 = 2 pi, S_3 = 4 pi) up to the lattice error.  Positive: the
    # pressure term diffuses pressure maxima into their neighbourhood.
    from scipy import integrate
    n, dx = (24, 0.01) if dim == 2 else (12, 0.01)
    h, kappa, c0 = 1.3 * dx, 3.0e5, 20.0
    r, x, interior = _lattice_sim(dim, n, dx)
    r.rho[:] = 1000.0
    r.pres[:] = kappa * x[:, dim - 1] ** 2
    r.dual_stage("density", 0.0)
    S = 2 * math.pi if dim == 2 else 4 * math.pi
    moment, _ = integrate.quad(lambda q: O.F(dim, h, q) * q ** (dim + 2), 0.0, 2 * h,
                               epsabs=0.0, epsrel=1e-12)
    want = -(kappa / c0) * (S / dim) * moment
    assert want > 0
    ratio = r.drho[interior] / want
    assert np.all(np.abs(ratio - 1.0) < 0.05), (ratio.min(), ratio.max())


def test_dual_continuity_pair_with_unequal_states():
    # one isolated pair with different densities, pressures and velocities:
    # Drho_1 = 2 rho_1 (m / rho_2) (v_1 - v*).grad_1 W with
    # v_1 - v* = Z_2 (v_1 - v_2) / (Z_1 + Z_2) + (p_1 - p_2) / (Z_1 + Z_2) e,
    # Z = rho c0, e = r_12 / |r_12|, evaluated from the numbers
    dim, dx, c0 = 2, 0.02, 20.0
    h = 1.3 * dx
    x = np.array([[0.1, 0.1], [0.1 + 1.1 * h * 0.8, 0.1 - 1.1 * h * 0.6]])
    v = np.array([[0.3, 0.05], [-0.2, 0.1]])
    r = O.OracleSim(dim, dx, h, (0.0, 0.0), (0.2, 0.2), x, np.zeros((0, 2)), c0,
                    g=(0.0, 0.0), reorder_every=0, v=v)
    r.keys(); r.sort()
    r.dual_stage("summation")
    rho = np.array([1000.0, 1200.0])
    p = np.array([3000.0, 5000.0])
    r.rho[:] = rho
    r.pres[:] = p
    r.dual_stage("density", 0.0)
    r12 = x[0] - x[1]
    e = r12 / np.linalg.norm(r12)
    z1, z2 = rho * c0
    dv = z2 * (v[0] - v[1]) / (z1 + z2) + (p[0] - p[1]) / (z1 + z2) * e
    eps = 1e-7 * h
    grad = np.array([(O.W(2, h, np.linalg.norm(r12 + eps * u)) - O.W(2, h, np.linalg.norm(r12 - eps * u)))
                     / (2 * eps) for u in np.eye(2)])
    want = 2.0 * rho[0] * (r.mass / rho[1]) * float(dv @ grad)
    assert r.drho[0] == pytest.approx(want, rel=1e-6)


def test_hydrostatic_column_time_average():
    case = dambreak.make_case("hydrostatic_2d")
    inst = case.instances[0]
    H, c0 = inst.height, inst.c0
    r = O.OracleSim.from_case(case)
    r.dual_prime()
    period = 4 * H / c0
    ke_early = 0.0
    while r.diag[14] < 6 * period:
        r.dual_step(10)
        if r.diag[14] < period:
            ke_early = max(ke_early, r.diag[6])
    bins = np.linspace(0.0, H, 11)
    acc = np.zeros(10)
    nsamp = 0
    vmax = rms_max = ke_late = 0.0
    while r.diag[14] < 10 * period:
        r.dual_step(4)
        band = (r.x[:, 1] > 0.2 * H) & (r.x[:, 1] < 0.8 * H)
        rms_max = max(rms_max, math.sqrt((r.v[band] ** 2).sum(1).mean()))
        ke_late = max(ke_late, r.diag[6])
        y = r.x[:, 1]
        p = np.maximum(0.0, c0 ** 2 * (r.rho - 1000.0))
        which = np.digitize(y, bins) - 1
        ok = (which >= 0) & (which < 10)
        acc += np.bincount(which[ok], weights=p[ok], minlength=10)[:10] / np.maximum(
            np.bincount(which[ok], minlength=10)[:10], 1)
        nsamp += 1
        vmax = max(vmax, r.diag[0])
    mean_p = acc / nsamp
    mid = 0.5 * (bins[1:] + bins[:-1])
    hydro = 1000.0 * 9.81 * (H - mid)
    band = (mid > 0.2 * H) & (mid < 0.8 * H)
    err = np.abs(mean_p - hydro)[band].max() / (1000.0 * 9.81 * H)
    assert err < 0.05, (err, mean_p, hydro)
    # the uncompressed start rings acoustically at g H / c0 ~ 0.071 sqrt(gH);
    # the Riemann dissipation acts on compression only, so the ringing is
    # bounded rather than damped: the bulk stays at that scale and the
    # kinetic energy does not grow beyond twice that of the first period
    sq = math.sqrt(9.81 * H)
    assert rms_max < 0.08 * sq, rms_max / sq
    assert ke_late < 2.0 * ke_early, (ke_late, ke_early)
    assert vmax < 0.2 * sq, vmax / sq


def test_dam_break_front_below_shallow_water_bound():
    case = dambreak.make_case("c1_2d")
    r = O.OracleSim.from_case(case)
    r.dual_prime()
    while r.diag[14] < 0.37:
        r.dual_step(10)
    t = r.diag[14]
    H = case.instances[0].height
    front = r.x[:, 0].max()
    assert 1.5 < front < 1.0 + 2 * math.sqrt(9.81 * H) * t
    assert r.diag[11] == 0


def test_determinism_across_thread_counts():
    code = (
        "import numpy as np, dambreak; from oracle import oracle as O;"
        "c=dambreak.make_case('tiny_3d'); s=O.OracleSim.from_case(c); s.dual_prime(); s.dual_step(3);"
        "import sys; sys.stdout.write(s.by_id(s.x).tobytes().hex()[:4000] + s.by_id(s.rho).tobytes().hex())"
    )
    outs = []
    for th in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=th, PYTHONPATH=ROOT)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout)
    assert outs[0] == outs[1] == outs[2]
