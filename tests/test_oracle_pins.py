"""Pins of the FP64 CPU reference against facts fixed by mathematics.

Each test checks the reference against something other than itself: a closed
form, an invariant, a special case that reduces to a textbook or library
routine, or brute force on tiny inputs.  None of these needs a GPU.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest
from scipy import integrate

import dambreak
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lattice(dim, n, dx, jitter=0.0, seed=0):
    axes = [np.arange(n) for _ in range(dim)]
    g = np.meshgrid(*axes, indexing="ij")
    x = np.stack([gi.reshape(-1) for gi in g], 1).astype(np.float64)
    x = (x + 0.5) * dx
    if jitter:
        x += np.random.default_rng(seed).uniform(-jitter * dx, jitter * dx, x.shape)
    return x


def _sim(dim, x, dx, box, walls=None, **kw):
    h = 1.3 * dx
    if walls is None:
        walls = np.zeros((0, dim))
    kw.setdefault("c0", 20.0)
    kw.setdefault("reorder_every", 0)
    return O.OracleSim(dim, dx, h, (0.0,) * dim, box, x, walls, **kw)


# ---------------------------------------------------------------------------
# Kernel (Wendland C2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_unit_integral(dim):
    h = 0.013
    f = (lambda r: O.W(2, h, r) * 2 * math.pi * r) if dim == 2 else \
        (lambda r: O.W(3, h, r) * 4 * math.pi * r * r)
    val, err = integrate.quad(f, 0.0, 2 * h, epsabs=1e-14, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_gradient_is_derivative(dim):
    h = 0.02
    for q in (0.1, 0.5, 0.77, 1.0, 1.3, 1.7, 1.95):
        r = q * h
        d = 1e-7 * h
        dWdr = (O.W(dim, h, r + d) - O.W(dim, h, r - d)) / (2 * d)
        assert O.F(dim, h, r) * r == pytest.approx(dWdr, rel=1e-6)
    assert O.W(dim, h, 2 * h) == 0.0 and O.F(dim, h, 2 * h) == 0.0
    assert O.W(dim, h, 3 * h) == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_sigma0_is_riemann_sum_of_unit_integral(dim):
    # the lattice sum of W tends to 1/dx^d as h/dx grows (quadrature of a unit integral)
    dx = 1.0
    for ratio, tol in ((2.0, 2e-3), (3.0, 2e-4), (4.0, 5e-5)):
        s = O.sigma0(dim, dx, ratio * dx)
        assert abs(s * dx ** dim - 1.0) < tol
    # at h = 1.3 dx the lattice over-counts by about 1 %: the summation density
    # is normalised by sigma0 rather than by 1/dx^d
    s = O.sigma0(dim, 0.01, 0.013) * 0.01 ** dim
    assert 1.005 < s < 1.015


@pytest.mark.parametrize("dim,want", [(2, 1.010473152107087), (3, 1.009500783784800)])
def test_sigma0_lattice_shell_closed_form(dim, want):
    # sigma0 dx^d at h = 1.3 dx as a finite sum over lattice shells |k|^2 = n < 6.76:
    # a_d dx^d sum_n r_d(n) w(sqrt(n) / 1.3), w(q) = (1 - q/2)^4 (2q + 1), with the
    # shell counts r_d(n) of tests/golden/lattice_shells.txt; the literal values are
    # this sum written out (2D: shells 0, 1, 2, 4, 5; 3D: 0..6)
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "lattice_shells.txt"))
    col = 1 if dim == 2 else 2
    a = 7.0 / (4.0 * math.pi * 1.3 ** 2) if dim == 2 else 21.0 / (16.0 * math.pi * 1.3 ** 3)
    shell_sum = 0.0
    for r in rows:
        q = math.sqrt(r[0]) / 1.3
        if q < 2.0:
            shell_sum += r[col] * (1.0 - q / 2.0) ** 4 * (2.0 * q + 1.0)
    assert a * shell_sum == pytest.approx(want, rel=1e-14)
    for dx in (1.0, 0.01, 0.0065):
        assert O.sigma0(dim, dx, 1.3 * dx) * dx ** dim == pytest.approx(want, rel=1e-13)


# ---------------------------------------------------------------------------
# Cell list, sort, neighbour set
# ---------------------------------------------------------------------------

def _shells(dim):
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "lattice_shells.txt"))
    col = 1 if dim == 2 else 2
    return {int(r[0]): int(r[col]) for r in rows}


@pytest.mark.parametrize("dim", [2, 3])
def test_interior_lattice_neighbour_count(dim):
    shells = _shells(dim)
    expected = sum(shells[n] for n in range(1, 7))   # |k|^2 < (2*1.3)^2 = 6.76
    assert expected == (20 if dim == 2 else 80)
    n = 16 if dim == 2 else 10
    dx = 0.01
    x = _lattice(dim, n, dx, jitter=1e-4, seed=3)
    s = _sim(dim, x, dx, (n * dx,) * dim)
    s.keys(); s.sort(); s.density(0.0)
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 3) & (idx < n - 3), axis=1)
    assert interior.sum() > 0
    assert np.all(s.count[interior] == expected)


def _brute_counts(x, xw, cut2):
    """O(N^2) neighbour counts with r^2 summed left to right (numpy does not fuse)."""
    def d2(a, b):
        s = None
        for k in range(a.shape[1]):
            d = a[:, None, k] - b[None, :, k]
            s = d * d if s is None else s + d * d
        return s
    r2 = d2(x, x)
    np.fill_diagonal(r2, np.inf)
    cnt = (r2 < cut2).sum(1)
    if xw.shape[0]:
        cnt += (d2(x, xw) < cut2).sum(1)
    return cnt


@pytest.mark.parametrize("dim,kind", [(2, "uniform"), (3, "uniform"), (2, "clustered"),
                                      (3, "clustered"), (2, "adversarial"), (3, "adversarial")])
def test_cell_list_matches_brute_force(dim, kind):
    rng = np.random.default_rng(7 + dim)
    dx = 0.02
    L = 0.3 if dim == 2 else 0.16
    h = 1.3 * dx
    if kind == "uniform":
        x = rng.uniform(0, L, (1500 if dim == 2 else 1200, dim))
    elif kind == "clustered":
        c = rng.uniform(0.2 * L, 0.8 * L, (6, dim))
        x = np.concatenate([c[k] + rng.normal(0, 0.02 * L, (250, dim)) for k in range(6)])
        x = np.clip(x, 0, L - 1e-9)
    else:
        # pairs straddling the cutoff r = 2h (1 +- 1e-9) in random directions
        base = rng.uniform(0.25 * L, 0.75 * L, (200, dim))
        u = rng.normal(size=(200, dim))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        fac = np.where(rng.random(200) < 0.5, 1 - 1e-9, 1 + 1e-9)
        x = np.concatenate([base, base + u * (2 * h * fac)[:, None]])
    xw = rng.uniform(-2.5 * dx, 0.0, (80, dim))   # a wall slab below the domain
    s = O.OracleSim(dim, dx, h, (0.0,) * dim, (L,) * dim, x, xw, c0=10.0, reorder_every=0)
    s.keys(); s.sort(); s.density(0.0)
    brute = _brute_counts(s.x, s.xw, (2 * h) * (2 * h))
    assert np.array_equal(s.count, brute)


def test_stable_sort_matches_numpy():
    rng = np.random.default_rng(11)
    for n, nc in ((1, 5), (1000, 7), (5000, 4000), (20000, 300)):
        key = rng.integers(0, nc, n).astype(np.int32)
        perm = np.zeros(n, np.int32)
        start = np.zeros(nc + 1, np.int32)
        O.lib().or_sort(n, key.ctypes.data_as(O._ip), nc, perm.ctypes.data_as(O._ip),
                        start.ctypes.data_as(O._ip))
        assert np.array_equal(perm, np.argsort(key, kind="stable"))
        assert np.array_equal(start, np.searchsorted(np.sort(key), np.arange(nc + 1), side="left"))


def test_keys_of_cell_centres_and_clamping():
    dx = 0.01
    x = np.array([[0.05, 0.05]])
    s = _sim(2, x, dx, (0.2, 0.1))
    lo = np.array(s.lo[:2])
    ncx, ncy = s.ncell[0], s.ncell[1]
    cs = 2 * 1.3 * dx
    pts = []
    want = []
    for j in range(ncy):
        for i in range(ncx):
            pts.append(lo + (np.array([i, j]) + 0.5) * cs)
            want.append(i + ncx * j)
    pts = np.array(pts)
    key = np.zeros(len(pts), np.int32)
    cl = O.lib().or_keys(O.C.byref(s.p), len(pts), pts.ctypes.data_as(O._dp), key.ctypes.data_as(O._ip))
    assert cl == 0 and np.array_equal(key, want)
    out = np.array([[lo[0] - 1.0, lo[1] + 0.5 * cs], [lo[0] + 1e3, lo[1] - 5.0], [np.nan, 0.05]])
    key = np.zeros(3, np.int32)
    cl = O.lib().or_keys(O.C.byref(s.p), 3, out.ctypes.data_as(O._dp), key.ctypes.data_as(O._ip))
    assert cl == 3
    iy = int(np.floor((0.05 - lo[1]) / cs))
    assert list(key) == [0, ncx - 1, ncx * iy]


# ---------------------------------------------------------------------------
# Sweeps: invariants and closed forms
# ---------------------------------------------------------------------------

def _blob(dim, n, seed):
    rng = np.random.default_rng(seed)
    dx = 0.02
    L = 0.2
    x = rng.uniform(0.3 * L, 0.7 * L, (n, dim))
    v = rng.normal(0, 0.5, (n, dim))
    rho = rng.uniform(995.0, 1010.0, n)
    return dx, L, x, v, rho


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_net_pairwise_momentum(dim):
    dx, L, x, v, rho = _blob(dim, 400, 5)
    s = _sim(dim, x, dx, (L,) * dim, v=v, rho=rho, g=(0.0,) * dim, c0=30.0, alpha=0.5)
    s.keys(); s.sort(); s.density(1e-4); s.forces()
    ma = s.mass * s.a
    assert np.linalg.norm(ma.sum(0)) <= 1e-12 * np.abs(ma).sum()
    assert np.abs(ma).sum() > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_galilean_invariance(dim):
    dx, L, x, v, rho = _blob(dim, 300, 9)
    U = np.array([3.0, -2.0, 1.0])[:dim]
    out = []
    for shift in (np.zeros(dim), U):
        s = _sim(dim, x, dx, (L,) * dim, v=v + shift, rho=rho, c0=30.0, alpha=0.5)
        s.keys(); s.sort(); s.density(1e-4); s.forces()
        out.append((s.rho.copy(), s.a.copy(), s.count.copy()))
    assert np.array_equal(out[0][2], out[1][2])
    assert np.allclose(out[0][0], out[1][0], rtol=1e-13, atol=0)
    scale = np.abs(out[0][1]).max()
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-10 * scale


def test_two_particle_force_closed_form():
    dim, dx = 2, 0.02
    h = 1.3 * dx
    x = np.array([[0.1, 0.1], [0.1 + 0.8 * h * 0.6, 0.1 + 0.8 * h * 0.8]])
    s = _sim(dim, x, dx, (0.2, 0.2), g=(0.0, 0.0), alpha=0.0)
    s.keys(); s.sort()
    s.rho[:] = [1002.0, 1005.0]
    s.P[:] = [300.0 / 1002.0 ** 2, 500.0 / 1005.0 ** 2]
    s.forces()
    r12 = x[0] - x[1]
    r = np.linalg.norm(r12)
    # gradient of W at particle 1 by central differences of W (pinned above)
    e = 1e-7 * h
    grad = np.array([(O.W(2, h, np.linalg.norm(r12 + e * u)) - O.W(2, h, np.linalg.norm(r12 - e * u))) / (2 * e)
                     for u in np.eye(2)])
    want = -s.mass * (s.P[0] + s.P[1]) * grad
    assert np.allclose(s.a[0], want, rtol=1e-6)
    assert np.allclose(s.a[0], -s.a[1], rtol=1e-14)
    assert np.dot(s.a[0], r12) > 0          # positive pressure repels


def test_artificial_viscosity_acts_only_on_approach():
    dim, dx = 2, 0.02
    h = 1.3 * dx
    x = np.array([[0.1, 0.1], [0.1 + 1.1 * h, 0.1]])
    res = {}
    for name, v in (("approach", [[1.0, 0], [-1.0, 0]]), ("recede", [[-1.0, 0], [1.0, 0]]),
                    ("still", [[0, 0], [0, 0]])):
        s = _sim(dim, x, dx, (0.2, 0.2), v=np.array(v, float), g=(0.0, 0.0), alpha=1.0)
        s.keys(); s.sort()
        s.rho[:] = 1000.0
        s.P[:] = 0.0
        s.forces()
        res[name] = s.a.copy()
    assert np.all(res["recede"] == 0.0) and np.all(res["still"] == 0.0)
    # approaching pair: the viscous force decelerates the relative motion
    rel_v = np.array([2.0, 0.0])
    assert np.dot(res["approach"][0] - res["approach"][1], rel_v) < 0


def _fd_grad_W(dim, h, r12):
    """Gradient of W at r12 by central differences of W (pinned above)."""
    e = 1e-7 * h
    return np.array([(O.W(dim, h, np.linalg.norm(r12 + e * u)) - O.W(dim, h, np.linalg.norm(r12 - e * u)))
                     / (2 * e) for u in np.eye(dim)])


def test_viscosity_magnitude_two_particles():
    # an approaching pair with unequal densities and pressures: the Monaghan
    # term Pi = -alpha c0 h (v12.r12) / (rhobar (r^2 + eps h^2)), rhobar the
    # mean density, enters a_1 = -m (P_1 + P_2 + Pi) grad_1 W beside the
    # pressure terms.  Every factor is set to a value that a slip would move:
    # alpha = 0.7, c0 = 20, h = 0.026, eps = 0.01, rho = 1000 and 1100
    dim, dx = 2, 0.02
    h = 1.3 * dx
    x = np.array([[0.1, 0.1], [0.1 + 0.9 * h * 0.6, 0.1 + 0.9 * h * 0.8]])
    v = np.array([[0.4, 0.9], [-0.5, -0.2]])
    s = _sim(dim, x, dx, (0.2, 0.2), v=v, g=(0.0, 0.0), alpha=0.7, c0=20.0)
    s.keys(); s.sort()
    rho = np.array([1000.0, 1100.0])
    p = np.array([150.0, 420.0])
    s.rho[:] = rho
    s.P[:] = p / rho ** 2
    s.forces()
    r12 = x[0] - x[1]
    v12 = v[0] - v[1]
    vr = float(v12 @ r12)
    assert vr < 0.0                      # approaching
    r2 = float(r12 @ r12)
    Pi = -0.7 * 20.0 * h * vr / (1050.0 * (r2 + 0.01 * h * h))
    grad = _fd_grad_W(dim, h, r12)
    want = -s.mass * (p[0] / 1000.0 ** 2 + p[1] / 1100.0 ** 2 + Pi) * grad
    assert np.allclose(s.a[0], want, rtol=1e-6, atol=0)
    # the viscous part is a sizeable share of the force (the pin has teeth)
    assert Pi > 0.5 * (p[0] / 1000.0 ** 2 + p[1] / 1100.0 ** 2)
    assert np.allclose(s.a[1], -s.a[0] * 1.0, rtol=1e-13)


def test_viscosity_magnitude_at_a_wall():
    # a fluid particle approaching a fixed wall particle: the wall mirrors the
    # target (rho_j = rho_i, v_j = 0) and carries the hydrostatic pressure
    # p_j = max(0, p_i + rho_i g.(x_j - x_i)); here g = (0, -9.81) and the
    # wall sits below, so p_j = p_i + rho_i 9.81 (y_i - y_j)
    dim, dx = 2, 0.02
    h = 1.3 * dx
    xi = np.array([[0.1, 0.1]])
    xw = np.array([[0.1 - 0.5 * h, 0.1 - 0.7 * h]])
    v = np.array([[0.3, -1.2]])
    s = _sim(dim, xi, dx, (0.2, 0.2), walls=xw, v=v, alpha=0.7, c0=20.0)
    s.keys(); s.sort()
    rho_i, p_i = 1010.0, 20.0 ** 2 * 10.0
    s.rho[:] = rho_i
    s.P[:] = p_i / rho_i ** 2
    s.forces()
    r = xi[0] - xw[0]
    vr = float(v[0] @ r)
    assert vr < 0.0
    p_j = p_i + rho_i * 9.81 * (xi[0, 1] - xw[0, 1])
    Pi = -0.7 * 20.0 * h * vr / (rho_i * (float(r @ r) + 0.01 * h * h))
    grad = _fd_grad_W(dim, h, r)
    want = np.array([0.0, -9.81]) - s.mass * (p_i / rho_i ** 2 + p_j / rho_i ** 2 + Pi) * grad
    assert np.allclose(s.a[0], want, rtol=1e-6, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_cfl_time_step_closed_form(dim):
    # two far-apart particles (no neighbours), one moving, after the prime:
    # max|v| = that speed, max|a| = |g|, and
    # dt = min(0.25 h / (c0 + max|v|), 0.25 sqrt(h / max|a|)), per branch:
    #   dx = 0.02, h = 0.026, c0 = 15, 2 m/s, g = 9.81:  0.25 * 0.026 / 17 = 3.823529411764706e-4
    #   c0 = 1, 0.2 m/s, g = 100:  0.25 * sqrt(0.026 / 100) = 4.031128874149275e-3
    #   (against 0.25 * 0.026 / 1.2 = 5.4e-3 on the acoustic branch)
    dx = 0.02
    x = np.full((2, dim), 0.2)
    x[1, 0] = 0.8
    v = np.zeros((2, dim))
    v[0, 0] = 2.0
    s = _sim(dim, x, dx, (1.0,) * dim, v=v, c0=15.0)
    s.prime()
    assert s.dt[0] == pytest.approx(3.823529411764706e-4, rel=1e-15)
    g = [0.0] * dim
    g[-1] = -100.0
    v[0, 0] = 0.2
    s = _sim(dim, x, dx, (1.0,) * dim, v=v, c0=1.0, g=tuple(g))
    s.prime()
    assert s.dt[0] == pytest.approx(4.031128874149275e-3, rel=1e-15)
    # one step later both particles fell for dt: max|v| = |(0.2, -100 dt)|
    dt0 = s.dt[0]
    s.step(1)
    vmax = math.hypot(0.2, 100.0 * dt0)
    want = min(0.25 * 0.026 / (1.0 + vmax), 0.25 * math.sqrt(0.026 / 100.0))
    assert s.dt[0] == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_pressure_gives_gravity(dim):
    n = 14 if dim == 2 else 9
    dx = 0.01
    x = _lattice(dim, n, dx)
    s = _sim(dim, x, dx, (n * dx,) * dim, alpha=0.0)
    s.keys(); s.sort()
    s.rho[:] = 1003.0
    s.P[:] = 2500.0 / 1003.0 ** 2
    s.forces()
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 3) & (idx < n - 3), axis=1)
    g = np.zeros(dim); g[-1] = -9.81
    assert np.abs(s.a[interior] - g).max() < 1e-9


def test_linear_pressure_field_gradient():
    # a = -grad(p)/rho for p linear in y, up to the lattice discretisation error
    dim, n, dx = 2, 30, 0.02
    x = _lattice(dim, n, dx)
    s = _sim(dim, x, dx, (n * dx,) * dim, g=(0.0, 0.0), alpha=0.0)
    s.keys(); s.sort()
    kappa, rho = 1000.0, 1000.0
    s.rho[:] = rho
    s.P[:] = (2000.0 + kappa * x[:, 1]) / rho ** 2
    s.forces()
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 4) & (idx < n - 4), axis=1)
    ay = s.a[interior, 1]
    assert np.allclose(ay, ay.mean(), rtol=1e-9)
    assert abs(ay.mean() / (-kappa / rho) - 1.0) < 0.05
    assert np.abs(s.a[interior, 0]).max() < 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_continuity_of_linear_compression(dim):
    # v = -beta x: div v = -d beta, so Drho = rho0 d beta up to lattice error
    n = 24 if dim == 2 else 12
    dx, beta = 0.01, 2.0
    x = _lattice(dim, n, dx)
    c = x.mean(0)
    v = -beta * (x - c)
    s = _sim(dim, x, dx, (n * dx,) * dim, v=v)
    s.keys(); s.sort()
    dt = 1e-6
    s.density(dt)
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 3) & (idx < n - 3), axis=1)
    rho_sum = s.mass * O.sigma0(dim, dx, 1.3 * dx)          # = rho0 on the perfect lattice
    assert np.allclose(rho_sum, 1000.0, rtol=1e-12)
    # rho* = rho0 + dt Drho > rho_sum = rho0 in the interior, so the update keeps
    # the excess scaled by rho0/rho* (a relative change of dt Drho / rho0 ~ 1e-5)
    drho = (s.rho[interior] - 1000.0) / dt
    ratio = drho / (1000.0 * dim * beta)
    assert np.all(np.abs(ratio - 1.0) < 0.05)


def test_density_update_branches():
    dim, dx = 2, 0.02
    n = 12
    x = _lattice(dim, n, dx)
    s = _sim(dim, x, dx, (n * dx,) * dim)
    s.keys(); s.sort()
    # interior: rho_sum = rho0 >= rho* = 990 -> summation density
    s.rho[:] = 990.0
    s.density(0.0)
    idx = np.round(x / dx - 0.5).astype(int)
    interior = np.all((idx >= 3) & (idx < n - 3), axis=1)
    corner = np.all(idx == 0, axis=1)
    assert np.allclose(s.rho[interior], 1000.0, rtol=1e-13)
    # corner: rho_sum << rho* = 990 -> rho - rho0 = (rho_sum/rho*)(rho* - rho0)
    rho_sum_corner = None
    s2 = _sim(dim, x, dx, (n * dx,) * dim)
    s2.keys(); s2.sort()
    s2.rho[:] = 1e9          # rho* huge: rho = rho_sum + (rho*-rho_sum) rho0/rho* ~ rho_sum + rho0
    s2.density(0.0)
    rho_sum_corner = s2.rho[corner][0] - 1000.0 * (1.0 - (s2.rho[corner][0] - 1000.0) / 1e9)
    want = rho_sum_corner + (990.0 - rho_sum_corner) * 1000.0 / 990.0
    assert s.rho[corner][0] == pytest.approx(want, rel=1e-9)
    # no tension: pressures are never negative
    assert np.all(s.P >= 0.0)


# ---------------------------------------------------------------------------
# Integrator, walls, gravity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_isolated_particle_free_fall(dim):
    dx = 0.02
    x0 = np.full((1, dim), 0.5)
    v0 = np.zeros((1, dim)); v0[0, 0] = 0.3
    s = _sim(dim, x0, dx, (1.0,) * dim, v=v0, c0=15.0)
    s.prime()
    s.step(200)
    t = s.diag[14]
    g = np.zeros(dim); g[-1] = -9.81
    want_x = x0[0] + v0[0] * t + 0.5 * g * t * t
    want_v = v0[0] + g * t
    assert s.rho[0] == 1000.0
    assert np.allclose(s.x[0], want_x, rtol=0, atol=1e-12)
    assert np.allclose(s.v[0], want_v, rtol=0, atol=1e-12)
    assert s.count[0] == 0


@pytest.mark.slow
def test_hydrostatic_column_time_average():
    case = dambreak.make_case("hydrostatic_2d")
    inst = case.instances[0]
    H, c0 = inst.height, inst.c0
    s = O.OracleSim.from_case(case)
    s.prime()
    period = 4 * H / c0
    ke_early = 0.0
    while s.diag[14] < 6 * period:
        s.step(50)
        if s.diag[14] < 3 * period:
            ke_early = max(ke_early, s.diag[6])
    bins = np.linspace(0.0, H, 11)
    acc = np.zeros(10)
    nsamp = 0
    vmax = rms_max = ke_late = 0.0
    while s.diag[14] < 10 * period:
        s.step(20)
        y = s.x[:, 1]
        p = s.P * s.rho ** 2
        which = np.digitize(y, bins) - 1
        ok = (which >= 0) & (which < 10)
        acc += np.bincount(which[ok], weights=p[ok], minlength=10)[:10] / np.maximum(
            np.bincount(which[ok], minlength=10)[:10], 1)
        nsamp += 1
        vmax = max(vmax, s.diag[0])
        band = (y > 0.2 * H) & (y < 0.8 * H)
        rms_max = max(rms_max, math.sqrt((s.v[band] ** 2).sum(1).mean()))
        ke_late = max(ke_late, s.diag[6])
    mean_p = acc / nsamp
    mid = 0.5 * (bins[1:] + bins[:-1])
    hydro = 1000.0 * 9.81 * (H - mid)
    band = (mid > 0.2 * H) & (mid < 0.8 * H)
    err = np.abs(mean_p - hydro)[band].max() / (1000.0 * 9.81 * H)
    assert err < 0.05, (err, mean_p, hydro)
    # the column starts uncompressed (rho = rho0), so it first falls and then
    # rings acoustically with a velocity scale g H / c0 = sqrt(gH) / (10 sqrt 2)
    # ~ 0.071 sqrt(gH); the artificial viscosity damps that ringing: after six
    # periods the bulk moves well below the transient scale, the kinetic
    # energy has decayed, and no surface particle runs away
    sq = math.sqrt(9.81 * H)
    assert rms_max < 0.04 * sq, rms_max / sq
    assert ke_late < 0.5 * ke_early, (ke_late, ke_early)
    assert vmax < 0.2 * sq, vmax / sq
    assert s.diag[11] == 0


def test_dam_break_front_below_shallow_water_bound():
    case = dambreak.make_case("c1_2d")
    s = O.OracleSim.from_case(case)
    s.prime()
    s.step(600)
    t = s.diag[14]
    H = case.instances[0].height
    front = s.x[:, 0].max()
    assert 1.0 < front < 1.0 + 2 * math.sqrt(9.81 * H) * t
    assert s.diag[11] == 0


def test_reorder_schedule_changes_only_rounding():
    case = dambreak.make_case("tiny_2d")
    runs = {}
    for K in (0, 1, 4):
        s = O.OracleSim.from_case(case, reorder_every=K)
        s.prime()
        s.step(12)
        runs[K] = (s.by_id(s.x), s.by_id(s.v), s.by_id(s.rho), s.by_id(s.count), s.dt[0])
    for K in (1, 4):
        assert np.array_equal(runs[0][3], runs[K][3])
        assert np.allclose(runs[0][0], runs[K][0], rtol=0, atol=1e-13)
        assert np.allclose(runs[0][2], runs[K][2], rtol=1e-12)
        assert runs[0][4] == pytest.approx(runs[K][4], rel=1e-12)


def test_energy_bookkeeping_without_viscosity():
    # alpha = 0: kinetic + potential + internal energy is conserved up to the
    # time-discretisation error and the free-surface density relaxation (which
    # is not conservative) over a short run; a sign slip in any energy term
    # would move the balance by the order of the kinetic energy itself
    case = dambreak.make_case("tiny_2d")
    s = O.OracleSim.from_case(case, alpha=0.0, cfl_ac=0.1, cfl_f=0.1)
    s.prime()
    e0 = s.diag[6] + s.diag[7] + s.diag[8]
    s.step(300)
    e1 = s.diag[6] + s.diag[7] + s.diag[8]
    assert s.diag[6] > 0
    assert abs(e1 - e0) < 0.05 * s.diag[6]


def test_determinism_across_thread_counts():
    code = (
        "import numpy as np, dambreak; from oracle import oracle as O;"
        "c=dambreak.make_case('tiny_3d'); s=O.OracleSim.from_case(c); s.prime(); s.step(5);"
        "import sys; sys.stdout.write(s.by_id(s.x).tobytes().hex()[:4000] + s.by_id(s.rho).tobytes().hex())"
    )
    outs = []
    for th in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=th, PYTHONPATH=ROOT)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout)
    assert outs[0] == outs[1] == outs[2]
