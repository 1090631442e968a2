"""Seeded synthetic dam-break workloads (inputs only).

This module builds the initial particle sets that both the HIP path and the CPU
reference consume: fluid blocks on a regular lattice with a tiny seeded jitter,
three layers of fixed wall particles lining a closed box, particle ids, and the
run parameters of each workload.  It holds no part of the SPH method itself: no
kernel function, no neighbour search, no cell grid, no lattice sums.

The paper (Sec. 6) benchmarks 2D and 3D dam breaks without stating sizes; the
shapes below are the workloads this project measures:

* ``c1_2d``      2D column 1.0 x 2.0 m at dx = 0.025 (40 x 80) in a 5 x 3 m tank.
* ``c2_3d``      3D block 1 x 1 x 2 m at dx = 0.01 (2.0 M) in a 4 x 1 x 3 m box.
* ``c3_3d``      the same box at dx = 0.005 (16 M).
* ``c4_batch``   64 independent 2D columns, widths U[0.5, 2.0] m, height 2w,
                 tank 5w x 3w, dx = 0.005 (20 k - 320 k particles each).
* ``c5_3d``      2 x 2 x 2 m block at dx = 0.0065 (308^3) in an 8 x 2 x 3 m box.

Lattice conventions: a box of extent L along an axis holds n = round(L/dx)
lattice cells; particle centres sit at lo + (i + 1/2) dx.  Walls continue the
lattice outward: indices -3..-1 and n..n+2 on every side (top included).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Instance", "Case", "make_case", "dam_break_instance", "probe_ids",
    "CASE_NAMES", "G_MAG", "RHO0",
]

G_MAG = 9.81
RHO0 = 1000.0
ALPHA = 0.1         # artificial-viscosity coefficient of the workloads
EPS = 0.01          # regulariser of the viscosity denominator (times h^2)
CFL_AC = 0.25       # acoustic/advective Courant number
CFL_F = 0.25        # body-force Courant number
H_OVER_DX = 1.3     # smoothing length over lattice spacing
WALL_LAYERS = 3
JITTER = 1e-4       # initial position jitter, in units of dx (uniform +-)


@dataclass
class Instance:
    """One independent dam break.  Arrays are float64, shape (n, dim)."""
    dim: int
    dx: float
    tank_lo: np.ndarray          # (3,) lower corner of the tank interior
    tank_hi: np.ndarray          # (3,) upper corner (lattice aligned)
    fluid: np.ndarray            # (n_fluid, dim) positions, ids 0..n_fluid-1
    wall: np.ndarray             # (n_wall, dim) fixed wall particle centres
    c0: float                    # artificial sound speed 10*sqrt(2 g H)
    height: float                # fluid column height H
    fluid_shape: tuple           # lattice counts of the fluid block
    seed: int

    @property
    def n_fluid(self) -> int:
        return int(self.fluid.shape[0])

    @property
    def n_wall(self) -> int:
        return int(self.wall.shape[0])


@dataclass
class Case:
    """A workload: run parameters plus one or more instances."""
    name: str
    dim: int
    dx: float
    h: float
    rho0: float = RHO0
    gmag: float = G_MAG
    alpha: float = ALPHA
    eps: float = EPS
    cfl_ac: float = CFL_AC
    cfl_f: float = CFL_F
    reorder_every: int = 20
    steps: int = 100
    instances: list = field(default_factory=list)

    @property
    def g(self) -> np.ndarray:
        g = np.zeros(3)
        g[self.dim - 1] = -self.gmag
        return g

    @property
    def n_fluid(self) -> int:
        return sum(i.n_fluid for i in self.instances)

    @property
    def n_wall(self) -> int:
        return sum(i.n_wall for i in self.instances)


def _lattice_count(length: float, dx: float) -> int:
    return int(round(length / dx))


def _fluid_lattice(dim, dx, lo, shape, rng):
    """Fluid centres lo + (i + 1/2) dx, ids x-fastest, plus seeded jitter."""
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    # x fastest: build with indexing='ij' over reversed axes then flip columns
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    pts = np.empty((int(np.prod(shape)), dim), dtype=np.float64)
    for a in range(dim):
        pts[:, a] = grids[dim - 1 - a].reshape(-1)
    del grids
    pts += 0.5
    pts *= dx
    pts += np.asarray(lo[:dim], dtype=np.float64)
    jit = rng.uniform(-JITTER * dx, JITTER * dx, size=pts.shape)
    pts += jit
    return pts


def _wall_shell(dim, dx, lo, n):
    """Centres of the WALL_LAYERS-thick shell around the box [0, n) (lattice)."""
    L = WALL_LAYERS
    out = []
    if dim == 2:
        nx, ny = n[0], n[1]
        for j in range(-L, ny + L):
            if 0 <= j < ny:
                i = np.concatenate([np.arange(-L, 0), np.arange(nx, nx + L)])
            else:
                i = np.arange(-L, nx + L)
            blk = np.empty((i.size, 2))
            blk[:, 0] = i
            blk[:, 1] = j
            out.append(blk)
    else:
        nx, ny, nz = n[0], n[1], n[2]
        full_i = np.arange(-L, nx + L)
        full_j = np.arange(-L, ny + L)
        for k in range(-L, nz + L):
            if 0 <= k < nz:
                # ring: rows j outside [0,ny) are full, rows inside hold the x-frame
                jj, ii = np.meshgrid(full_j, full_i, indexing="ij")
                inside = (jj >= 0) & (jj < ny) & (ii >= 0) & (ii < nx)
                ii = ii[~inside]
                jj = jj[~inside]
            else:
                jj, ii = np.meshgrid(full_j, full_i, indexing="ij")
                ii = ii.reshape(-1)
                jj = jj.reshape(-1)
            blk = np.empty((ii.size, 3))
            blk[:, 0] = ii
            blk[:, 1] = jj
            blk[:, 2] = k
            out.append(blk)
    w = np.concatenate(out, axis=0)
    w += 0.5
    w *= dx
    w += np.asarray(lo[:dim], dtype=np.float64)
    return w


def dam_break_instance(dim, dx, tank, fluid, seed, gmag=G_MAG):
    """Build one dam break.

    tank, fluid: extents (metres) per axis; the fluid block sits in the lower
    corner of the tank.  Both are rounded to whole lattice cells.
    """
    tank_n = [_lattice_count(t, dx) for t in tank]
    fl_n = [_lattice_count(f, dx) for f in fluid]
    lo = np.zeros(3)
    hi = np.zeros(3)
    for a in range(dim):
        hi[a] = tank_n[a] * dx
    rng = np.random.default_rng(seed)
    fl = _fluid_lattice(dim, dx, lo, fl_n, rng)
    wall = _wall_shell(dim, dx, lo, tank_n)
    height = fl_n[dim - 1] * dx
    c0 = 10.0 * math.sqrt(2.0 * gmag * height)
    return Instance(dim=dim, dx=dx, tank_lo=lo, tank_hi=hi, fluid=fl, wall=wall,
                    c0=c0, height=height, fluid_shape=tuple(fl_n), seed=seed)


CASE_NAMES = ("c1_2d", "c2_3d", "c3_3d", "c4_batch", "c5_3d",
              "hydrostatic_2d", "tiny_2d", "tiny_3d", "small_batch")


def make_case(name: str, n_instances: int | None = None) -> Case:
    """Build a named workload (see module docstring)."""
    if name == "c1_2d":
        dx = 0.025
        inst = [dam_break_instance(2, dx, (5.0, 3.0), (1.0, 2.0), 2603)]
        return Case(name, 2, dx, H_OVER_DX * dx, reorder_every=20, steps=100,
                    instances=inst)
    if name in ("c2_3d", "c3_3d"):
        dx = 0.01 if name == "c2_3d" else 0.005
        inst = [dam_break_instance(3, dx, (4.0, 1.0, 3.0), (1.0, 1.0, 2.0), 2603)]
        return Case(name, 3, dx, H_OVER_DX * dx, reorder_every=20, steps=500,
                    instances=inst)
    if name == "c5_3d":
        dx = 0.0065
        inst = [dam_break_instance(3, dx, (8.0, 2.0, 3.0), (2.0, 2.0, 2.0), 2603)]
        return Case(name, 3, dx, H_OVER_DX * dx, reorder_every=50, steps=1000,
                    instances=inst)
    if name == "c4_batch":
        dx = 0.005
        nb = 64 if n_instances is None else n_instances
        widths = np.random.default_rng(11868).uniform(0.5, 2.0, 64)[:nb]
        inst = []
        for b, w in enumerate(widths):
            n = _lattice_count(float(w), dx)
            wq = n * dx
            inst.append(dam_break_instance(2, dx, (5 * wq, 3 * wq), (wq, 2 * wq), 2603 + b))
        return Case(name, 2, dx, H_OVER_DX * dx, reorder_every=20, steps=200,
                    instances=inst)
    if name == "small_batch":
        # a few uneven 2D columns: the batched form at a size the oracle runs fast
        dx = 0.02
        nb = 5 if n_instances is None else n_instances
        widths = np.random.default_rng(11868).uniform(0.2, 0.6, nb)
        inst = []
        for b, w in enumerate(widths):
            n = _lattice_count(float(w), dx)
            wq = n * dx
            inst.append(dam_break_instance(2, dx, (5 * wq, 3 * wq), (wq, 2 * wq), 2603 + b))
        return Case(name, 2, dx, H_OVER_DX * dx, reorder_every=5, steps=20,
                    instances=inst)
    if name == "hydrostatic_2d":
        dx = 0.02
        inst = [dam_break_instance(2, dx, (1.0, 1.5), (1.0, 1.0), 7)]
        return Case(name, 2, dx, H_OVER_DX * dx, reorder_every=20, steps=0,
                    instances=inst)
    if name == "tiny_2d":
        dx = 0.05
        inst = [dam_break_instance(2, dx, (1.5, 1.0), (0.5, 0.75), 2603)]
        return Case(name, 2, dx, H_OVER_DX * dx, reorder_every=3, steps=10,
                    instances=inst)
    if name == "tiny_3d":
        dx = 0.05
        inst = [dam_break_instance(3, dx, (1.0, 0.5, 0.75), (0.3, 0.5, 0.5), 2603)]
        return Case(name, 3, dx, H_OVER_DX * dx, reorder_every=3, steps=10,
                    instances=inst)
    raise KeyError(f"unknown case {name!r}; known: {CASE_NAMES}")


def probe_ids(inst: Instance, count: int = 10000) -> np.ndarray:
    """Fluid ids compared on large cases: a seeded sample plus the block corners.

    All fluid ids when the instance has at most ``count`` particles.
    """
    n = inst.n_fluid
    if n <= count:
        return np.arange(n, dtype=np.int64)
    sample = np.random.default_rng(1).choice(n, count, replace=False)
    shape = inst.fluid_shape
    corners = []
    dim = inst.dim
    for c in range(1 << dim):
        idx = [(shape[a] - 1) if (c >> a) & 1 else 0 for a in range(dim)]
        lin = 0
        stride = 1
        for a in range(dim):
            lin += idx[a] * stride
            stride *= shape[a]
        corners.append(lin)
    return np.unique(np.concatenate([sample, np.asarray(corners)])).astype(np.int64)
