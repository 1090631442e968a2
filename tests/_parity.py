"""Helpers shared by the GPU parity tests: run the HIP path and the CPU
reference on the same seeded inputs and compare them by particle id."""
import numpy as np

import dambreak
from oracle import oracle as O


def by_id(arr, ids):
    out = np.empty_like(arr)
    out[ids] = arr
    return out


def gpu_instance_view(sim, h, b):
    """Per-instance host arrays of a Simulation, ids and keys made local."""
    f0, f1 = sim.fluid_offset[b], sim.fluid_offset[b + 1]
    w0, w1 = sim.wall_offset[b], sim.wall_offset[b + 1]
    lo, nc, base = sim.grid(b)
    ncells = nc[0] * nc[1] * nc[2]
    ids = h["id"][f0:f1] - f0
    perm = h["perm"][f0:f1] - f0
    return {
        "ids": ids,
        "key": h["key"][f0:f1] - base,
        "perm": perm,
        "sorted_ids": ids[perm],
        "cell_start": h["cell_start"][base:base + ncells + 1] - f0,
        "wall_start": h["wall_start"][base:base + ncells + 1] - w0,
        "wall_perm": h["wall_perm"][w0:w1] - w0,
        "x": by_id(h["x"][f0:f1], ids), "v": by_id(h["v"][f0:f1], ids),
        "a": by_id(h["a"][f0:f1], ids), "rho": by_id(h["rho"][f0:f1], ids),
        "count": by_id(h["count"][f0:f1], ids),
        "dt": h["dt"][b], "diag": h["diag"][b],
        "ncell": nc,
    }


def oracle_view(o):
    return {
        "key": o.key.copy(), "perm": o.perm.copy(), "sorted_ids": o.sorted_ids(),
        "cell_start": o.start.copy(), "wall_start": o.wstart.copy(),
        "wall_perm": o.wperm[:o.nw].copy(),
        "x": o.by_id(o.x), "v": o.by_id(o.v), "a": o.by_id(o.a), "rho": o.by_id(o.rho),
        "count": o.by_id(o.count), "dt": o.dt[0], "diag": o.diag.copy(),
    }


def errors(g, r, x0, rho0=1000.0):
    """Relative errors as defined for the parity gates: density per particle
    over rho0, velocity and acceleration norm-wise, position over the largest
    displacement from the initial state."""
    e = {"rho": float(np.abs(g["rho"] - r["rho"]).max() / rho0)}
    vm = np.abs(r["v"]).max()
    e["v"] = float(np.abs(g["v"] - r["v"]).max() / vm) if vm > 0 else float(np.abs(g["v"]).max())
    am = np.abs(r["a"]).max()
    e["a"] = float(np.abs(g["a"] - r["a"]).max() / am)
    dm = np.abs(r["x"] - x0).max()
    dx = np.abs(g["x"] - r["x"]).max()
    e["x"] = float(dx / dm) if dm > 0 else float(dx)
    # the same with the FP64 rounding of the absolute positions taken out:
    # after one step the displacement is ~1e-8 m while |x| ~ 1 m rounds at ~1e-16
    slack = 8 * np.finfo(np.float64).eps * np.abs(r["x"]).max()
    e["x_beyond_rounding"] = float(max(dx - slack, 0.0) / dm) if dm > 0 else float(max(dx - slack, 0.0))
    e["dt"] = float(abs(g["dt"] - r["dt"]) / r["dt"])
    return e


# The method's gates (relative errors of density, velocity and position on
# the probe set): 1e-5 after one step, 1e-3 after 100 steps.  The mixed path
# is held to them; the FP64 path to far tighter bounds in each test.
GATE_1_STEP = 1e-5
GATE_100_STEPS = 1e-3


def total_energy(x, v, rho, mass, c0, g, rho0=1000.0):
    """Kinetic + potential + internal energy of one instance's fluid state
    (x, v: (n, dim); internal energy of the clipped equation of state,
    m c0^2 (ln(rho/rho0) + rho0/rho - 1) for rho > rho0), summed on the host in
    one fixed order so that two states differ only by their values."""
    dim = x.shape[1]
    ke = 0.5 * mass * np.sum(v * v, axis=1)
    pe = -mass * (x @ np.asarray(g, dtype=np.float64)[:dim])
    ie = np.where(rho > rho0, mass * c0 * c0 * (np.log(rho / rho0) + rho0 / rho - 1.0), 0.0)
    return float(np.sum(ke + pe + ie)), float(np.sum(ke))


def energy_error(g, r, mass, c0, gvec, rho0=1000.0):
    """|E_G - E_ref| / KE_ref for two views of the same instance."""
    eg, _ = total_energy(g["x"], g["v"], g["rho"], mass, c0, gvec, rho0)
    er, ke = total_energy(r["x"], r["v"], r["rho"], mass, c0, gvec, rho0)
    return abs(eg - er) / ke if ke > 0 else abs(eg - er)


def integer_mismatches(g, r):
    out = {}
    for k in ("key", "perm", "sorted_ids", "cell_start", "wall_start", "wall_perm", "count"):
        out[k] = int(np.count_nonzero(np.asarray(g[k]) != np.asarray(r[k]))) if \
            np.shape(g[k]) == np.shape(r[k]) else -1
    return out


def oracles_for(case, **kw):
    return [O.OracleSim.from_case(case, b, **kw) for b in range(len(case.instances))]


def make_case(name):
    return dambreak.make_case(name)


def _bound(refs):
    # the largest drift bound of the next step over the instances
    return max(r.dt[0] * (r.diag[0] + 0.5 * r.dt[0] * r.diag[1]) for r in refs)


class BuildPlan:
    """The documented rebuild rule, applied to the reference's reductions."""

    def __init__(self, skin):
        self.skin = skin
        self.total = 0.0
        self.builds = 0
        self.built = True          # the prime builds
        self.close_calls = 0

    def after_step(self, refs):
        nxt = _bound(refs)
        if self.built:
            self.builds += 1
        since = (0.0 if self.built else self.total) + nxt
        lim = self.skin * (1.0 - 1e-4)
        if abs(2.0 * since - lim) <= 1e-9 * lim:
            self.close_calls += 1
        rebuild = not (2.0 * since < lim)
        self.total = 0.0 if rebuild else since
        self.built = rebuild


class DualBuildPlan:
    """The exact rebuild rule of the dual scheme with a skin, applied to the
    reference's positions: after an advection step, the next one rebuilds
    when twice the largest distance of a particle from its position at the
    last build reaches skin (1 - 1e-4).  Start it right after the prime."""

    def __init__(self, skin, refs):
        import numpy as np
        self.np = np
        self.skin = skin
        self.xb = [r.by_id(r.x).copy() for r in refs]
        self.builds = 1            # the prime builds
        self.pending = False
        self.close_calls = 0

    def after_step(self, refs):
        np = self.np
        if self.pending:
            self.builds += 1
        x = [r.by_id(r.x) for r in refs]
        D = max((float(np.sqrt(((xi - xb) ** 2).sum(1)).max()) if len(xi) else 0.0)
                for xi, xb in zip(x, self.xb))
        lim = self.skin * (1.0 - 1e-4)
        # the device's positions differ from these by summation rounding
        if abs(2.0 * D - lim) <= 1e-6 * lim:
            self.close_calls += 1
        self.pending = not (2.0 * D < lim)
        if self.pending:
            self.xb = [xi.copy() for xi in x]


def tiled_morton_key(cx, cy, cz, ncell, dim):
    """Cell key of the tiled Morton order as documented for SPH_KEYS_MORTON_TILES:
    tiles of 8^d cells in row-major order, the cells of a tile on the Morton
    curve (bit b of x, y, z at bit d*b, d*b+1, d*b+2).  Vectorised over numpy
    integer arrays."""
    import numpy as np
    cx, cy, cz = (np.asarray(a, dtype=np.int64) for a in (cx, cy, cz))
    ntx, nty = (ncell[0] + 7) // 8, (ncell[1] + 7) // 8
    tile = (cx >> 3) + ntx * ((cy >> 3) + nty * (cz >> 3))
    m = np.zeros_like(cx)
    for b in range(3):
        m |= ((cx >> b) & 1) << (dim * b)
        m |= ((cy >> b) & 1) << (dim * b + 1)
        if dim == 3:
            m |= ((cz >> b) & 1) << (dim * b + 2)
    return (tile << (3 * dim)) | m
