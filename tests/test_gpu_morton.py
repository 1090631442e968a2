"""Tiled Morton cell keys (SPH_KEYS_MORTON_TILES).  The sort order and the
cell tables change; what a step computes does not.  Keys, the sort and the
start table are checked bit for bit against the documented mapping applied to
the positions; the state against the FP64 CPU reference (which uses row-major
cells), with bit-exact neighbour counts."""
import numpy as np
import pytest

import dambreak
from _parity import (GATE_100_STEPS, BuildPlan, errors, gpu_instance_view, oracle_view, oracles_for,
                     tiled_morton_key)

pytestmark = pytest.mark.gpu


def _sim(case, **kw):
    from paper_2603_11868_amd import sph
    return sph.Simulation(case, key_order="morton", **kw)


def _expected_keys(sim, case, x):
    """Global keys of storage-order positions x (N x dim): cells as the
    library computes them (subtract, multiply by 1/cs, floor, clamp)."""
    out = np.empty(len(x), dtype=np.int64)
    inv_cs = 1.0 / sim.info.cell_size
    for b in range(sim.B):
        f0, f1 = sim.fluid_offset[b], sim.fluid_offset[b + 1]
        lo, nc, base = sim.grid(b)
        c = [np.zeros(f1 - f0, dtype=np.int64) for _ in range(3)]
        for a in range(case.dim):
            v = np.floor((x[f0:f1, a] - lo[a]) * inv_cs)
            c[a] = np.clip(v, 0, nc[a] - 1).astype(np.int64)
        out[f0:f1] = base + tiled_morton_key(c[0], c[1], c[2], nc, case.dim)
    return out


@pytest.mark.parametrize("name", ["c1_2d", "tiny_3d", "small_batch"])
def test_morton_keys_sort_and_tables_at_prime(name):
    case = dambreak.make_case(name)
    sim = _sim(case)
    refs = oracles_for(case)
    sim.prime()
    for r in refs:
        r.prime()
    h = sim.host()
    key = _expected_keys(sim, case, h["x"])
    assert np.array_equal(h["key"].astype(np.int64), key)
    perm = np.argsort(key, kind="stable")
    assert np.array_equal(h["perm"], perm)
    start = np.searchsorted(np.sort(key), np.arange(sim.C + 1), side="left")
    assert np.array_equal(h["cell_start"].astype(np.int64), start)
    for b, r in enumerate(refs):
        g = gpu_instance_view(sim, h, b)
        rv = oracle_view(r)
        assert np.array_equal(g["count"], rv["count"])
        assert np.abs(g["rho"] - rv["rho"]).max() <= 1e-13 * case.rho0
        assert np.abs(g["a"] - rv["a"]).max() <= 1e-10 * np.abs(rv["a"]).max()
    sim.close()


@pytest.mark.parametrize("name,skin_h", [("c1_2d", 0.0), ("tiny_3d", 0.0), ("c1_2d", 0.01), ("small_batch", 0.005)])
def test_morton_parity_100_steps_fp64(name, skin_h):
    case = dambreak.make_case(name)
    sim = _sim(case, skin=skin_h * case.h)
    refs = oracles_for(case)
    sim.prime()
    for r in refs:
        r.prime()
    plan = BuildPlan(skin_h * case.h) if skin_h else None
    if plan:
        plan.after_step(refs)
    for n in range(100 if name != "small_batch" else 60):
        sim.step(1)
        for r in refs:
            r.step(1)
        if plan:
            plan.after_step(refs)
    h = sim.host()
    for b, r in enumerate(refs):
        g = gpu_instance_view(sim, h, b)
        rv = oracle_view(r)
        e = errors(g, rv, case.instances[b].fluid)
        assert max(e["rho"], e["v"], e["x_beyond_rounding"], e["dt"]) < 1e-6, (b, e)
        assert np.array_equal(g["count"], rv["count"]), b
    if plan:
        assert abs(sim.cell_builds() - plan.builds) <= plan.close_calls
    assert sim.poll_errors() == 0
    sim.close()


def test_morton_mixed_with_skin():
    case = dambreak.make_case("small_batch")
    sim = _sim(case, precision="mixed", skin=0.01 * case.h, use_graph=True)
    refs = oracles_for(case)
    sim.prime()
    for r in refs:
        r.prime()
    sim.step(40)
    for r in refs:
        r.step(40)
    h = sim.host()
    for b, r in enumerate(refs):
        g = gpu_instance_view(sim, h, b)
        rv = oracle_view(r)
        e = errors(g, rv, case.instances[b].fluid)
        assert max(e["rho"], e["v"], e["x"]) < GATE_100_STEPS, (b, e)
        assert np.count_nonzero(g["count"] != rv["count"]) <= 1, b
    assert sim.poll_errors() == 0
    sim.close()


@pytest.mark.slow
def test_morton_full_size_c2_with_skin():
    """The 2.0 M-particle 3D dam break, FP64, skin 0.1 h, tiled Morton keys:
    two steps against the reference particle by particle."""
    case = dambreak.make_case("c2_3d")
    sim = _sim(case, skin=0.1 * case.h)
    (r,) = oracles_for(case)
    sim.prime()
    r.prime()
    sim.step(2)
    r.step(2)
    h = sim.host()
    g = gpu_instance_view(sim, h, 0)
    rv = oracle_view(r)
    e = errors(g, rv, case.instances[0].fluid)
    print("c2 morton", e)
    assert max(e["rho"], e["v"], e["x_beyond_rounding"], e["dt"]) < 1e-9, e
    assert np.array_equal(g["count"], rv["count"])
    assert sim.poll_errors() == 0
    sim.close()
