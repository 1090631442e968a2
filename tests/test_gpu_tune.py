"""The autotuner and the two list builds on the GPU.

The cell-pair build and the lane-per-target build must write the same lists,
so every output of a run is identical bit for bit; a variant the tuner picks
keeps the integers of the default run and matches the CPU reference."""
import numpy as np
import pytest

import dambreak
from _parity import errors, gpu_instance_view, integer_mismatches, oracle_view, oracles_for

pytestmark = pytest.mark.gpu


def _run(case, steps, **kw):
    from paper_2603_11868_amd import sph
    sim = sph.Simulation(case, **kw)
    sim.prime()
    sim.step(steps)
    flags = sim.poll_errors()
    h = sim.host()
    sim.close()
    return h, flags


@pytest.mark.parametrize("name,precision,skin_h", [
    ("tiny_3d", "fp64", 0.0), ("tiny_3d", "mixed", 0.0), ("c1_2d", "fp64", 0.0),
    ("small_batch", "mixed", 0.0), ("tiny_3d", "fp64", 0.05), ("small_batch", "fp64", 0.02)])
def test_cell_pair_build_equals_lane_per_target_build(name, precision, skin_h):
    case = dambreak.make_case(name)
    print(f"builds: {name} {precision} skin {skin_h} h", flush=True)
    a, fa = _run(case, 25, precision=precision, skin=skin_h * case.h, build=2)
    b, fb = _run(case, 25, precision=precision, skin=skin_h * case.h, build=1)
    assert fa == fb == 0
    for k in ("key", "perm", "cell_start", "count", "id", "x", "v", "a", "rho", "dt", "diag"):
        assert np.array_equal(a[k], b[k]), k


def test_cell_pair_build_overflow_matches():
    """A capacity below the neighbour counts: both builds flag the overflow and
    their targets search the cells; results identical."""
    from paper_2603_11868_amd import sph
    case = dambreak.make_case("tiny_3d")
    a, fa = _run(case, 5, list_cap=16, build=2)
    b, fb = _run(case, 5, list_cap=16, build=1)
    assert fa & sph.SPH_FLAG_CAPACITY and fb & sph.SPH_FLAG_CAPACITY
    for k in ("count", "x", "v", "rho"):
        assert np.array_equal(a[k], b[k]), k


def test_tuned_variant_keeps_integers_and_matches_reference(tmp_path):
    from paper_2603_11868_amd import tune
    case = dambreak.make_case("tiny_3d")
    cache = str(tmp_path / "tune.json")
    entry = tune.tune(case, "fp64", steps=3, warmup=1, blocks=(64, 256), builds=(1, 2),
                      prefetches=(4, 8), cache_path=cache, log=None)
    best = tune.lookup(case, "fp64", cache_path=cache)
    assert best == entry["best"] and best["flags"] == 0
    assert len(entry["all"]) >= 4
    steps = 10
    ref, _ = _run(case, steps, precision="fp64")
    got, flags = _run(case, steps, precision="fp64", block_threads=best["block_threads"],
                      build=best["build"], prefetch=best["prefetch"])
    assert flags == 0
    for k in ("key", "perm", "cell_start", "count", "id"):
        assert np.array_equal(ref[k], got[k]), k
    (r,) = oracles_for(case)
    r.prime()
    r.step(steps)
    from paper_2603_11868_amd import sph
    sim = sph.Simulation(case, precision="fp64", block_threads=best["block_threads"],
                         build=best["build"], prefetch=best["prefetch"])
    sim.prime()
    sim.step(steps)
    g = gpu_instance_view(sim, sim.host(), 0)
    sim.close()
    rv = oracle_view(r)
    assert all(v == 0 for v in integer_mismatches(g, rv).values())
    e = errors(g, rv, case.instances[0].fluid)
    assert max(e["rho"], e["v"], e["x_beyond_rounding"], e["dt"]) < 1e-9, e
