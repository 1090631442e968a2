"""The host execution policy (SPH_POLICY_HOST): the step's per-particle and
per-pair bodies, shared with the GPU kernels, run on the host's threads.  On
the CPU it is checked against the FP64 reference like the device path is on
the GPU: integers (keys, sort permutation, cell and wall tables, neighbour
counts) bit for bit, FP64 fields to the same tolerances.  It never runs unless
asked for."""
import os

import numpy as np
import pytest

import dambreak
from _parity import errors, gpu_instance_view, integer_mismatches, oracle_view, oracles_for


@pytest.fixture(scope="module")
def sph():
    from paper_2603_11868_amd import sph, _build
    if not os.path.exists(sph.LIB_PATH):
        _build.build()
    sph.lib()
    return sph


def _host(sph, case, **kw):
    return sph.Simulation(case, precision="fp64", policy="host", **kw)


def _check_integers(g, r, what):
    mm = integer_mismatches(g, r)
    assert all(v == 0 for v in mm.values()), f"{what}: integer mismatches {mm}"


@pytest.mark.parametrize("name", ["tiny_2d", "c1_2d", "tiny_3d", "small_batch"])
def test_host_prime_matches_reference(sph, name):
    case = dambreak.make_case(name)
    sim = _host(sph, case)
    refs = oracles_for(case)
    sim.prime()
    for r in refs:
        r.prime()
    h = sim.host()
    assert sim.poll_errors() == 0
    for b, r in enumerate(refs):
        g = gpu_instance_view(sim, h, b)
        rv = oracle_view(r)
        _check_integers(g, rv, f"{name}[{b}] prime")
        assert np.abs(g["rho"] - rv["rho"]).max() <= 1e-13 * case.rho0
        assert np.abs(g["a"] - rv["a"]).max() <= 1e-10 * np.abs(rv["a"]).max()
        assert abs(g["dt"] - rv["dt"]) <= 1e-13 * rv["dt"]
        for slot in (0, 1, 2, 6, 7, 12):
            assert g["diag"][slot] == pytest.approx(rv["diag"][slot], rel=1e-11, abs=1e-300)
    sim.close()


@pytest.mark.parametrize("name", ["c1_2d", "tiny_3d"])
def test_host_steps_match_reference(sph, name):
    case = dambreak.make_case(name)
    sim = _host(sph, case)
    (r,) = oracles_for(case)
    sim.prime()
    r.prime()
    x0 = case.instances[0].fluid
    for n_done, tol in ((1, 1e-9), (100, 1e-6)):
        sim.step(n_done - sim.steps_done)
        r.step(n_done - r.step_count)
        h = sim.host()
        g = gpu_instance_view(sim, h, 0)
        rv = oracle_view(r)
        e = errors(g, rv, x0)
        print(name, "host policy", n_done, e)
        assert max(e["rho"], e["v"], e["x_beyond_rounding"], e["dt"]) < tol, e
        _check_integers(g, rv, f"{name} after {n_done}")
    assert sim.poll_errors() == 0
    sim.close()


def test_host_batch_equals_instances_alone(sph):
    case = dambreak.make_case("small_batch")
    sim = _host(sph, case)
    sim.prime()
    sim.step(7)
    h = sim.host()
    for b, inst in enumerate(case.instances):
        single = dambreak.Case(case.name, case.dim, case.dx, case.h,
                               reorder_every=case.reorder_every, instances=[inst])
        s1 = _host(sph, single)
        s1.prime()
        s1.step(7)
        h1 = s1.host()
        g = gpu_instance_view(sim, h, b)
        g1 = gpu_instance_view(s1, h1, 0)
        for k in ("key", "perm", "sorted_ids", "cell_start", "wall_start", "wall_perm", "count",
                  "x", "v", "a", "rho"):
            assert np.array_equal(g[k], g1[k]), (b, k)
        assert g["dt"] == g1["dt"]
        assert np.array_equal(g["diag"], g1["diag"])
        s1.close()
    sim.close()


def test_host_results_do_not_depend_on_the_thread_count(sph, monkeypatch):
    case = dambreak.make_case("c1_2d")
    out = []
    for threads in ("1", "3", "8"):
        monkeypatch.setenv("SPH_HOST_THREADS", threads)
        sim = _host(sph, case)
        sim.prime()
        sim.step(25)
        out.append(sim.host())
        sim.close()
    for k in ("x", "v", "a", "rho", "id", "perm", "count", "dt", "diag"):
        assert np.array_equal(out[0][k], out[1][k]) and np.array_equal(out[0][k], out[2][k]), k


def test_host_edge_cases_empty_instance_single_particle_and_clamping(sph):
    dx = 0.05
    # instance 0: one particle in free fall; 1: no fluid at all;
    # 2: particles outside the tank (keys clamped, flagged)
    i0 = dambreak.dam_break_instance(2, dx, (1.0, 1.0), (0.05, 0.05), 1)
    i0.fluid = np.array([[0.5, 0.6]])
    i1 = dambreak.dam_break_instance(2, dx, (0.5, 0.5), (0.0, 0.0), 2)
    i2 = dambreak.dam_break_instance(2, dx, (0.5, 0.5), (0.2, 0.2), 3)
    i2.fluid = i2.fluid.copy()
    i2.fluid[0] = [-5.0, 0.1]
    i2.fluid[1] = [0.1, 7.0]
    for inst in (i0, i1, i2):
        inst.c0 = 10.0
    case = dambreak.Case("edge", 2, dx, 1.3 * dx, reorder_every=2, instances=[i0, i1, i2])
    sim = _host(sph, case)
    refs = oracles_for(case)
    sim.prime()
    for r in refs:
        r.prime()
    assert sim.poll_errors() & sph.SPH_FLAG_CLAMPED
    sim.step(5)
    for r in refs:
        r.step(5)
    h = sim.host()
    for b, r in enumerate(refs):
        g = gpu_instance_view(sim, h, b)
        rv = oracle_view(r)
        _check_integers(g, rv, f"edge[{b}]")
        if r.n:
            assert np.abs(g["x"] - rv["x"]).max() < 1e-12
            assert np.abs(g["v"] - rv["v"]).max() < 1e-9
        assert g["dt"] == pytest.approx(rv["dt"], rel=1e-12)
        assert g["diag"][11] == rv["diag"][11]
    g0 = gpu_instance_view(sim, h, 0)
    t = g0["diag"][14]
    assert g0["x"][0, 1] == pytest.approx(0.6 - 0.5 * 9.81 * t * t, abs=1e-12)
    sim.close()


def test_host_policy_options_and_calls_are_checked(sph):
    case = dambreak.make_case("tiny_2d")
    for kw, status in ((dict(precision="mixed"), "UNSUPPORTED"), (dict(skin=0.1 * case.h), "UNSUPPORTED"),
                       (dict(key_order="morton"), "UNSUPPORTED"), (dict(scheme="dual"), "UNSUPPORTED"),
                       (dict(use_graph=True), "UNSUPPORTED")):
        args = dict(precision="fp64")
        args.update(kw)
        with pytest.raises(sph.SphError, match=status):
            sph.Simulation(case, policy="host", **args)
    with pytest.raises(ValueError):
        sph.Simulation(case, policy="elsewhere")
    sim = _host(sph, case)
    assert sph.sph_workspace_size(sim.ctx) == 0
    with pytest.raises(sph.SphError, match="SPH_E_STATE"):
        sim.step(1)                           # not primed
    sim.prime()
    for call in (sim.build_cells, sim.density, sim.forces, lambda: sim.sort(False), lambda: sim.integrate(1)):
        with pytest.raises(sph.SphError, match="UNSUPPORTED"):
            call()
    with pytest.raises(sph.SphError, match="UNSUPPORTED"):
        sph.sph_set_timing(sim.ctx, 1)
    with pytest.raises(sph.SphError, match="UNSUPPORTED"):
        sph.sph_bind_static(sim.ctx, sim.buffers, stream=0)
    sim.close()
