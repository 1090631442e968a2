"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, validates its arguments and derives
the same grid and lattice constants as the CPU reference."""
import os
import re

import numpy as np
import pytest

import dambreak
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sphmod():
    from paper_2603_11868_amd import sph, _build
    if not os.path.exists(sph.LIB_PATH):
        _build.build()
    sph.lib()
    return sph


def header_functions():
    with open(os.path.join(ROOT, "include", "sph.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(sphmod):
    names = header_functions()
    assert len(names) >= 19
    L = sphmod.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(sphmod.SYMBOLS)


def _params(sphmod, case, **over):
    B = len(case.instances)
    descs = (sphmod.sph_instance_desc * B)()
    for b, inst in enumerate(case.instances):
        descs[b].n_fluid = inst.n_fluid
        descs[b].n_wall = inst.n_wall
        for a in range(3):
            descs[b].tank_lo[a] = inst.tank_lo[a]
            descs[b].tank_hi[a] = inst.tank_hi[a]
        descs[b].c0 = inst.c0
    p = sphmod.sph_params()
    p.dim, p.precision, p.n_instances, p.reorder_every = case.dim, 0, B, case.reorder_every
    p.dx, p.h, p.rho0, p.alpha, p.eps, p.cfl_ac, p.cfl_f = (case.dx, case.h, case.rho0, case.alpha,
                                                          case.eps, case.cfl_ac, case.cfl_f)
    for a in range(3):
        p.g[a] = case.g[a]
    p.inst = descs
    for k, v in over.items():
        setattr(p, k, v)
    return p, descs


@pytest.mark.parametrize("name", ["c1_2d", "tiny_3d", "small_batch", "c2_3d"])
def test_derived_grid_and_constants_match_reference(sphmod, name):
    case = dambreak.make_case(name)
    p, descs = _params(sphmod, case)
    ctx = sphmod.sph_create(p)
    try:
        info = sphmod.sph_get_info(ctx)
        assert info.n_fluid == case.n_fluid and info.n_wall == case.n_wall
        base = 0
        for b, inst in enumerate(case.instances):
            ref = O.OracleSim(case.dim, case.dx, case.h, inst.tank_lo, inst.tank_hi,
                              inst.fluid[:2], inst.wall[:2], inst.c0)
            lo, nc, cb = sphmod.sph_get_grid(ctx, b)
            assert nc == ref.ncell and cb == base
            assert lo[:case.dim] == ref.lo[:case.dim]
            base += ref.ncells
            assert info.sigma0 == pytest.approx(ref.sigma0, rel=1e-14)
            assert info.mass == pytest.approx(ref.mass, rel=1e-14)
        assert info.n_cells == base
        assert info.cell_size == 2 * case.h
        assert info.workspace_bytes > 0 and sphmod.sph_workspace_size(ctx) == info.workspace_bytes
    finally:
        sphmod.sph_destroy(ctx)


def test_argument_validation(sphmod):
    case = dambreak.make_case("tiny_2d")
    bad = [dict(dim=4), dict(precision=7), dict(n_instances=0), dict(dx=0.0), dict(h=-1.0),
           dict(block_threads=100), dict(reorder_every=-1), dict(eps=0.0),
           dict(list_cap=5000), dict(prefetch=3)]
    for over in bad:
        p, descs = _params(sphmod, case, **over)
        with pytest.raises(sphmod.SphError, match="SPH_E_ARG"):
            sphmod.sph_create(p)
    p, descs = _params(sphmod, case)
    descs[0].c0 = 0.0
    with pytest.raises(sphmod.SphError, match="SPH_E_ARG"):
        sphmod.sph_create(p)
    p, descs = _params(sphmod, case)
    descs[0].n_fluid = -3
    with pytest.raises(sphmod.SphError, match="SPH_E_ARG"):
        sphmod.sph_create(p)
    assert "negative" in sphmod.sph_last_error()


def test_calls_before_bind_are_rejected(sphmod):
    case = dambreak.make_case("tiny_2d")
    p, descs = _params(sphmod, case)
    ctx = sphmod.sph_create(p)
    try:
        for fn in (sphmod.sph_prime, sphmod.sph_build_cells, sphmod.sph_density, sphmod.sph_forces):
            with pytest.raises(sphmod.SphError, match="SPH_E_STATE"):
                fn(ctx, 0)
        with pytest.raises(sphmod.SphError, match="SPH_E_STATE"):
            sphmod.sph_step_batched(ctx, 1, 0)
        with pytest.raises(sphmod.SphError, match="SPH_E_ARG"):
            sphmod.sph_step_batched(ctx, -1, 0)
        with pytest.raises(sphmod.SphError, match="SPH_E_ARG"):
            sphmod.sph_get_grid(ctx, 5)
    finally:
        sphmod.sph_destroy(ctx)
    sphmod.sph_destroy(None)


def test_stage_names(sphmod):
    n = sphmod.sph_stage_count()
    names = [sphmod.sph_stage_name(i) for i in range(n)]
    assert names[:2] == ["keys", "cell_scan"] and "density" in names and "force" in names
    assert sphmod.sph_stage_name(n) == ""


def test_product_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2603_11868_amd import sph
    monkeypatch.setattr(sph, "_lib", None)
    monkeypatch.setattr(sph, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        sph.lib()


def test_dual_scheme_options_are_checked(sphmod):
    case = dambreak.make_case("tiny_2d")
    base = dict(scheme=sphmod.SPH_SCHEME_DUAL, cfl_ac=sphmod.DUAL_CFL_AC,
                cfl_adv=sphmod.DUAL_CFL_ADV, eta=sphmod.DUAL_ETA)
    p, descs = _params(sphmod, case, **base)
    ctx = sphmod.sph_create(p)
    sphmod.sph_destroy(ctx)
    # graphs replay whole advection steps (the sub-step plan stays on the device)
    p, descs = _params(sphmod, case, use_graph=1, **base)
    sphmod.sph_destroy(sphmod.sph_create(p))
    for over, status in ((dict(precision=1), "UNSUPPORTED"), (dict(cfl_adv=0.0), "E_ARG"),
                         (dict(scheme=7), "E_ARG"), (dict(cfl_adv=300.0), "E_ARG")):
        p, descs = _params(sphmod, case, **dict(base, **over))
        with pytest.raises(sphmod.SphError, match=status):
            sphmod.sph_create(p)


def test_skin_options_and_grid(sphmod):
    import math
    case = dambreak.make_case("c1_2d")
    skin = 0.25 * case.h
    p, descs = _params(sphmod, case, skin=skin)
    ctx = sphmod.sph_create(p)
    try:
        info = sphmod.sph_get_info(ctx)
        cs = 2 * case.h + skin
        assert info.cell_size == cs
        inst = case.instances[0]
        lo, nc, cb = sphmod.sph_get_grid(ctx, 0)
        for a in range(case.dim):
            assert lo[a] == inst.tank_lo[a] - 3 * case.dx
            assert nc[a] == math.ceil((inst.tank_hi[a] - inst.tank_lo[a] + 6 * case.dx) / cs)
    finally:
        sphmod.sph_destroy(ctx)
    for over, status in ((dict(skin=-1e-3), "E_ARG"), (dict(skin=3 * case.h), "E_ARG"),
                         (dict(skin=float("nan")), "E_ARG")):
        p, descs = _params(sphmod, case, **over)
        with pytest.raises(sphmod.SphError, match=status):
            sphmod.sph_create(p)


def test_dual_scheme_with_a_skin_keeps_positions_of_the_build(sphmod):
    # the dual scheme tests exact displacements: its workspace also holds x
    # at the last build (dim * N doubles, 256-byte aligned)
    case = dambreak.make_case("tiny_3d")
    dual = dict(scheme=sphmod.SPH_SCHEME_DUAL, cfl_adv=0.25, eta=3.0)
    sizes = {}
    for sk, extra in (("wcsph", {}), ("dual", dual)):
        p, descs = _params(sphmod, case, skin=0.5 * case.h, **extra)
        ctx = sphmod.sph_create(p)
        sizes[sk] = sphmod.sph_workspace_size(ctx)
        sphmod.sph_destroy(ctx)
    n = case.n_fluid
    # dual adds Drho (N doubles) and the build positions (dim N doubles) in
    # place of two 256-byte placeholders
    extra = sizes["dual"] - sizes["wcsph"]
    assert 8 * 4 * n - 512 <= extra <= 8 * 4 * n + 512, (extra, n)


def test_skin_scales_the_default_list_capacity(sphmod):
    # the workspace holds the list: its size grows with ((2h + skin) / 2h)^dim
    case = dambreak.make_case("tiny_3d")
    sizes = []
    for skin in (0.0, 0.5 * case.h):
        p, descs = _params(sphmod, case, skin=skin)
        ctx = sphmod.sph_create(p)
        sizes.append(sphmod.sph_workspace_size(ctx))
        sphmod.sph_destroy(ctx)
    n = case.n_fluid
    grown = 4 * ((int(-(-96 * 1.25 ** 3 // 1)) + 3) // 4) - 96
    # (less the smaller cell arrays of the coarser grid)
    assert 0.9 * grown * 4 * n <= sizes[1] - sizes[0] <= grown * 4 * n + 4096


def test_key_order_option(sphmod):
    case = dambreak.make_case("tiny_3d")
    p, descs = _params(sphmod, case, key_order=sphmod.SPH_KEYS_MORTON_TILES)
    ctx = sphmod.sph_create(p)
    try:
        info = sphmod.sph_get_info(ctx)
        lo, nc, cb = sphmod.sph_get_grid(ctx, 0)
        tiles = ((nc[0] + 7) // 8) * ((nc[1] + 7) // 8) * ((nc[2] + 7) // 8)
        assert info.n_cells == tiles * 512
    finally:
        sphmod.sph_destroy(ctx)
    p, descs = _params(sphmod, case, key_order=5)
    with pytest.raises(sphmod.SphError, match="E_ARG"):
        sphmod.sph_create(p)


def test_bind_static_rejects_workspaces_beyond_its_scratch(sphmod):
    """sph_bind_static checks the workspace size against the static scratch
    before it touches the device: the 2.0 M-particle case needs far more."""
    case = dambreak.make_case("c2_3d")
    p, descs = _params(sphmod, case)
    ctx = sphmod.sph_create(p)
    try:
        assert sphmod.sph_workspace_size(ctx) > sphmod.SPH_STATIC_SCRATCH_BYTES
        bufs = sphmod.sph_buffers()
        with pytest.raises(sphmod.SphError, match="SPH_E_CAPACITY.*static scratch"):
            sphmod.sph_bind_static(ctx, bufs, stream=0)
    finally:
        sphmod.sph_destroy(ctx)


def test_static_scratch_size_matches_header(sphmod):
    with open(os.path.join(ROOT, "include", "sph.h")) as f:
        text = f.read()
    m = re.search(r"#define SPH_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == sphmod.SPH_STATIC_SCRATCH_BYTES
