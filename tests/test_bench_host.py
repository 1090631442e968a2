"""Host-side checks of the benchmark driver and of the list-size limit of the
C ABI (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import dambreak  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_summary_is_used_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2603_11868_amd").symlink_to(os.path.join(ROOT, "paper_2603_11868_amd"))
    h = bench.kernel_source_hash()
    f = prof / "density_w_fp64_pmc.md"
    f.write_text(f"# x\n- hbm_bytes_per_launch: 2.5e+09\n- source_hash: `{h}`\n")
    assert bench.load_traffic("w", "fp64", "density") == 2.5e9
    f.write_text("- hbm_bytes_per_launch: 2.5e+09\n- source_hash: `0000000000000000`\n")
    assert bench.load_traffic("w", "fp64", "density") is None
    assert bench.load_traffic("w", "mixed", "density") is None


class _FakeSim:
    """Grid of one instance for candidate_count."""
    def __init__(self, case, oracle):
        self.dim = case.dim
        self.B = 1
        self.fluid_offset = [0, oracle.n]
        self._grid = (oracle.lo, oracle.ncell, 0)

    def grid(self, b):
        return self._grid


def test_candidate_count_matches_brute_force():
    """Candidates of direct search = particles (fluid + wall) in the 3^d cells
    around each target's cell, minus the target itself."""
    from oracle import oracle as O
    case = dambreak.make_case("tiny_3d")
    r = O.OracleSim.from_case(case, 0)
    r.prime()
    nc = r.ncell
    cs = r.start.astype(np.int64)
    ws = r.wstart.astype(np.int64)
    occ = (cs[1:] - cs[:-1]) + (ws[1:] - ws[:-1])
    brute = 0
    for key in r.key:
        cx, cy, cz = key % nc[0], (key // nc[0]) % nc[1], key // (nc[0] * nc[1])
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    x, y, z = cx + dx, cy + dy, cz + dz
                    if 0 <= x < nc[0] and 0 <= y < nc[1] and 0 <= z < nc[2]:
                        brute += occ[x + nc[0] * (y + nc[1] * z)]
        brute -= 1
    h = {"cell_start": r.start, "wall_start": r.wstart, "key": r.key}
    assert bench.candidate_count(_FakeSim(case, r), h) == brute


def test_list_size_limit_is_reported(monkeypatch):
    """The neighbour list addresses fewer than 2^25 particles per kind; a
    larger set must be refused at sph_create (no device memory involved)."""
    from paper_2603_11868_amd import sph, _build
    if not os.path.exists(sph.LIB_PATH):
        _build.build()
    case = dambreak.make_case("tiny_3d")
    inst = case.instances[0]
    descs = (sph.sph_instance_desc * 1)()
    descs[0].n_fluid = 1 << 25
    descs[0].n_wall = inst.n_wall
    for a in range(3):
        descs[0].tank_lo[a] = inst.tank_lo[a]
        descs[0].tank_hi[a] = inst.tank_hi[a]
    descs[0].c0 = inst.c0
    p = sph.sph_params()
    p.dim, p.precision, p.n_instances, p.reorder_every = 3, 0, 1, 20
    p.dx, p.h, p.rho0, p.alpha, p.eps, p.cfl_ac, p.cfl_f = (case.dx, case.h, case.rho0, case.alpha,
                                                          case.eps, case.cfl_ac, case.cfl_f)
    p.g[2] = -9.81
    p.inst = descs
    with pytest.raises(sph.SphError, match="2\\^25"):
        sph.sph_create(p)
    p.list_cap = -1
    ctx = sph.sph_create(p)
    sph.sph_destroy(ctx)
