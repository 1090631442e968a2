"""The stable cell sort (Sec. 5: cell keys, radix sort) on fluid stored in
three orders: the generator's lattice order, already in cell order (every
wave's digits non-decreasing, the run-based ranking) and a seeded shuffle
(nearly every wave takes the ballot ranking).  Keys are checked bit for bit
against the row-major cell mapping applied to the positions, the permutation
against numpy's stable argsort and the start table against a search of the
sorted keys."""
import dataclasses

import numpy as np
import pytest

import dambreak

pytestmark = pytest.mark.gpu


def _row_keys(sim, case, x):
    """Global row-major keys of storage-order positions x (N x dim): subtract
    the grid origin, multiply by 1/cs, floor, clamp."""
    out = np.empty(len(x), dtype=np.int64)
    inv_cs = 1.0 / sim.info.cell_size
    for b in range(sim.B):
        f0, f1 = sim.fluid_offset[b], sim.fluid_offset[b + 1]
        lo, nc, base = sim.grid(b)
        c = [np.zeros(f1 - f0, dtype=np.int64) for _ in range(3)]
        for a in range(case.dim):
            v = np.floor((x[f0:f1, a] - lo[a]) * inv_cs)
            c[a] = np.clip(v, 0, nc[a] - 1).astype(np.int64)
        out[f0:f1] = base + c[0] + nc[0] * (c[1] + nc[1] * c[2])
    return out


def _reordered(case, order, key_of):
    """The case with each instance's fluid in the given order."""
    rng = np.random.default_rng(2603)
    insts = []
    off = 0
    for inst in case.instances:
        n = inst.n_fluid
        if order == "sorted":
            idx = np.argsort(key_of[off:off + n], kind="stable")
        elif order == "shuffled":
            idx = rng.permutation(n)
        else:
            idx = np.arange(n)
        insts.append(dataclasses.replace(inst, fluid=np.ascontiguousarray(inst.fluid[idx])))
        off += n
    return dataclasses.replace(case, instances=insts)


@pytest.mark.parametrize("name", ["c1_2d", "small_batch", "c2_3d"])
def test_sort_in_three_storage_orders(name):
    from paper_2603_11868_amd import sph
    base_case = dambreak.make_case(name)
    probe = sph.Simulation(base_case, precision="fp64")
    key0 = _row_keys(probe, base_case, np.concatenate([i.fluid for i in base_case.instances]))
    probe.close()
    for order in ("lattice", "sorted", "shuffled"):
        case = _reordered(base_case, order, key0)
        sim = sph.Simulation(case, precision="fp64")
        sph.sph_build_cells(sim.ctx)
        sph.sph_sort(sim.ctx, 0)
        h = sim.host()
        key = _row_keys(sim, case, h["x"])
        assert np.array_equal(h["key"].astype(np.int64), key), order
        perm = np.argsort(key, kind="stable")
        assert np.array_equal(h["perm"].astype(np.int64), perm), order
        if order == "sorted":
            assert np.array_equal(perm, np.arange(len(key))), order
        start = np.searchsorted(np.sort(key), np.arange(sim.C + 1), side="left")
        assert np.array_equal(h["cell_start"].astype(np.int64), start), order
        sim.close()
