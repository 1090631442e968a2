"""Throughput of the WCSPH step on one MI355X.

Default workload: the large 3D dam break, a 2 x 2 x 2 m fluid block at
dx = 0.0065 (308^3 = 29,218,112 fluid particles) in an 8 x 2 x 3 m box with
three layers of wall particles (6,613,248), on the mixed-precision path, the
arrays re-sorted by cell every 50 steps.  A step is the whole hot path: half
kick + drift + cell keys, cell scan, radix sort, (reorder), sweep records,
density sweep (candidate tests and neighbour lists), force sweep fused with
the second half kick, and the FP64 reductions for dt and the diagnostics.
The headline rebuilds the cell table and the neighbour lists in every step.

Prints one JSON line.  Besides the headline value it reports the roofline of
the dominant kernel (algorithmic FLOPs per launch over its HIP-event time in
the timed steps; only the pair sweeps carry events there, the other stages are
timed on eager steps right after), the conservation drift over the timed
steps, the same workload on the plain FP64 path together with the error of
the mixed run against it (density, velocity, position, total energy), the
headline precision again with a Verlet skin (cells and lists reused between
builds the device decides on), and the CPU reference timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "M particle-updates/s (3D WCSPH step) + achieved HBM GB/s vs FP64 path"
FP64_VALU_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 64 lanes x 2 x 2.4 GHz)
FP32_VALU_PEAK_TFLOPS = 157.3    # MI355X FP32 vector, packed (twice the unpacked rate)
HBM_PEAK_GBS = 8000.0
SWEEP_STAGES = ("build", "density", "force", "sub_pressure", "sub_density")
CLOCK_HZ, N_CU = 2.4e9, 256

# Flops per candidate test and per neighbour pair (viscosity excluded: it
# runs on approaching pairs only, so leaving it out keeps the count a lower
# bound).  Candidate (list build, FP32 on both paths): r = x_i - x_j, r^2.
# Density pair: sqrt, q, t, t^3, W, F, v_ij.r, two accumulations.  Force
# pair: sqrt, q, t, t^3, F, v_ij.r, (P_i + P_j) F, two vector accumulations.
FLOPS = {
    2: {"cand": 5, "density": 20, "force": 24},
    3: {"cand": 8, "density": 23, "force": 30},
}
# dual-criteria scheme, FP64 flops per neighbour pair of a sub-step sweep.
# Both sweeps: unit vector and normal velocities (sqrt, division, 2 dot
# products), the limiter and the Riemann state (about 12), the kernel
# gradient factor (sqrt, q, t, t^3, F).  Pressure: P*/(rho_i rho_j) F and the
# vector accumulation.  Density: the velocity jump, its dot product with r and
# the accumulation.
FLOPS_DUAL = {
    2: {"sub_pressure": 37, "sub_density": 41},
    3: {"sub_pressure": 45, "sub_density": 51},
}

WORKLOADS = {
    "c2_3d": "3D WCSPH dam break: 1x1x2 m fluid block at dx=0.01 (2,000,000 fluid + "
             "1,169,016 wall particles) in a 4x1x3 m box, Wendland C2 h=1.3dx, "
             "re-sort every 20 steps",
    "c3_3d": "3D WCSPH dam break: 1x1x2 m block at dx=0.005 (16,000,000 fluid + "
             "4,617,816 wall particles) in a 4x1x3 m box",
    "c5_3d": "3D WCSPH dam break: 2x2x2 m block at dx=0.0065 (29,218,112 fluid + "
             "6,613,248 wall particles) in an 8x2x3 m box, re-sort every 50 steps",
    "c4_batch": "64 independent 2D dam breaks, widths U[0.5,2] m, dx=0.005 "
                "(8.37 M fluid particles in total), one launch per stage",
    "c1_2d": "2D WCSPH dam break: 1x2 m column at dx=0.025 (3,200 fluid particles)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def candidate_count(sim, h):
    """Sum over fluid targets of the particles (fluid + wall) in their 3^d
    stencil cells, minus the target itself: the candidates direct search tests."""
    dim = sim.dim
    cs = h["cell_start"].astype(np.int64)
    ws = h["wall_start"].astype(np.int64)
    occ = (cs[1:] - cs[:-1]) + (ws[1:] - ws[:-1])
    total = 0
    for b in range(sim.B):
        f0, f1 = sim.fluid_offset[b], sim.fluid_offset[b + 1]
        if f1 == f0:
            continue
        lo, nc, base = sim.grid(b)
        nx, ny, nz = nc
        if getattr(sim, "key_order", "row") == "morton":
            # tables in tiled Morton order: move them to row-major cells
            cells = np.arange(nx * ny * nz)
            cx, cy, cz = cells % nx, (cells // nx) % ny, cells // (nx * ny)
            mk = morton_key(cx, cy, cz, nc, dim)
            occ_b = occ[base + mk].reshape(nz, ny, nx)
        else:
            occ_b = occ[base:base + nx * ny * nz].reshape(nz, ny, nx)
        # 3^d box sum of occupancy with clamping at the grid edge
        pad = np.pad(occ_b, ((1, 1) if dim == 3 else (0, 0), (1, 1), (1, 1)))
        box = np.zeros_like(occ_b)
        for dz in ((-1, 0, 1) if dim == 3 else (0,)):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    zz = slice(1 + dz, 1 + dz + nz) if dim == 3 else slice(0, nz)
                    box += pad[zz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        keys = h["key"][f0:f1].astype(np.int64) - base
        if getattr(sim, "key_order", "row") == "morton":
            inv = np.empty(int(mk.max()) + 1, dtype=np.int64)
            inv[mk] = cells
            keys = inv[keys]
        total += int(box.reshape(-1)[keys].sum()) - (f1 - f0)
    return total


def morton_key(cx, cy, cz, nc, dim):
    """Local key of the tiled Morton order (tiles of 8^d cells, row-major;
    Morton inside a tile), as the library defines it."""
    ntx, nty = (nc[0] + 7) // 8, (nc[1] + 7) // 8
    tile = (cx >> 3) + ntx * ((cy >> 3) + nty * (cz >> 3))
    m = np.zeros_like(cx)
    for b in range(3):
        m |= ((cx >> b) & 1) << (dim * b)
        m |= ((cy >> b) & 1) << (dim * b + 1)
        if dim == 3:
            m |= ((cz >> b) & 1) << (dim * b + 2)
    return (tile << (3 * dim)) | m


def kernel_source_hash():
    hsh = hashlib.sha256()
    for name in ("sph_sweeps.hip", "sph_step_common.h", "sph_device.h", "sph_bodies.h"):
        with open(os.path.join(ROOT, "paper_2603_11868_amd", "csrc", name), "rb") as f:
            hsh.update(f.read())
    return hsh.hexdigest()[:16]


def load_traffic(workload, precision, kernel):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel source (else None).  The summary is a text file
    with `source_hash: ...` and `hbm_bytes_per_launch: ...` lines."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_pmc.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^\W*(source_hash|hbm_bytes_per_launch)\W*:\s*`?([0-9A-Za-z.+e-]+)", line)
            if m:
                rec[m.group(1)] = m.group(2)
    if rec.get("source_hash") != kernel_source_hash() or "hbm_bytes_per_launch" not in rec:
        return None
    return float(rec["hbm_bytes_per_launch"])


def library_source_hash():
    """Hash of every source of libsph (all kernels of a step)."""
    hsh = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_11868_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                hsh.update(f.read())
    return hsh.hexdigest()[:16]


def load_step_traffic(workload, precision):
    """HBM bytes of one whole step (every kernel) from a committed rocprofv3
    PMC summary taken on the current library sources (else None)."""
    import re
    path = os.path.join(ROOT, "profiles", f"step_{workload}_{precision}_pmc.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^\W*(library_hash|hbm_bytes_per_step)\W*:\s*`?([0-9A-Za-z.+e-]+)", line)
            if m:
                rec[m.group(1)] = m.group(2)
    if rec.get("library_hash") != library_source_hash() or "hbm_bytes_per_step" not in rec:
        return None
    return float(rec["hbm_bytes_per_step"])


def load_l1(workload, precision, kernel):
    """L1 (TCP) accesses per launch of a sweep from a committed rocprofv3 summary
    taken on the current kernel sources (else None)."""
    import re
    path = os.path.join(ROOT, "profiles", f"l1_{workload}_{precision}_tcp.md")
    if not os.path.exists(path):
        return None
    acc, hsh = None, None
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+) l1_accesses_per_launch: ([0-9.e+-]+)", line)
            if m and m.group(1) == kernel:
                acc = float(m.group(2))
            m = re.match(r"^- source_hash: `([0-9a-f]+)`", line)
            if m:
                hsh = m.group(1)
    return acc if hsh == kernel_source_hash() else None


def load_valu(workload, precision, kernel, unit="valu"):
    """VALU (or, with unit="salu", SALU) instructions (wave64) per launch of a
    sweep or the list build from a committed rocprofv3 summary taken on the
    current kernel sources (else None)."""
    import re
    path = os.path.join(ROOT, "profiles", f"valu_{workload}_{precision}_sq.md")
    if not os.path.exists(path):
        return None
    val, hsh = None, None
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+) " + unit + r"_insts_per_launch: ([0-9.e+-]+)", line)
            if m and m.group(1) == kernel:
                val = float(m.group(2))
            m = re.match(r"^- source_hash: `([0-9a-f]+)`", line)
            if m:
                hsh = m.group(1)
    return val if hsh == kernel_source_hash() else None


def run_gpu(case, precision, steps, warmup, graph, timing, reorder_every=None, block=0,
            list_cap=0, prefetch=0, stage_steps=0, scheme="wcsph", skin_h=0.0, key_order="row",
            tuned=True, build=None):
    """One timed leg: prime, `warmup` untimed steps, `steps` timed steps, then
    optionally `stage_steps` eager steps with events around every stage.
    tuned: launch parameters left unset come from the autotuner's cache."""
    import torch
    from paper_2603_11868_amd import sph

    sim = sph.Simulation(case, precision=precision, reorder_every=reorder_every,
                         use_graph=graph, block_threads=block,
                         list_cap=list_cap, prefetch=prefetch, scheme=scheme,
                         skin=skin_h * case.h, key_order=key_order, tuned=tuned, build=build)
    sim.key_order = key_order
    sim.prime()
    sim.step(warmup)
    torch.cuda.synchronize()
    sub0 = int(sph.sph_get_info(sim.ctx).substeps_done)
    builds0 = sim.cell_builds()
    diag0 = sim.diag.detach().cpu().numpy().copy()
    if timing:
        # HIP events around the pair sweeps only: events around every stage
        # would slow the timed steps by ~4 %
        names = [sph.sph_stage_name(i) for i in range(sph.sph_stage_count())]
        mask = sum(1 << i for i, nm in enumerate(names) if nm in SWEEP_STAGES)
        sph.sph_set_timing_mask(sim.ctx, mask)
        sph.sph_stage_times(sim.ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    diag1 = sim.diag.detach().cpu().numpy().copy()
    sub1 = int(sph.sph_get_info(sim.ctx).substeps_done)
    sim.timed_builds = sim.cell_builds() - builds0
    sweeps = sph.sph_stage_times(sim.ctx, reset=True) if timing else {}
    sph.sph_set_timing(sim.ctx, 0)
    # state at the end of the timed steps (before the stage-timing steps)
    h = sim.host()
    stages = {}
    if stage_steps:
        # every stage, on eager launches of the steps right after the timed
        # region (graph replays carry no per-stage events)
        sph.sph_set_timing(sim.ctx, 1)
        sph.sph_stage_times(sim.ctx, reset=True)
        sim.step(stage_steps)
        torch.cuda.synchronize()
        stages = sph.sph_stage_times(sim.ctx, reset=True)
        sph.sph_set_timing(sim.ctx, 0)
    # the sweeps' times from the timed steps themselves where they were taken
    for k, v in sweeps.items():
        if v[1]:
            stages[k] = v
    sim.sweeps_timed = bool(sweeps and any(v[1] for v in sweeps.values()))
    flags = sim.poll_errors()
    sim.timed_substeps = sub1 - sub0
    sim.diag0, sim.diag1 = diag0, diag1
    return sim, h, t1 - t0, stages, flags


def drift(case, mass, d0, d1):
    """Conservation over the timed steps from the per-instance diagnostics
    (slots as in include/sph.h), summed over instances.

    mass_rel: change of the fluid mass (particles are never created or lost,
    so exactly 0 unless one left the grid); rho_mean: change of mean(rho)/rho0;
    momentum_residual_rel: impulse of the fluid-fluid forces (zero in exact
    arithmetic: pairwise forces cancel) over the gravity impulse M |g| t of the
    same steps; energy: total energy before and after (kinetic + potential +
    internal; the artificial viscosity dissipates it)."""
    M0, M1 = d0[:, 2].sum(), d1[:, 2].sum()
    dt_sum = d1[:, 14] - d0[:, 14]
    grav = float((d1[:, 2] * case.gmag * dt_sum).sum())
    res = float((d1[:, 13] - d0[:, 13]).sum())
    e0 = float((d0[:, 6] + d0[:, 7] + d0[:, 8]).sum())
    e1 = float((d1[:, 6] + d1[:, 7] + d1[:, 8]).sum())
    return {
        "mass_rel": float((M1 - M0) / M0) if M0 else 0.0,
        "rho_mean_change": float((d1[:, 10] - d0[:, 10]).mean()),
        "momentum_residual_rel": (res / grav) if grav > 0 else None,
        "energy_before": e0, "energy_after": e1,
        "sim_time_s": float(dt_sum.mean()),
    }


def total_energy(case, mass, st):
    """Kinetic + potential + internal energy of a fluid state (by particle id),
    internal energy of the clipped equation of state, m c0^2 (ln(rho/rho0) +
    rho0/rho - 1) for rho > rho0; summed on the host in one fixed order so that
    two states differ only by their values.  Returns (E, kinetic)."""
    dim = case.dim
    off = np.concatenate([[0], np.cumsum([i.n_fluid for i in case.instances])])
    e_tot, ke_tot = 0.0, 0.0
    for b, inst in enumerate(case.instances):
        sl = slice(off[b], off[b + 1])
        x, v, rho = st["x"][sl], st["v"][sl], st["rho"][sl]
        ke = 0.5 * mass * np.sum(v * v, axis=1)
        pe = -mass * (x @ case.g[:dim])
        ie = np.where(rho > case.rho0,
                      mass * inst.c0 ** 2 * (np.log(rho / case.rho0) + case.rho0 / rho - 1.0), 0.0)
        e_tot += float(np.sum(ke + pe + ie))
        ke_tot += float(np.sum(ke))
    return e_tot, ke_tot


def state_errors(case, mass, test, ref):
    """Errors of one run against another after the same steps, by particle id,
    over the probe set (a seeded sample of 10,000 fluid ids plus the corners of
    the block, per instance) and over all particles:
    e_rho = max|d rho| / rho0, e_v = max|d v| / max|v_ref|,
    e_x = max|d x| / max|x_ref - x0| (displacement-normalised), and the total
    energy error |E - E_ref| / KE_ref (E = kinetic + potential + internal)."""
    import dambreak

    def by_id(st):
        out = {}
        for k in ("x", "v", "rho"):
            arr = np.empty_like(st[k])
            arr[st["id"]] = st[k]
            out[k] = arr
        return out

    a, b = by_id(test), by_id(ref)
    x0 = np.concatenate([i.fluid[:, :case.dim] for i in case.instances], 0)
    off = np.concatenate([[0], np.cumsum([i.n_fluid for i in case.instances])])
    probe = np.concatenate([off[bb] + dambreak.probe_ids(inst) for bb, inst in enumerate(case.instances)])

    def errs(sel):
        vref = np.abs(b["v"][sel]).max()
        disp = np.abs(b["x"][sel] - x0[sel]).max()
        return {"rho": float(np.abs(a["rho"][sel] - b["rho"][sel]).max() / case.rho0),
                "v": float(np.abs(a["v"][sel] - b["v"][sel]).max() / max(vref, 1e-300)),
                "x": float(np.abs(a["x"][sel] - b["x"][sel]).max() / max(disp, 1e-300))}

    e_t, _ = total_energy(case, mass, a)
    e_r, ke = total_energy(case, mass, b)
    return {"probe": errs(probe), "all": errs(slice(None)), "n_probe": int(probe.size),
            "energy_rel_ke": float(abs(e_t - e_r) / ke) if ke > 0 else None}


def cpu_baseline(case, nsteps, scheme="wcsph"):
    """The CPU reference on the same workload: M updates/s over nsteps steps of
    every instance of the case, one after the other (dual scheme: advection
    steps, counted in acoustic sub-steps).  Returns the rate, the threads it
    used, the seconds timed and the particle updates counted."""
    from oracle import oracle as O

    secs, updates = 0.0, 0
    for b, inst in enumerate(case.instances):
        ref = O.OracleSim.from_case(case, index=b)
        if scheme == "dual":
            ref.dual_prime()
            t0 = time.perf_counter()
            subs = 0
            for _ in range(nsteps):
                subs += ref.dual_plan()[1]
                ref.dual_step(1)
            secs += time.perf_counter() - t0
            updates += inst.n_fluid * subs
        else:
            ref.prime()
            t0 = time.perf_counter()
            ref.step(nsteps)
            secs += time.perf_counter() - t0
            updates += inst.n_fluid * nsteps
        del ref
    return updates / secs / 1e6, O.num_threads(), secs, updates


def roofline(args, case, sim, h, stages, precision, skin_h):
    """Roofline of the dominant kernel of a leg: algorithmic FLOPs per launch
    over its average HIP-event duration, against the vector peak of the
    precision it computes in."""
    if not stages:
        return None
    name, (ms, n) = max(stages.items(), key=lambda kv: kv[1][0])
    avg_s = ms / n / 1e3
    dim = case.dim
    pairs = float(h["diag"][:, 12].sum())
    peak = FP64_VALU_PEAK_TFLOPS if precision == "fp64" else FP32_VALU_PEAK_TFLOPS
    key = precision + ("_skin" if skin_h else "")
    if name in ("sub_pressure", "sub_density"):
        # a sub-step sweep walks the pairs of the advection step's list
        flops = FLOPS_DUAL[dim][name] * pairs
        achieved = flops / avg_s / 1e12
        key = "dual" + ("_skin" if skin_h else "")
        roof = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                "traffic": load_traffic(args.case, key, name),
                "flops_per_launch": float(flops), "pairs": float(pairs), "avg_ms": round(avg_s * 1e3, 4)}
    elif name in ("build", "density", "force"):
        cands = 0
        if name == "build":
            # the candidate tests of the list build, on build steps only
            # (every step without a skin); the sweeps walk the lists
            cands = candidate_count(sim, h)
            flops = FLOPS[dim]["cand"] * cands * (sim.timed_builds / args.steps)
        else:
            flops = FLOPS[dim][name] * pairs
        achieved = flops / avg_s / 1e12
        traffic = load_traffic(args.case, key, name)
        if name == "build":
            # the candidate tests are FP32 arithmetic on both paths
            peak = FP32_VALU_PEAK_TFLOPS
        roof = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "peak_kind": "FP32 vector (packed)" if peak == FP32_VALU_PEAK_TFLOPS else "FP64 vector",
                "traffic": traffic, "flops_per_launch": float(flops),
                "candidates": int(cands), "pairs": float(pairs), "avg_ms": round(avg_s * 1e3, 4)}
        if traffic:
            roof["hbm_gbs"] = round(traffic / avg_s / 1e9, 1)
    else:
        return {"bound": "hbm", "kernel": name, "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": None, "avg_ms": round(avg_s * 1e3, 4)}
    # what bounds the list walks: L1 tag lookups (about one cache access per
    # clock per CU) and VALU issue (one wave64 instruction per clock per CU,
    # FP64 and FP32 alike without packed math)
    acc = load_l1(args.case, key, name)
    if acc:
        per = acc / (avg_s * CLOCK_HZ * N_CU)
        roof["l1"] = {"accesses_per_launch": acc, "per_clock_per_cu": round(per, 3),
                      "ceiling_per_clock_per_cu": 1.0, "frac": round(per, 3)}
    for unit in ("valu", "salu"):
        vi = load_valu(args.case, key, name, unit)
        if vi:
            per = vi / (avg_s * CLOCK_HZ * N_CU)
            roof[unit + "_issue"] = {"insts_per_launch": vi, "per_clock_per_cu": round(per, 3),
                                     "ceiling_per_clock_per_cu": 1.0, "frac": round(per, 3)}
    return roof


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--case", default="c5_3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=("fp64", "mixed"))
    ap.add_argument("--scheme", default="wcsph", choices=("wcsph", "dual"),
                    help="dual: dual-criteria Riemann scheme (steps are advection steps, "
                         "updates are acoustic sub-steps)")
    ap.add_argument("--compare", default="fp64", choices=("mixed", "fp64", "none"),
                    help="second precision timed on the same workload (its state after the "
                         "run is the reference of the error statement)")
    ap.add_argument("--graph", action="store_true", help="replay captured HIP graphs")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--build", type=int, default=None, choices=(0, 1, 2),
                    help="list build: 1 lane per target, 2 cell pairs, 0 the library's default "
                         "(default: tuned, else 0)")
    ap.add_argument("--no-tuned", action="store_true",
                    help="ignore the autotuner's cache for launch parameters left unset")
    ap.add_argument("--list", type=int, default=0, help="neighbour-list capacity (-1: no list)")
    ap.add_argument("--prefetch", type=int, default=0, help="candidate records in flight (4 or 8)")
    ap.add_argument("--reorder-every", type=int, default=None)
    ap.add_argument("--skin", type=float, default=0.0,
                    help="Verlet skin of the headline, in units of h (0: the cell table and "
                         "the neighbour lists are rebuilt every step)")
    ap.add_argument("--skin-leg", type=float, default=0.1,
                    help="also time the headline precision with this skin (units of h; 0: skip)")
    ap.add_argument("--key-order", default="row", choices=("row", "morton"),
                    help="cell keys: row-major, or tiles of 8^d cells in Morton order")
    ap.add_argument("--cpu-steps", type=int, default=-1,
                    help="oracle steps of the CPU sample (0: skip; -1: about 15 s of work)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (PMC calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path "
              "here is single-GPU and multi-GPU sharding is not built", file=sys.stderr)
        return 2

    import torch
    import dambreak

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.scheme == "dual":
        args.compare = "none"          # the dual scheme runs in FP64 only
        args.precision = "fp64"
    case = dambreak.make_case(args.case)
    n_fluid = case.n_fluid
    log(f"case {args.case}: {n_fluid} fluid, {case.n_wall} wall; {args.precision}; "
        f"skin {args.skin} h; steps {args.steps} warmup {args.warmup}")

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 8
        a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    common = dict(reorder_every=args.reorder_every, block=args.block, list_cap=args.list,
                  prefetch=args.prefetch, scheme=args.scheme, key_order=args.key_order,
                  stage_steps=min(args.steps, 50), tuned=not args.no_tuned, build=args.build)
    sim, h, secs, stages, flags = run_gpu(case, args.precision, args.steps, args.warmup,
                                          args.graph, timing=not args.graph,
                                          skin_h=args.skin, **common)
    updates = sim.timed_substeps if args.scheme == "dual" else args.steps
    value = n_fluid * updates / secs / 1e6
    log(f"{args.precision}: {secs * 1e3 / args.steps:.3f} ms/step, {value:.1f} M updates/s, "
        f"{sim.timed_builds} builds, flags {flags}")
    for k, (ms, n) in stages.items():
        if n:
            log(f"  {k:12s} {ms / n * 1e3:9.1f} us x {n}")
    roof = roofline(args, case, sim, h, stages, args.precision, args.skin)
    stage_us = {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages.items() if n}
    cons = drift(case, sim.info.mass, sim.diag0, sim.diag1)
    state_head = {"x": h["x"], "v": h["v"], "rho": h["rho"], "id": h["id"]}
    mass = float(sim.info.mass)
    tuned_params = sim.tuned
    launch = {"block_threads": int(sim.params.block_threads) or 256, "build": int(sim.params.build),
              "prefetch": int(sim.params.prefetch) or 8}
    timed_builds = sim.timed_builds
    sweeps_timed = sim.sweeps_timed
    sim_time = cons["sim_time_s"]
    ms_step = secs * 1e3 / args.steps
    sim.close()
    del sim, h
    torch.cuda.empty_cache()

    other = None
    if args.compare != "none" and args.compare != args.precision:
        sim2, h2, secs2, stages2, flags2 = run_gpu(case, args.compare, args.steps, args.warmup,
                                                   args.graph, timing=not args.graph,
                                                   skin_h=args.skin, **common)
        v2 = n_fluid * args.steps / secs2 / 1e6
        # the FP64 run is the reference of the mixed run (either way round)
        if args.compare == "fp64":
            err = state_errors(case, mass, state_head, h2)
        else:
            err = state_errors(case, mass, h2, state_head)
        other = {
            "precision": args.compare, "value": round(v2, 2),
            "ms_per_step": round(secs2 * 1e3 / args.steps, 4),
            "headline_speedup": round(value / v2, 3),
            "cell_builds": int(sim2.timed_builds),
            "stage_us": {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages2.items() if n},
            "roofline": roofline(args, case, sim2, h2, stages2, args.compare, args.skin),
            "mixed_vs_fp64_after_run": err,
            "steps_compared": args.warmup + args.steps,
            "flags": int(flags2),
        }
        log(f"{args.compare}: {secs2 * 1e3 / args.steps:.3f} ms/step, {v2:.1f} M updates/s; "
            f"mixed vs fp64: {err['probe']} E {err['energy_rel_ke']}")
        sim2.close()
        del sim2, h2
        torch.cuda.empty_cache()

    skin_leg = None
    if args.skin_leg > 0 and args.skin_leg != args.skin:
        # the same precision with a Verlet skin: cells and lists reused until
        # the particles may have moved half the skin (builds decided on the device)
        sim3, h3, secs3, stages3, flags3 = run_gpu(case, args.precision, args.steps, args.warmup,
                                                   args.graph, timing=not args.graph,
                                                   skin_h=args.skin_leg, **common)
        upd3 = sim3.timed_substeps if args.scheme == "dual" else args.steps
        v3 = n_fluid * upd3 / secs3 / 1e6
        skin_leg = {"skin_h": args.skin_leg, "value": round(v3, 3),
                    "ms_per_step": round(secs3 * 1e3 / args.steps, 4),
                    "cell_builds": int(sim3.timed_builds),
                    "stage_us": {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages3.items() if n},
                    "flags": int(flags3)}
        log(f"{args.precision} with a {args.skin_leg} h skin: {secs3 * 1e3 / args.steps:.3f} ms/step, "
            f"{v3:.1f} M updates/s, {sim3.timed_builds} builds")
        sim3.close()
        del sim3, h3
        torch.cuda.empty_cache()

    cpu = None
    cpu_steps = args.cpu_steps
    if cpu_steps < 0:
        # about 15 s of oracle work at ~3.5 M updates/s
        cpu_steps = max(1, int(round(5e7 / max(n_fluid, 1))))
        cpu_steps = min(cpu_steps, 100)
    if cpu_steps > 0:
        cv, cores, csecs, cupd = cpu_baseline(case, cpu_steps, args.scheme)
        what = "advection steps (their acoustic sub-steps counted)" if args.scheme == "dual" else "full steps"
        cpu = {"value": round(cv, 4), "unit": "M particle-updates/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{args.case}: FP64 CPU reference, {cpu_steps} {what} after the prime, "
                         f"every instance, all {n_fluid} fluid particles ({cupd} particle updates, "
                         f"{csecs:.1f} s timed)"}
        log(f"cpu oracle: {cv:.3f} M updates/s on {cores} threads ({csecs:.1f} s)")

    dtype = "f64" if args.precision == "fp64" else "f32+f64"
    hbm = None
    step_traffic = load_step_traffic(args.case, args.precision + ("_skin" if args.skin else ""))
    if step_traffic:
        hbm = {"bytes_per_step": step_traffic, "achieved_gbs": round(step_traffic / (ms_step / 1e3) / 1e9, 1),
               "peak_gbs": HBM_PEAK_GBS,
               "frac": round(step_traffic / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
               "source": "rocprofv3 FETCH_SIZE/WRITE_SIZE of every kernel of a step (profiles/)"}
    extra = {"sim_seconds_per_second": (round(sim_time / secs, 6) if sim_time else None),
             "cell_builds": int(timed_builds),
             "conservation": cons,
             "stage_timing": ("pair sweeps: HIP events on the library stream in the timed steps; "
                              if sweeps_timed else "") +
                             f"other stages: HIP events on {min(args.steps, 50)} eager steps right after"}
    if args.scheme == "dual":
        # one update = one acoustic sub-step of one fluid particle
        extra["substeps"] = int(updates)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "M particle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": WORKLOADS[args.case], "case": args.case,
                   "precision": args.precision, "n_fluid": n_fluid, "n_wall": case.n_wall,
                   "reorder_every": case.reorder_every if args.reorder_every is None else args.reorder_every,
                   "graph": bool(args.graph), **launch, "tuned": tuned_params,
                   "list_cap": args.list, "scheme": args.scheme,
                   "skin_h": args.skin, "key_order": args.key_order},
        "roofline": roof, "hbm": hbm, "cpu_baseline": cpu, "stage_us": stage_us,
        "compare": other, "skin_leg": skin_leg, "flags": int(flags), **extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
