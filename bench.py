"""Throughput of the WCSPH step on one MI355X.

Default workload: the 3D dam break of 2.0 M fluid particles (1 x 1 x 2 m block
at dx = 0.01 in a 4 x 1 x 3 m box, 1.17 M wall particles), plain FP64 path,
arrays re-sorted by cell every 20 steps, 500 timed steps.  A step is the whole
hot path: half kick + drift + cell keys, cell scan, radix sort, (reorder),
sweep records, density sweep, force sweep fused with the second half kick,
and the FP64 reductions for dt and the diagnostics.  By default the cell
table and the neighbour lists carry a Verlet skin of 0.1 h: the device
rebuilds them only when the particles may have moved half the skin (the
number of builds in the timed steps is reported), and the same steps are
timed again without a skin.

Prints one JSON line.  Besides the headline value it reports the roofline of
the dominant kernel (algorithmic FLOPs per launch over its HIP-event time in
the timed steps; only the pair sweeps carry events there, the other stages are
timed on 50 steps right after),
the same workload on the mixed-precision path, and the CPU reference timed on
a bounded sample of the same workload.
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
HBM_PEAK_GBS = 8000.0
SWEEP_STAGES = ("density", "force", "sub_pressure", "sub_density")
CLOCK_HZ, N_CU = 2.4e9, 256

# FP64 flops per candidate test and per neighbour pair (viscosity excluded:
# it runs on approaching pairs only, so leaving it out keeps the count a
# lower bound).  Candidate: r = x_i - x_j, r^2.  Density pair: sqrt, q, t,
# t^3, W, F, v_ij.r, two accumulations.  Force pair: sqrt, q, t, t^3, F,
# v_ij.r, (P_i + P_j) F, two vector accumulations.
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
    for name in ("sph_sweeps.hip", "sph_step_common.h", "sph_device.h"):
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


def load_valu(workload, precision, kernel):
    """VALU instructions (wave64) per launch of a sweep from a committed
    rocprofv3 summary taken on the current kernel sources (else None)."""
    import re
    path = os.path.join(ROOT, "profiles", f"valu_{workload}_{precision}_sq.md")
    if not os.path.exists(path):
        return None
    val, hsh = None, None
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+) valu_insts_per_launch: ([0-9.e+-]+)", line)
            if m and m.group(1) == kernel:
                val = float(m.group(2))
            m = re.match(r"^- source_hash: `([0-9a-f]+)`", line)
            if m:
                hsh = m.group(1)
    return val if hsh == kernel_source_hash() else None


def run_gpu(case, precision, steps, warmup, graph, timing, reorder_every=None, block=0,
            list_cap=0, prefetch=0, stage_steps=0, scheme="wcsph", skin_h=0.0, key_order="row"):
    import torch
    from paper_2603_11868_amd import sph

    sim = sph.Simulation(case, precision=precision, reorder_every=reorder_every,
                         use_graph=graph, block_threads=block,
                         list_cap=list_cap, prefetch=prefetch, scheme=scheme,
                         skin=skin_h * case.h, key_order=key_order)
    sim.key_order = key_order
    sim.prime()
    sim.step(warmup)
    torch.cuda.synchronize()
    sub0 = int(sph.sph_get_info(sim.ctx).substeps_done)
    builds0 = sim.cell_builds()
    tsim0 = sim.host()["diag"][:, 14].copy()
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
    tsim1 = sim.host()["diag"][:, 14].copy()
    sub1 = int(sph.sph_get_info(sim.ctx).substeps_done)
    sim.timed_builds = sim.cell_builds() - builds0
    sweeps = sph.sph_stage_times(sim.ctx, reset=True) if timing else {}
    sph.sph_set_timing(sim.ctx, 0)
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
    h = sim.host()
    sim.timed_substeps = sub1 - sub0
    # simulated seconds advanced in the timed region (mean over instances)
    sim.timed_sim_time = float(np.mean(tsim1 - tsim0))
    return sim, h, t1 - t0, stages, flags


def cpu_baseline(case, nsteps, scheme="wcsph"):
    """The CPU reference on the same workload: M updates/s over nsteps steps
    (dual scheme: advection steps, counted in acoustic sub-steps)."""
    from oracle import oracle as O

    ref = O.OracleSim.from_case(case)
    if scheme == "dual":
        ref.dual_prime()
        t0 = time.perf_counter()
        subs = 0
        for _ in range(nsteps):
            subs += ref.dual_plan()[1]
            ref.dual_step(1)
        t1 = time.perf_counter()
        return ref, case.n_fluid * subs / (t1 - t0) / 1e6, O.num_threads(), t1 - t0
    ref.prime()
    t0 = time.perf_counter()
    ref.step(nsteps)
    t1 = time.perf_counter()
    return ref, case.n_fluid * nsteps / (t1 - t0) / 1e6, O.num_threads(), t1 - t0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--case", default="c2_3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--scheme", default="wcsph", choices=("wcsph", "dual"),
                    help="dual: dual-criteria Riemann scheme (steps are advection steps, "
                         "updates are acoustic sub-steps)")
    ap.add_argument("--compare", default="mixed", choices=("mixed", "fp64", "none"),
                    help="second precision timed on the same workload")
    ap.add_argument("--graph", action="store_true", help="replay captured HIP graphs")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--list", type=int, default=0, help="neighbour-list capacity (-1: no list)")
    ap.add_argument("--prefetch", type=int, default=0, help="candidate records in flight (4 or 8)")
    ap.add_argument("--reorder-every", type=int, default=None)
    ap.add_argument("--skin", type=float, default=None,
                    help="Verlet skin in units of h (0: cells and lists rebuilt every step; "
                         "default 0.1, and 0 for the dual scheme)")
    ap.add_argument("--key-order", default="row", choices=("row", "morton"),
                    help="cell keys: row-major, or tiles of 8^d cells in Morton order")
    ap.add_argument("--no-skin-leg", action="store_true",
                    help="skip the second timing of the headline path without a skin")
    ap.add_argument("--cpu-steps", type=int, default=8, help="oracle steps of the CPU sample (0: skip)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (PMC calibration)")
    args = ap.parse_args(argv)

    if args.skin is None:
        args.skin = 0.0 if args.scheme == "dual" else 0.1
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path "
              "here is single-GPU and multi-GPU sharding is not built", file=sys.stderr)
        return 2

    import torch
    import dambreak

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    case = dambreak.make_case(args.case)
    n_fluid = case.n_fluid
    log(f"case {args.case}: {n_fluid} fluid, {case.n_wall} wall; {args.precision}; "
        f"steps {args.steps} warmup {args.warmup}")

    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 8
        a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    sim, h, secs, stages, flags = run_gpu(case, args.precision, args.steps, args.warmup,
                                          args.graph, timing=not args.graph,
                                          stage_steps=min(args.steps, 50),
                                          reorder_every=args.reorder_every, block=args.block,
                                          list_cap=args.list,
                                          prefetch=args.prefetch, scheme=args.scheme,
                                          skin_h=args.skin, key_order=args.key_order)
    updates = sim.timed_substeps if args.scheme == "dual" else args.steps
    sim_time = sim.timed_sim_time
    value = n_fluid * updates / secs / 1e6
    log(f"{args.precision}: {secs * 1e3 / args.steps:.3f} ms/step, {value:.1f} M updates/s, flags {flags}")
    for k, (ms, n) in stages.items():
        if n:
            log(f"  {k:12s} {ms / n * 1e3:9.1f} us x {n}")

    # roofline of the dominant kernel
    roof = None
    if stages:
        name, (ms, n) = max(stages.items(), key=lambda kv: kv[1][0])
        avg_s = ms / n / 1e3
        dim = case.dim
        pairs = float(h["diag"][:, 12].sum())
        cands = candidate_count(sim, h)
        if name in ("sub_pressure", "sub_density"):
            # a sub-step sweep walks the pairs of the advection step's list
            flops = FLOPS_DUAL[dim][name] * pairs
            achieved = flops / avg_s / 1e12
            roof = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                    "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                    "traffic": load_traffic(args.case, "dual" + ("_skin" if args.skin else ""), name),
                    "flops_per_launch": float(flops), "pairs": float(pairs), "avg_ms": round(avg_s * 1e3, 4)}
            vi = load_valu(args.case, "dual" + ("_skin" if args.skin else ""), name)
            if vi:
                per = vi / (avg_s * CLOCK_HZ * N_CU)
                roof["valu_issue"] = {"insts_per_launch": vi, "per_clock_per_cu": round(per, 3),
                                      "ceiling_per_clock_per_cu": 1.0, "frac": round(per, 3)}
        elif name in ("density", "force"):
            # with a skin the candidates are tested at builds only
            build_frac = sim.timed_builds / args.steps
            flops = FLOPS[dim]["cand"] * cands * build_frac + FLOPS[dim][name] * pairs
            achieved = flops / avg_s / 1e12
            traffic = load_traffic(args.case, args.precision + ("_skin" if args.skin else ""), name)
            roof = {"bound": "alu", "kernel": name, "achieved": round(achieved, 3),
                    "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                    "traffic": traffic, "flops_per_launch": float(flops),
                    "candidates": int(cands), "pairs": float(pairs), "avg_ms": round(avg_s * 1e3, 4)}
            if traffic:
                roof["hbm_gbs"] = round(traffic / avg_s / 1e9, 1)
            # what bounds the list walks: L1 tag lookups, about one cache
            # access per clock per CU at most
            key = args.precision + ("_skin" if args.skin else "")
            acc = load_l1(args.case, key, name)
            if acc:
                per = acc / (avg_s * CLOCK_HZ * N_CU)
                roof["l1"] = {"accesses_per_launch": acc, "per_clock_per_cu": round(per, 3),
                              "ceiling_per_clock_per_cu": 1.0, "frac": round(per, 3)}
            # VALU issue: a CU issues at most one wave64 VALU instruction per
            # clock (4 SIMDs, 4 clocks each); FP64 and FP32 alike here
            vi = load_valu(args.case, key, name)
            if vi:
                per = vi / (avg_s * CLOCK_HZ * N_CU)
                roof["valu_issue"] = {"insts_per_launch": vi, "per_clock_per_cu": round(per, 3),
                                      "ceiling_per_clock_per_cu": 1.0, "frac": round(per, 3)}
        else:
            roof = {"bound": "hbm", "kernel": name, "achieved": None, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": None, "traffic": None, "avg_ms": round(avg_s * 1e3, 4)}
    stage_us = {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages.items() if n}
    state_fp = {"x": h["x"], "v": h["v"], "rho": h["rho"], "id": h["id"]}
    timed_builds = sim.timed_builds
    sweeps_timed = sim.sweeps_timed
    sim.close()
    del sim
    torch.cuda.empty_cache()

    other = None
    if args.scheme == "dual":
        args.compare = "none"          # the dual scheme runs in FP64 only
    if args.compare != "none" and args.compare != args.precision:
        sim2, h2, secs2, stages2, flags2 = run_gpu(case, args.compare, args.steps, args.warmup,
                                                   args.graph, timing=not args.graph,
                                                   stage_steps=min(args.steps, 50),
                                                   reorder_every=args.reorder_every,
                                                   block=args.block,
                                                   list_cap=args.list, prefetch=args.prefetch,
                                                   skin_h=args.skin, key_order=args.key_order)
        v2 = n_fluid * args.steps / secs2 / 1e6
        # difference between the two precisions after the same steps, by particle id
        def by_id(st):
            out = {}
            for k in ("x", "v", "rho"):
                arr = np.empty_like(st[k])
                arr[st["id"]] = st[k]
                out[k] = arr
            return out
        a_, b_ = by_id(state_fp), by_id({"x": h2["x"], "v": h2["v"], "rho": h2["rho"], "id": h2["id"]})
        other = {
            "precision": args.compare, "value": round(v2, 2),
            "ms_per_step": round(secs2 * 1e3 / args.steps, 4),
            "ratio_vs_headline": round(v2 / value, 3),
            "stage_us": {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages2.items() if n},
            "diff_vs_headline_after_run": {
                "rho_rel": float(np.abs(a_["rho"] - b_["rho"]).max() / case.rho0),
                "v_rel": float(np.abs(a_["v"] - b_["v"]).max() / max(np.abs(a_["v"]).max(), 1e-300)),
                "x_abs_over_dx": float(np.abs(a_["x"] - b_["x"]).max() / case.dx),
            },
            "flags": int(flags2),
        }
        log(f"{args.compare}: {secs2 * 1e3 / args.steps:.3f} ms/step, {v2:.1f} M updates/s")
        sim2.close()
        del sim2
        torch.cuda.empty_cache()

    no_skin = None
    if args.skin > 0 and not args.no_skin_leg:
        # the same steps with the cell table and lists rebuilt every step
        sim3, h3, secs3, stages3, flags3 = run_gpu(case, args.precision, args.steps, args.warmup,
                                                   args.graph, timing=not args.graph,
                                                   stage_steps=min(args.steps, 50),
                                                   reorder_every=args.reorder_every,
                                                   block=args.block, list_cap=args.list,
                                                   prefetch=args.prefetch, scheme=args.scheme,
                                                   skin_h=0.0, key_order=args.key_order)
        upd3 = sim3.timed_substeps if args.scheme == "dual" else args.steps
        v3 = n_fluid * upd3 / secs3 / 1e6
        no_skin = {"value": round(v3, 3), "ms_per_step": round(secs3 * 1e3 / args.steps, 4),
                   "stage_us": {k: round(ms / n * 1e3, 2) for k, (ms, n) in stages3.items() if n},
                   "flags": int(flags3)}
        log(f"{args.precision} without skin: {secs3 * 1e3 / args.steps:.3f} ms/step, {v3:.1f} M updates/s")
        sim3.close()
        del sim3
        torch.cuda.empty_cache()

    cpu = None
    if args.cpu_steps > 0:
        _, cv, cores, csecs = cpu_baseline(case, args.cpu_steps, args.scheme)
        what = "advection steps (their acoustic sub-steps counted)" if args.scheme == "dual" else "full steps"
        cpu = {"value": round(cv, 4), "unit": "M particle-updates/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{args.case}: FP64 CPU reference, prime + {args.cpu_steps} {what} "
                         f"of all {n_fluid} fluid particles ({csecs:.1f} s)"}
        log(f"cpu oracle: {cv:.3f} M updates/s on {cores} threads ({csecs:.1f} s)")

    dtype = "f64" if args.precision == "fp64" else "f32+f64"
    extra = {"sim_seconds_per_second": (round(sim_time / secs, 6) if sim_time else None),
             "cell_builds": int(timed_builds),
             "stage_timing": ("pair sweeps: HIP events on the library stream in the timed steps; "
                              if sweeps_timed else "") +
                             f"other stages: HIP events on {min(args.steps, 50)} eager steps right after"}
    if args.scheme == "dual":
        # one update = one acoustic sub-step of one fluid particle
        extra["substeps"] = int(updates)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "M particle-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(secs * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": WORKLOADS[args.case], "case": args.case,
                   "precision": args.precision, "n_fluid": n_fluid, "n_wall": case.n_wall,
                   "reorder_every": case.reorder_every if args.reorder_every is None else args.reorder_every,
                   "graph": bool(args.graph), "block_threads": args.block or 256,
                   "list_cap": args.list,
                   "prefetch": args.prefetch or 8, "scheme": args.scheme,
                   "skin_h": args.skin, "key_order": args.key_order},
        "roofline": roof, "cpu_baseline": cpu, "stage_us": stage_us,
        "compare": other, "no_skin": no_skin, "flags": int(flags), **extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
