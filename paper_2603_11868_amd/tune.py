"""Autotuner for the launch parameters of the hot path.

Searches threads per sweep block, the neighbour-list build (cell pairs, or one
lane per target), the number of candidate records in flight per thread of the
lane-per-target build, the neighbour-list capacity (default, or plain direct
search in both sweeps), and optionally the reorder period K (how often the
state arrays are physically re-sorted by cell; it changes results only through
summation order), the Verlet skin (in units of h) and the cell key order.
By default the window is the benchmark's: the workload's own K, no skin, so
that every timed step builds its cell table and lists.  A skin pays off
through the builds it saves, and how many it saves depends on the flow speed:
time it on steps that are representative of the run (a window of a few steps
from rest saves every build and favours large skins).
Each variant runs whole steps through the C ABI and is timed with HIP events
on the stream; the fastest is cached in a JSON file keyed by
(arch, dim, precision, particle-count bucket), which Simulation(tuned=True)
and the benchmark read.

Command line:  python -m paper_2603_11868_amd.tune --case c5_3d --precision mixed
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import time

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
BLOCKS = (64, 128, 256)
BUILDS = (1, 2)
LISTS = (0,)
PREFETCHES = (4, 8)
REORDERS = ()            # empty: the workload's own K
SKINS = (0.0,)
KEY_ORDERS = ("row",)


def cache_key(arch, dim, precision, n_fluid):
    bucket = int(math.log2(max(n_fluid, 1)))
    return f"{arch}/d{dim}/{precision}/n2^{bucket}"


def time_variant(case, precision, block, list_cap, prefetch, reorder, steps, warmup, skin_h=0.0,
                 key_order="row", build=0):
    import torch
    from .sph import Simulation

    sim = Simulation(case, precision=precision, block_threads=block, list_cap=list_cap,
                     prefetch=prefetch, reorder_every=reorder, skin=skin_h * case.h,
                     key_order=key_order, build=build)
    try:
        sim.prime()
        sim.step(warmup)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        sim.step(steps)
        stop.record()
        torch.cuda.synchronize()
        flags = sim.poll_errors()
        return start.elapsed_time(stop) / steps, flags
    finally:
        sim.close()


def tune(case, precision="fp64", steps=20, warmup=3, blocks=BLOCKS, lists=LISTS,
         prefetches=PREFETCHES, reorders=REORDERS, cache_path=DEFAULT_CACHE, log=print,
         skins=SKINS, key_orders=KEY_ORDERS, builds=BUILDS):
    """Time every variant; return the fastest as a dict and store it."""
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    reorders = tuple(reorders) or (case.reorder_every,)
    results = []
    for block, bld, lst, pf, reorder, sk, ko in itertools.product(blocks, builds, lists, prefetches, reorders,
                                                                  skins, key_orders):
        if lst < 0 and (pf != prefetches[0] or bld != builds[0]):
            continue          # direct search has no list to build
        if bld == 2 and pf != prefetches[0] and ko == "row":
            continue          # the cell-pair build does not prefetch candidates
        ms, flags = time_variant(case, precision, block, lst, pf, reorder, steps, warmup, sk, ko, bld)
        results.append({"block_threads": block, "build": bld, "list_cap": lst, "prefetch": pf,
                        "reorder_every": reorder, "skin_h": sk, "key_order": ko,
                        "ms_per_step": round(ms, 5), "flags": flags})
        if log:
            log(f"  block {block:3d} build {bld} list {lst:3d} prefetch {pf} K {reorder:3d} "
                f"skin {sk:4.2f}h keys {ko}: {ms:8.4f} ms/step")
    ok = [r for r in results if r["flags"] == 0]
    best = min(ok or results, key=lambda r: r["ms_per_step"])
    key = cache_key(arch, case.dim, precision, case.n_fluid)
    entry = {"best": best, "case": case.name, "n_fluid": case.n_fluid, "steps": steps,
             "when": time.strftime("%Y-%m-%d %H:%M:%S"), "all": results}
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = entry
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return entry


def lookup(case, precision, arch="gfx950", cache_path=DEFAULT_CACHE):
    """Cached best launch parameters for a workload, or None."""
    if not os.path.exists(cache_path):
        return None
    with open(cache_path) as f:
        cache = json.load(f)
    e = cache.get(cache_key(arch, case.dim, precision, case.n_fluid))
    return e["best"] if e else None


def main(argv=None):
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import dambreak

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--case", default="c2_3d")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "mixed"))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--blocks", default=",".join(map(str, BLOCKS)))
    ap.add_argument("--builds", default=",".join(map(str, BUILDS)), help="1 lane per target, 2 cell pairs")
    ap.add_argument("--prefetches", default=",".join(map(str, PREFETCHES)))
    ap.add_argument("--reorders", default="", help="reorder periods (default: the workload's)")
    ap.add_argument("--lists", default=",".join(map(str, LISTS)))
    ap.add_argument("--skins", default=",".join(map(str, SKINS)), help="Verlet skins in units of h")
    ap.add_argument("--key-orders", default=",".join(KEY_ORDERS), help="row and/or morton")
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    case = dambreak.make_case(args.case)
    ints = lambda s: tuple(int(v) for v in s.split(",") if v)
    e = tune(case, args.precision, args.steps, args.warmup, ints(args.blocks), ints(args.lists),
             ints(args.prefetches), ints(args.reorders), args.cache,
             skins=tuple(float(v) for v in args.skins.split(",")),
             key_orders=tuple(args.key_orders.split(",")), builds=ints(args.builds))
    print(json.dumps({"case": args.case, "precision": args.precision, "best": e["best"]}))


if __name__ == "__main__":
    main()
