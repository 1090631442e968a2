"""Autotuner for the launch parameters of the hot path.

Searches threads per sweep block, the neighbour-list capacity (default, or
plain direct search in both sweeps), the number of candidate records in
flight per thread of the density sweep, and the reorder period K (how often the
state arrays are physically re-sorted by cell; the cell table itself is
rebuilt every step, so K changes results only through summation order), and
the Verlet skin (in units of h) and the cell key order.  A skin pays off through the builds it saves,
and how many it saves depends on the flow speed: time it on steps that are
representative of the run (a window of a few steps from rest saves every
build and favours large skins).
Each variant runs whole steps through the C ABI and is timed with HIP events
on the stream; the fastest is cached in a JSON file keyed by
(arch, dim, precision, particle-count bucket).

Command line:  python -m paper_2603_11868_amd.tune --case c2_3d --precision fp64
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
LISTS = (0, -1)
PREFETCHES = (4, 8)
REORDERS = (1, 5, 20, 50)
SKINS = (0.0, 0.1)
KEY_ORDERS = ("row",)


def cache_key(arch, dim, precision, n_fluid):
    bucket = int(math.log2(max(n_fluid, 1)))
    return f"{arch}/d{dim}/{precision}/n2^{bucket}"


def time_variant(case, precision, block, list_cap, prefetch, reorder, steps, warmup, skin_h=0.0,
                 key_order="row"):
    import torch
    from .sph import Simulation

    sim = Simulation(case, precision=precision, block_threads=block, list_cap=list_cap,
                     prefetch=prefetch, reorder_every=reorder, skin=skin_h * case.h,
                     key_order=key_order)
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
         skins=SKINS, key_orders=KEY_ORDERS):
    """Time every variant; return the fastest as a dict and store it."""
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    results = []
    for block, lst, pf, reorder, sk, ko in itertools.product(blocks, lists, prefetches, reorders, skins,
                                                             key_orders):
        if lst < 0 and pf != prefetches[0]:
            continue          # direct search has no list to prefetch for
        ms, flags = time_variant(case, precision, block, lst, pf, reorder, steps, warmup, sk, ko)
        results.append({"block_threads": block, "list_cap": lst, "prefetch": pf,
                        "reorder_every": reorder, "skin_h": sk, "key_order": ko,
                        "ms_per_step": round(ms, 5), "flags": flags})
        if log:
            log(f"  block {block:3d} list {lst:3d} prefetch {pf} K {reorder:3d} skin {sk:4.2f}h "
                f"keys {ko}: {ms:8.4f} ms/step")
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
    ap.add_argument("--prefetches", default=",".join(map(str, PREFETCHES)))
    ap.add_argument("--reorders", default=",".join(map(str, REORDERS)))
    ap.add_argument("--lists", default=",".join(map(str, LISTS)))
    ap.add_argument("--skins", default=",".join(map(str, SKINS)), help="Verlet skins in units of h")
    ap.add_argument("--key-orders", default=",".join(KEY_ORDERS), help="row and/or morton")
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    args = ap.parse_args(argv)
    case = dambreak.make_case(args.case)
    ints = lambda s: tuple(int(v) for v in s.split(","))
    e = tune(case, args.precision, args.steps, args.warmup, ints(args.blocks), ints(args.lists),
             ints(args.prefetches), ints(args.reorders), args.cache,
             skins=tuple(float(v) for v in args.skins.split(",")),
             key_orders=tuple(args.key_orders.split(",")))
    print(json.dumps({"case": args.case, "precision": args.precision, "best": e["best"]}))


if __name__ == "__main__":
    main()
