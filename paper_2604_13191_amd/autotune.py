"""Autotuner of the work decomposition: tile edge, unit budget and launch grids.

The voxelize pass bins primitives into leaf tiles of 2^tile_bits voxels per axis and hands tiles
(or octants of them) to work units that keep at most `unit_budget` candidates in LDS; the
streaming kernels stride over their work with a grid-sized loop.  None of these changes a
result (every voxel sums its pairs in primitive order whichever unit or block takes it), only
the time.  The tuner, for one workload:

  1. builds the path once per (tile_bits, unit_budget) pair with the default grids and times
     whole steps (voxelize + pyramid);
  2. with the fastest pair, runs the workload once per candidate grid (all tunable kernels at
     that grid), times each tunable kernel's own launches with the library's event timing and
     keeps, kernel by kernel, the fastest grid;
  3. times whole steps with the default tuning and with the tuned one.

The table is JSON, read-only for the library (the tuning travels with every call):

    {"device": ..., "tables": {workload: {"tuning": {...}, "step_ms": {"default": .., "tuned": ..},
                                          "decomposition_ms": {...}, "kernel_ms": {...}}}}

    python -m paper_2604_13191_amd.autotune --workload brushed_metal   (needs a GPU)
"""
from __future__ import annotations

import argparse
import json
import os
import time

import paper_2604_13191_amd as vx

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tunings.json")
TILE_BITS = (3, 4)
BUDGETS = (1024, 1536, 2048, 3072)
GRIDS = (256, 512, 1024, 2048, 4096, 8192, 16384)


def _time_steps(run, reps):
    import torch
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune(make_run, reps=3, tile_bits=TILE_BITS, budgets=BUDGETS, grids=GRIDS):
    """make_run(tuning) -> run(): plans built for `tuning`, run() enqueues one step.
    Returns (best Tuning, report dict)."""
    import torch
    decomposition = {}
    best, best_ms = None, None
    for tb in tile_bits:
        for b in budgets:
            t = vx.Tuning(tile_bits=tb, unit_budget=b)
            run = make_run(t)
            ms = _time_steps(run, reps)
            del run
            torch.cuda.empty_cache()
            decomposition[f"{tb}/{b}"] = round(ms, 4)
            if best_ms is None or ms < best_ms:
                best, best_ms = t, ms
    # grids, kernel by kernel, with the chosen decomposition
    times = {k: {} for k in vx.TUNE_KERNELS}
    for g in grids:
        t = vx.Tuning(best.tile_bits, best.unit_budget, (g,) * len(vx.TUNE_KERNELS))
        run = make_run(t)
        run()
        torch.cuda.synchronize()
        vx.timing_reset()
        vx.timing_filter(None)
        vx.timing_enable(True)
        try:
            for _ in range(reps):
                run()
        finally:
            vx.timing_enable(False)
        kt = vx.timing_collect()
        for k in vx.TUNE_KERNELS:
            names = ("unit_tri", "unit_fib") if k == "unit" else (k, k + "_up") if k == "lod_cluster" else (k,)
            ms = sum(kt[n][0] for n in names if n in kt)
            if any(n in kt for n in names):
                times[k][g] = ms / reps
        del run
        torch.cuda.empty_cache()
    chosen = tuple(min(times[k], key=times[k].get) if times[k] else 0 for k in vx.TUNE_KERNELS)
    tuned = vx.Tuning(best.tile_bits, best.unit_budget, chosen)
    run = make_run(None)
    default_ms = _time_steps(run, reps)
    del run
    run = make_run(tuned)
    tuned_ms = _time_steps(run, reps)
    del run
    torch.cuda.empty_cache()
    report = {"tuning": tuned.as_dict(), "step_ms": {"default": round(default_ms, 4), "tuned": round(tuned_ms, 4)},
              "decomposition_ms": decomposition,
              "kernel_ms": {k: {str(g): round(v, 4) for g, v in t.items()} for k, t in times.items()},
              "candidates": {"tile_bits": list(tile_bits), "unit_budget": list(budgets), "grids": list(grids)}}
    return tuned, report


def save(workload, report, path=TABLE):
    import torch
    table = {"device": torch.cuda.get_device_name(0), "tables": {}}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table["tables"][workload] = report
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load(workload, path=TABLE):
    """The tuned decomposition of `workload` as a vx.Tuning, or None when it was never tuned."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get("tables", {}).get(workload)
    if not t:
        return None
    return vx.Tuning.from_dict(t["tuning"])


def _runner(name):
    """make_run(tuning) for the named workload (inputs generated once)."""
    import torch
    import synth
    if name == "weave_patches":
        wls = synth.weave_patches()
        patches = [vx.Patch(w.grid, torch.as_tensor(w.pts).cuda(), torch.as_tensor(w.offsets), w.radius) for w in wls]

        def make(t):
            plan = vx.BatchPlan(patches, K=4, iters=2, tuning=t)
            return plan.run
        return make
    if name in ("plain_weave", "brushed_metal"):
        if name == "plain_weave":
            wl = synth.plain_weave()
            data = torch.as_tensor(wl.pts).cuda()
            offs = torch.as_tensor(wl.offsets).cuda()
            kind, K = 1, 1
        else:
            wl = synth.brushed_metal()
            data = torch.as_tensor(wl.tris).cuda()
            offs, kind, K = None, 0, 4

        def make(t):
            plan = vx.VoxelizePlan(kind, wl.grid, data, offsets=offs, radius=wl.radius if kind else 0.0, tuning=t)
            plan.run()
            leaf = plan.check()
            cal = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], wl.levels, tuning=t).run()
            caps = [max(v.n, 1) for v in cal.check()[1:]]
            del cal
            lod = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], wl.levels, K=K, iters=2, caps=caps, tuning=t)
            return lambda: (plan.run(), lod.run())
        return make
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="brushed_metal", choices=["brushed_metal", "plain_weave", "weave_patches"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    make = _runner(args.workload)
    tuned, report = tune(make, reps=args.reps)
    save(args.workload, report, args.out)
    print(json.dumps({"workload": args.workload, **report}), flush=True)


if __name__ == "__main__":
    main()
