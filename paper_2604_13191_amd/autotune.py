"""Autotuner for the launch grids of the persistent kernels.

Every streaming kernel of the path strides over its work with a grid-sized loop, so its grid
size (blocks of 256 threads) trades occupancy and tail balance against per-block overhead.  The
grid changes no result: each output element is computed the same way whichever block takes it.
The tuner runs a given workload once per candidate grid (all tunable kernels at that grid),
times each tunable kernel's own launches with the library's event timing, and keeps, kernel by
kernel, the fastest grid.  The table is JSON:

    {"device": ..., "tables": {workload: {"grids": [...], "kernel_ms": {...}, "candidates": [...]}}}

and ``apply(path, workload)`` loads it into the library (``vx_set_launch_grids``).

    python -m paper_2604_13191_amd.autotune --workload weave_patches   (needs a GPU)
"""
from __future__ import annotations

import argparse
import json
import os

import paper_2604_13191_amd as vx

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_grids.json")
CANDIDATES = (256, 512, 1024, 2048, 4096, 8192)


def tune(run, candidates=CANDIDATES, reps=3):
    """run(): enqueue one pass of the workload.  Returns (grids, {kernel: {grid: ms}})."""
    import torch
    default = vx.get_launch_grids()
    times = {k: {} for k in vx.TUNE_KERNELS}
    try:
        for c in candidates:
            vx.set_launch_grids([c] * len(vx.TUNE_KERNELS))
            run()
            torch.cuda.synchronize()
            vx.timing_reset()
            vx.timing_enable(True)
            for _ in range(reps):
                run()
            vx.timing_enable(False)
            kt = vx.timing_collect()
            for k in vx.TUNE_KERNELS:
                if k in kt:
                    times[k][c] = kt[k][0] / reps
    finally:
        vx.timing_enable(False)
        vx.set_launch_grids(default)
    grids = []
    for i, k in enumerate(vx.TUNE_KERNELS):
        t = times[k]
        grids.append(min(t, key=t.get) if t else default[i])
    return grids, times


def save(workload, grids, times, path=TABLE):
    import torch
    table = {"device": torch.cuda.get_device_name(0), "tables": {}}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table["tables"][workload] = {"grids": [int(g) for g in grids], "kernels": list(vx.TUNE_KERNELS),
                                 "kernel_ms": {k: {str(c): round(v, 4) for c, v in t.items()}
                                               for k, t in times.items()},
                                 "candidates": list(CANDIDATES)}
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def apply(workload, path=TABLE):
    """Load the tuned grids of `workload` into the library; returns them, or None if untuned."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get("tables", {}).get(workload)
    if not t:
        return None
    vx.set_launch_grids(t["grids"])
    return t["grids"]


def _workload_runner(name):
    import torch
    import synth
    if name == "weave_patches":
        wls = synth.weave_patches()
        plan = vx.BatchPlan([vx.Patch(w.grid, torch.as_tensor(w.pts).cuda(), torch.as_tensor(w.offsets), w.radius)
                             for w in wls], K=4, iters=2)
        return plan.run
    if name == "plain_weave":
        wl = synth.plain_weave()
        pts = torch.as_tensor(wl.pts).cuda()
        plan = vx.VoxelizePlan(1, wl.grid, pts, offsets=torch.as_tensor(wl.offsets).cuda(), radius=wl.radius)
        plan.run()
        leaf = plan.check()
        lod = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], wl.levels)
        return lambda: (plan.run(), lod.run())
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="weave_patches", choices=["weave_patches", "plain_weave"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    run = _workload_runner(args.workload)
    grids, times = tune(run, reps=args.reps)
    save(args.workload, grids, times, args.out)
    print(json.dumps({"workload": args.workload, "grids": grids,
                      "kernel_ms": {k: {str(c): round(v, 4) for c, v in t.items()} for k, t in times.items()}}),
          flush=True)


if __name__ == "__main__":
    main()
