"""Benchmark: voxelize + LoD pyramid of the plain-weave fabric on one MI355X.

Workload: 2,000 fibers x 256 segments (float32 polylines), sinusoidal warp/weft crimp
(period 64 voxels, amplitude 4), helix twist U(-5, 5) deg, N(0, 0.3^2) jitter, radius 0.5
voxel, sparse 1024^3 grid, fiber lobe S = I - t t^T, 11-level LoD with one lobe per voxel
(synth.plain_weave, seed 1).  A step is one full pass of the hot path on that input, already
resident in HBM: snap + candidates, exact capsule tests with ballot compaction, clipped
lengths, radix sort by Morton key, segmented SGGX reduce, and the 10 parent levels.

Prints one JSON line.  ``value`` is primitive-voxel pairs per second of whole steps.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "primitive-voxel pairs/s & LoD build ms; fwd+bwd SGGX fit ms vs plain path"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64


def kernel_flops(name, c):
    """Lower-bound FP64 operation count of the exact-test kernels: the centre-ball filter that
    every candidate takes (45 operations: box-relative coordinates and scale bound, the
    projection of the box centre on the segment, the clamped distance and the two comparisons) and the clipped length of every touching pair (32: two divisions and the
    clamps per axis, the product by the length).  The exact bracketing of the candidates the
    filter leaves undecided is not counted."""
    if name in ("unit_fib",):
        return 45 * c["n_cand"] + 32 * c["n_pairs"]
    return None


def kernel_bytes(name, c):
    """Algorithmic bytes one launch of `name` must move (counted once), from the run's counts:
    P pairs, C candidates, N primitives, V leaf voxels, F fibers, T records, U units."""
    kb, P, N, V, F = c["key_bytes"], c["n_pairs"], c["n_prims"], c["n_vox"], c["n_fib"]
    T, U = c["n_records"], c["n_units"]
    rec = 64   # per-primitive record
    table = {
        "prep_fib": 12 * N + 8 * (F + 1) + rec * N + 16 * N + 8 * N,
        "check_offsets": 8 * (F + 1),
        # per record of a unit: primitive id, record and the primitive's direction; per voxel the
        # staged key (leaf key width), count, w and S; per unit its descriptor
        "unit_fib": (4 + rec + 16) * T + (kb + 32) * V + 32 * U,
        "unit_compact": 2 * (kb + 32) * V + 24 * U,
        "radix_scatter": 2 * (kb + 8) * T,
        "radix_hist": kb * T,
    }
    return table.get(name)


def source_digest():
    """Digest of the HIP sources: counter figures taken from another build are not reused."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2604_13191_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy of known size), or None when absent or taken from
    other sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_plain_weave.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    if not k or t.get("source_digest") != source_digest():
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def cpu_baseline(wl, nthreads):
    import oracle
    t0 = time.perf_counter()
    ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius, nthreads=nthreads)
    oracle.build_lod(ref, wl.levels)
    dt = time.perf_counter() - t0
    return {"value": ref.n_pairs / dt, "unit": "pairs/s", "cores": nthreads, "kind": "oracle",
            "sample": f"the full workload once (voxelize + {wl.levels}-level pyramid, FP64, "
                      f"{ref.n_pairs} pairs) in {dt:.2f} s on {nthreads} host threads"}


def fit_timing(vx, wl, pts, offs, args, plain_ms):
    """Differentiable two-lobe fit (levels 1..6, 128 directions) on the same fabric: one forward
    (voxelize + 7-level pyramid + fit loss) plus one backward (lobe and control-point gradients)."""
    import torch
    plan = vx.FitPlan(wl.grid, pts, offs, wl.radius, 1, 6)
    params = vx.fit_init(plan, seed=4)
    one = torch.ones(1, device=pts.device)
    for _ in range(max(1, args.warmup)):
        plan.forward(pts, params)
        plan.backward(one, params)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for a, b, c in ev:
        a.record()
        plan.forward(pts, params)
        b.record()
        plan.backward(one, params)
        c.record()
    torch.cuda.synchronize()
    plan.check()
    fwd = sum(a.elapsed_time(b) for a, b, _ in ev) / args.steps
    bwd = sum(b.elapsed_time(c) for _, b, c in ev) / args.steps
    return {"levels": "1-6", "lobes": 2, "directions": 128, "fwd_ms": fwd, "bwd_ms": bwd, "fwd_bwd_ms": fwd + bwd,
            "plain_path_ms": plain_ms, "fwd_bwd_over_plain": (fwd + bwd) / plain_ms,
            "fitted_voxels": int(sum(plan.counts[1:7]))}


def compact_timing(vx, leaf, args):
    """Leaf eigen-fit + 6-byte SGGX code over every leaf voxel of the fabric, and the decoding of
    those codes; kernel times from events around each launch on the launch stream."""
    import torch
    n = leaf.n
    code = None
    for _ in range(max(1, args.warmup)):
        lam, vec, code = vx.sggx_compact(leaf.w, leaf.S, n=n, eps=1e-3)
        vx.sggx_decode(code, n=n)
    torch.cuda.synchronize()
    vx.timing_reset()
    vx.timing_filter(None)
    vx.timing_enable(True)
    for _ in range(args.steps):
        vx.sggx_compact(leaf.w, leaf.S, n=n, eps=1e-3)
        vx.sggx_decode(code, n=n)
    vx.timing_enable(False)
    kt = vx.timing_collect()
    out = {"workload": "leaf voxels of the plain weave", "voxels": n}
    # storage error of the byte code (untimed): decoded SGGX against S / w scaled to a largest
    # diagonal entry of 1, per voxel the largest entry difference (it includes the eigenvalue floor)
    dec = vx.sggx_decode(code, n=n)[:, :n].double()
    pos = leaf.w[:n] > 0
    M = leaf.S[:, :n].double()[:, pos] / leaf.w[:n].double()[pos]
    M = M / M[:3].max(dim=0).values.clamp_min(1e-30)
    err = (dec[:, pos] - M).abs().max(dim=0).values
    out["code_error_max"] = float(err.max())
    out["code_error_mean"] = float(err.mean())
    # algorithmic bytes per voxel: w + S in (28), code (6) + eigenvalues (12) + eigenvectors (36) out;
    # decoding reads the code (6) and writes S (24)
    for name, per in (("sggx_compact", 82), ("sggx_decode", 30)):
        ms, cnt = kt.get(name, (0.0, 0))
        avg = ms / max(cnt, 1)
        gbs = per * n / (avg * 1e-3) / 1e9 if avg > 0 else None
        out[name] = {"avg_ms": avg, "launches": cnt, "bytes_per_voxel": per, "GBps": gbs,
                     "hbm_frac": gbs / 8000.0 if gbs else None}
    return out


def _single_build(vx, wl, K):
    """Single-instance plain path for one fiber set: voxelize + full pyramid with K lobes."""
    import torch
    pts = torch.as_tensor(wl.pts).cuda()
    offs = torch.as_tensor(wl.offsets).cuda()
    plan = vx.VoxelizePlan(1, wl.grid, pts, offsets=offs, radius=wl.radius)
    plan.run()
    leaf = plan.check()
    levels = wl.grid.log2_res + 1
    cal = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], levels).run()
    caps = [max(v.n, 1) for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], levels, K=K, iters=2, caps=caps)
    return plan, lod


def batch_timing(vx, args):
    """Uneven batch: 64 weave patches (fiber counts log-uniform in [100, 20000], grids 256^3 ..
    2048^3, full pyramids, K = 4): one replay of the captured batched build against the 64
    single-instance builds of the same patches, each timed on its own."""
    import torch
    import synth
    from paper_2604_13191_amd import autotune
    wls = synth.weave_patches()
    default = vx.get_launch_grids()
    grids = autotune.apply("weave_patches")
    stream = torch.cuda.Stream()
    plan = vx.BatchPlan([vx.Patch(w.grid, torch.as_tensor(w.pts).cuda(), torch.as_tensor(w.offsets), w.radius)
                         for w in wls], K=4, iters=2)
    plan.run(stream)
    plan.check(stream)
    torch.cuda.synchronize()
    g = plan.capture(stream)
    for _ in range(max(1, args.warmup)):
        g.replay()
    stream.synchronize()
    steps = max(1, min(args.steps, 10))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        g.replay()
        b.record(stream)
    stream.synchronize()
    plan.check(stream)
    batch_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    n_pairs, levels_n = plan.n_pairs, [v.n for v in plan.out]
    del g, plan
    torch.cuda.empty_cache()
    single_ms, single_pairs = 0.0, 0
    for wl in wls:
        sp, sl = _single_build(vx, wl, 4)
        sp.run()
        sl.run()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, b in ev:
            a.record()
            sp.run()
            sl.run()
            b.record()
        torch.cuda.synchronize()
        sp.check()
        sl.check()
        single_ms += sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        single_pairs += sp.n_pairs
        del sp, sl
    torch.cuda.empty_cache()
    vx.set_launch_grids(default)
    assert single_pairs == n_pairs, (single_pairs, n_pairs)
    return {"workload": "64 weave patches, 100-20,000 fibers x 256 segments, 256^3-2048^3, full pyramids, K=4",
            "fibers": int(sum(len(w.offsets) - 1 for w in wls)), "pairs": n_pairs, "voxels_per_level": levels_n,
            "graph_replay_ms": batch_ms, "pairs_per_s": n_pairs / (batch_ms * 1e-3),
            "single_instance_sum_ms": single_ms, "speedup_vs_single": single_ms / batch_ms,
            "launch_grids": grids if grids is not None else "default (1024)"}


def brushed_timing(vx, args):
    """Brushed-metal height field at full size (33,538,050 triangles, 4096^3, 13 levels, K = 4):
    voxelize (exact triangle-box test, clipped areas) and the pyramid with lobe clustering."""
    import torch
    import synth
    wl = synth.brushed_metal()
    tris = torch.as_tensor(wl.tris).cuda()
    grid, levels = wl.grid, wl.levels
    del wl
    plan = vx.VoxelizePlan(0, grid, tris)
    plan.run()
    leaf = plan.check()
    cal = vx.LodPlan(grid, leaf, plan.stats[2:3], levels).run()
    caps = [max(v.n, 1) for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(grid, leaf, plan.stats[2:3], levels, K=4, iters=2, caps=caps)
    for _ in range(max(1, min(args.warmup, 2))):
        plan.run()
        lod.run()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    vx.timing_reset()
    vx.timing_filter(None)
    vx.timing_enable(True)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for a, b, c in ev:
        a.record()
        plan.run()
        b.record()
        lod.run()
        c.record()
    torch.cuda.synchronize()
    vx.timing_enable(False)
    kt = vx.timing_collect()
    plan.check()
    lod.check()
    vox = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    lodm = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    top = sorted(kt.items(), key=lambda x: -x[1][0])[:6]
    out = {"workload": "brushed metal: 4096x4096 vertices (33,538,050 triangles), 4096^3, 13 levels, K=4",
           "pairs": plan.n_pairs, "leaf_voxels": leaf.n, "voxelize_ms": vox, "lod_build_ms": lodm,
           "pairs_per_s": plan.n_pairs / ((vox + lodm) * 1e-3), "voxelize_pairs_per_s": plan.n_pairs / (vox * 1e-3),
           "kernels_ms_per_step": {k: round(ms / steps, 3) for k, (ms, n) in top}}
    del plan, lod, leaf, tris
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-brushed", action="store_true")
    ap.add_argument("--no-compact", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; sharding across GPUs is a design note only, "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import torch
    import paper_2604_13191_amd as vx
    import synth

    torch.cuda.set_device(0)
    from paper_2604_13191_amd import autotune
    tuned = autotune.apply("plain_weave")          # launch grids chosen by the autotuner, if tuned
    wl = synth.plain_weave()
    pts = torch.as_tensor(wl.pts).cuda()
    offs = torch.as_tensor(wl.offsets).cuda()
    plan = vx.VoxelizePlan(1, wl.grid, pts, offsets=offs, radius=wl.radius)
    plan.run()
    leaf = plan.check()
    n_leaf_dev = plan.stats[2:3]
    cal = vx.LodPlan(wl.grid, leaf, n_leaf_dev, wl.levels).run()
    caps = [v.n for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(wl.grid, leaf, n_leaf_dev, wl.levels, caps=caps)

    for _ in range(args.warmup):
        plan.run()
        lod.run()
    torch.cuda.synchronize()
    counts = {"key_bytes": 4 if wl.grid.log2_res <= 10 else 8, "n_pairs": plan.n_pairs, "n_cand": plan.n_cand,
              "n_prims": plan.n_prims, "n_vox": leaf.n, "n_fib": plan.n_fib, "n_records": plan.n_records,
              "n_units": plan.n_units}

    # kernel breakdown: a few untimed steps with events around every launch
    prof_steps = 5
    vx.timing_reset()
    vx.timing_filter(None)
    vx.timing_enable(True)
    for _ in range(prof_steps):
        plan.run()
        lod.run()
    vx.timing_enable(False)
    kt = vx.timing_collect()
    kernels = {}
    for name, (ms, n) in sorted(kt.items(), key=lambda x: -x[1][0]):
        avg = ms / max(n, 1)
        b = kernel_bytes(name, counts)
        kernels[name] = {"ms_per_step": round(ms / prof_steps, 4), "launches_per_step": n // prof_steps,
                         "avg_ms": round(avg, 4),
                         "GBps": round(b / (avg * 1e-3) / 1e9, 1) if b is not None and avg > 0 else None}
    dom = next(iter(kernels))                       # largest share of the step

    # timed region: K whole steps; events only around the dominant kernel's launches
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    vx.timing_reset()
    vx.timing_filter(dom)
    vx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b, c in ev:
        a.record()
        plan.run()
        b.record()
        lod.run()
        c.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    vx.timing_enable(False)
    kd = vx.timing_collect()
    vx.timing_filter(None)
    plan.check()
    lod.check()
    ms_step = (t1 - t0) * 1e3 / args.steps
    vox_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / args.steps
    lod_ms = sum(b.elapsed_time(c) for _, b, c in ev) / args.steps
    dom_ms, dom_n = kd[dom]
    dom_avg = dom_ms / dom_n

    # the same step captured once as a graph and replayed
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = vx.capture(lambda st: (plan.run(st), lod.run(st)), side)
    for _ in range(args.warmup):
        graph.replay()
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    side.synchronize()
    for a, b in gev:
        a.record(side)
        graph.replay()
        b.record(side)
    side.synchronize()
    graph_ms = sum(a.elapsed_time(b) for a, b in gev) / args.steps
    del graph
    plan.check()

    # a plain copy of known size, for scaling the HBM byte counters of a profiler run
    probe = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
    probe2 = torch.empty_like(probe)
    probe2.copy_(probe)
    torch.neg(probe.view(torch.float32), out=probe2.view(torch.float32))
    torch.cuda.synchronize()
    del probe, probe2

    dom_b = kernel_bytes(dom, counts)
    dom_f = kernel_flops(dom, counts)
    if dom_f is not None:
        ach = dom_f / (dom_avg * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4), "traffic": traffic_bytes(dom),
                "algorithmic_flops_per_launch": dom_f, "algorithmic_bytes_per_launch": dom_b,
                "hbm_GBps_at_algorithmic_bytes": round(dom_b / (dom_avg * 1e-3) / 1e9, 1) if dom_b else None,
                "avg_launch_ms": round(dom_avg, 5), "launches_timed": dom_n}
    elif dom_b is not None:
        ach = dom_b / (dom_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_bytes(dom),
                "algorithmic_bytes_per_launch": dom_b, "avg_launch_ms": round(dom_avg, 5),
                "launches_timed": dom_n}
    else:
        roof = {"bound": "unmodelled", "kernel": dom, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "avg_launch_ms": round(dom_avg, 5)}
    out = {
        "metric": METRIC, "value": plan.n_pairs / (ms_step * 1e-3), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": "plain_weave: 2000 fibers x 256 segments, radius 0.5 voxel, 1024^3, 11 levels, K=1",
                   "n_pairs": plan.n_pairs, "n_candidates": plan.n_cand, "n_leaf_voxels": leaf.n,
                   "n_tile_records": plan.n_records, "n_units": plan.n_units,
                   "launch_grids": tuned if tuned is not None else vx.get_launch_grids(),
                   "level_voxels": [leaf.n] + caps},
        "voxelize_ms": vox_ms, "lod_build_ms": lod_ms, "graph_ms_per_step": graph_ms,
        "graph_pairs_per_s": plan.n_pairs / (graph_ms * 1e-3),
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_fit:
        out["fit"] = fit_timing(vx, wl, pts, offs, args, ms_step)
    if not args.no_compact:
        out["sggx_compact"] = compact_timing(vx, leaf, args)
    if not args.no_batch or not args.no_brushed:
        del plan, lod
        torch.cuda.empty_cache()
    if not args.no_brushed:
        out["brushed_metal"] = brushed_timing(vx, args)
    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batched"] = batch_timing(vx, args)
    if not args.no_cpu_baseline:
        nth = max(1, min(16, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(wl, nth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
