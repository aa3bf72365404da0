"""Benchmark: voxelize + LoD pyramid with lobe clustering of the brushed-metal height field on one
MI355X, with the plain-weave fabric, the batched patches, the differentiable fit and the compact
SGGX code as further sections.

Headline workload (synth.brushed_metal, seed 2): a 4096 x 4096 vertex height field (33,538,050
float32 triangles, two per cell) with anisotropic ridges (wavelength about 8 cells along x and
256 along y, amplitude 2 voxels), sparse 4096^3 grid, surface lobe S = n n^T weighted by clipped
area, 13-level pyramid with K = 4 merged lobes per coarse voxel.  A step is one full pass of the
hot path on that input, already resident in HBM: snap + candidate boxes, primitive-tile records and
their radix sort, exact closed-box tests, clipped areas, per-voxel SGGX sums in primitive order,
then the 12 parent levels with Ward + Lloyd lobe clustering.

Prints one JSON line.  ``value`` is primitive-voxel pairs per second of whole steps (wall clock
between two device synchronisations around K steps).  The roofline uses the algorithmic byte
model of the path (bytes the method must move with pair lists in HBM):
    B = B_in + 12 N_prims + 4 rec N_pairs + sum_L out_L N_L (written once, read once by the next level)
with rec = 12 (32-bit keys) or 16 bytes (64-bit keys) per pair, out_0 = key + 4 + 4 + 24 bytes per
leaf voxel, out_L = key + 4 + 28 (K = 1) or key + 4 + 28 (1 + K) bytes above it.  The unit kernel
does the work of the pair terms (emit, sort, reduce) on chip, so its share is
12 N_prims + 4 rec N_pairs + out_0 N_0.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "primitive-voxel pairs/s & LoD build ms; fwd+bwd SGGX fit ms vs plain path"
HBM_PEAK_GBS = 8000.0


# ------------------------------------------------------------------------------------------------
# byte model
# ------------------------------------------------------------------------------------------------

def rec_bytes(key_bytes):
    return 12 if key_bytes == 4 else 16


def step_bytes(c, K):
    """Algorithmic bytes of one step (voxelize + pyramid) from the run's counts."""
    kb = c["key_bytes"]
    out0 = kb + 4 + 4 + 24
    outL = kb + 4 + 28 * (1 + K) if K > 1 else kb + 4 + 28
    return (c["input_bytes"] + 12 * c["n_prims"] + 4 * rec_bytes(kb) * c["n_pairs"] + 2 * out0 * c["levels"][0]
            + 2 * outL * sum(c["levels"][1:]))


def kernel_bytes(name, c):
    """Algorithmic bytes one launch of `name` must move (counted once)."""
    kb, P, N, V = c["key_bytes"], c["n_pairs"], c["n_prims"], c["levels"][0]
    if name in ("unit_tri", "unit_fib"):
        return 12 * N + 4 * rec_bytes(kb) * P + (kb + 32) * V
    if name == "unit_compact":
        return 2 * (kb + 32) * V
    return None


def source_digest():
    """Digest of the HIP sources: counter figures taken from another build are not reused."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2604_13191_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of `workload`
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when absent or
    taken from other sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    if not k or t.get("source_digest") != source_digest():
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


# ------------------------------------------------------------------------------------------------
# one single-instance workload: plans, kernel table, timed steps, roofline
# ------------------------------------------------------------------------------------------------

def make_plans(vx, kind, grid, data, levels, K, offsets=None, radius=0.0, tuning=None):
    plan = vx.VoxelizePlan(kind, grid, data, offsets=offsets, radius=radius, tuning=tuning)
    plan.run()
    leaf = plan.check()
    cal = vx.LodPlan(grid, leaf, plan.stats[2:3], levels, tuning=tuning).run()
    caps = [max(v.n, 1) for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(grid, leaf, plan.stats[2:3], levels, K=K, iters=2, caps=caps, tuning=tuning)
    lod.run()
    lod.check()
    return plan, lod, leaf


def kernel_table(vx, plan, lod, counts, steps=5):
    """Per-kernel time per step from events around every launch (untimed steps)."""
    vx.timing_reset()
    vx.timing_filter(None)
    vx.timing_enable(True)
    for _ in range(steps):
        plan.run()
        lod.run()
    vx.timing_enable(False)
    kt = vx.timing_collect()
    kernels = {}
    for name, (ms, n) in sorted(kt.items(), key=lambda x: -x[1][0]):
        avg = ms / max(n, 1)
        b = kernel_bytes(name, counts)
        kernels[name] = {"ms_per_step": round(ms / steps, 4), "launches_per_step": n // steps, "avg_ms": round(avg, 4),
                         "GBps_algorithmic": round(b / (avg * 1e-3) / 1e9, 1) if b is not None and avg > 0 else None}
    return kernels


def timed_steps(vx, plan, lod, steps, warmup, dom):
    """K whole steps between two synchronisations; events only around the dominant kernel."""
    import torch
    for _ in range(warmup):
        plan.run()
        lod.run()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
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
    dom_ms, dom_n = kd.get(dom, (0.0, 0))
    return {"ms_per_step": (t1 - t0) * 1e3 / steps,
            "voxelize_ms": sum(a.elapsed_time(b) for a, b, _ in ev) / steps,
            "lod_build_ms": sum(b.elapsed_time(c) for _, b, c in ev) / steps,
            "dom_avg_ms": dom_ms / max(dom_n, 1), "dom_launches": dom_n}


def graph_steps(vx, plan, lod, steps, warmup):
    import torch
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = vx.capture(lambda st: (plan.run(st), lod.run(st)), side)
    for _ in range(warmup):
        graph.replay()
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    side.synchronize()
    for a, b in gev:
        a.record(side)
        graph.replay()
        b.record(side)
    side.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in gev) / steps
    del graph
    plan.check()
    return ms


def roofline(name, workload, counts, t, K):
    """HBM roofline of the dominant kernel (algorithmic bytes / its average launch) and of the step."""
    b = kernel_bytes(name, counts)
    B = step_bytes(counts, K)
    step_gbs = B / (t["ms_per_step"] * 1e-3) / 1e9
    out = {"bound": "hbm", "kernel": name, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
           "traffic": traffic_bytes(workload, name), "algorithmic_bytes_per_launch": b,
           "avg_launch_ms": round(t["dom_avg_ms"], 5), "launches_timed": t["dom_launches"],
           "step_algorithmic_bytes": B, "step_GBps": round(step_gbs, 1), "step_frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    if b is not None and t["dom_avg_ms"] > 0:
        ach = b / (t["dom_avg_ms"] * 1e-3) / 1e9
        out["achieved"] = round(ach, 1)
        out["frac"] = round(ach / HBM_PEAK_GBS, 4)
    return out


def single_section(vx, kind, grid, data, levels, K, args, workload, offsets=None, radius=0.0, input_bytes=0,
                   graph=True, tuning=None):
    plan, lod, leaf = make_plans(vx, kind, grid, data, levels, K, offsets, radius, tuning)
    counts = {"key_bytes": 4 if grid.log2_res <= 10 else 8, "n_pairs": plan.n_pairs, "n_cand": plan.n_cand,
              "n_prims": plan.n_prims, "levels": [leaf.n] + [v.n for v in lod.out], "n_records": plan.n_records,
              "n_units": plan.n_units, "input_bytes": input_bytes}
    kernels = kernel_table(vx, plan, lod, counts)
    dom = next(iter(kernels))
    t = timed_steps(vx, plan, lod, args.steps, args.warmup, dom)
    out = {"n_pairs": plan.n_pairs, "n_candidates": plan.n_cand, "n_leaf_voxels": leaf.n,
           "level_voxels": counts["levels"], "n_tile_records": plan.n_records, "n_units": plan.n_units,
           "ms_per_step": t["ms_per_step"], "pairs_per_s": plan.n_pairs / (t["ms_per_step"] * 1e-3),
           "voxelize_ms": t["voxelize_ms"], "lod_build_ms": t["lod_build_ms"],
           "roofline": roofline(dom, workload, counts, t, K), "kernels": kernels}
    if graph:
        g = graph_steps(vx, plan, lod, args.steps, args.warmup)
        out["graph_ms_per_step"] = g
        out["graph_pairs_per_s"] = plan.n_pairs / (g * 1e-3)
    return out, plan, lod, leaf


# ------------------------------------------------------------------------------------------------
# extension sections
# ------------------------------------------------------------------------------------------------

def fit_timing(vx, wl, pts, offs, args, plain_ms):
    """Differentiable two-lobe fit (levels 1..6, 128 directions) on the plain weave: one forward
    (voxelize + 7-level pyramid + fit loss) plus one backward (lobe and control-point gradients)."""
    import torch
    plan = vx.FitPlan(wl.grid, pts, offs, wl.radius, 1, 6)
    params = vx.fit_init(plan, seed=4)
    one = torch.ones(1, device=pts.device)
    for _ in range(max(1, args.warmup)):
        plan.forward(pts, params, check=False)
        plan.backward(one, params)
    torch.cuda.synchronize()
    plan.check()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for a, b, c in ev:
        a.record()
        plan.forward(pts, params, check=False)
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
                     "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None}
    return out


def _single_build(vx, wl, K, tuning):
    """Single-instance plain path for one fiber set: voxelize + full pyramid with K lobes."""
    import torch
    pts = torch.as_tensor(wl.pts).cuda()
    offs = torch.as_tensor(wl.offsets).cuda()
    plan, lod, _ = make_plans(vx, 1, wl.grid, pts, wl.grid.log2_res + 1, K, offs, wl.radius, tuning)
    return plan, lod


def batch_timing(vx, args):
    """Uneven batch: 64 weave patches (fiber counts log-uniform in [100, 20000], grids 256^3 ..
    2048^3, full pyramids, K = 4): one replay of the captured batched build against the 64
    single-instance builds of the same patches, each captured as a graph and replayed."""
    import torch
    import synth
    from paper_2604_13191_amd import autotune
    wls = synth.weave_patches()
    tuning = autotune.load("weave_patches")
    stream = torch.cuda.Stream()
    plan = vx.BatchPlan([vx.Patch(w.grid, torch.as_tensor(w.pts).cuda(), torch.as_tensor(w.offsets), w.radius)
                         for w in wls], K=4, iters=2, tuning=tuning)
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
    n_prims = plan.n_pts
    del g, plan
    torch.cuda.empty_cache()
    single_ms, single_pairs = 0.0, 0
    for wl in wls:
        sp, sl = _single_build(vx, wl, 4, tuning)
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        sg = vx.capture(lambda st: (sp.run(st), sl.run(st)), side)
        sg.replay()
        side.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, b in ev:
            a.record(side)
            sg.replay()
            b.record(side)
        side.synchronize()
        sp.check()
        sl.check()
        single_ms += sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        single_pairs += sp.n_pairs
        del sg, sp, sl
    torch.cuda.empty_cache()
    assert single_pairs == n_pairs, (single_pairs, n_pairs)
    counts = {"key_bytes": 8, "n_pairs": n_pairs, "n_prims": n_prims, "levels": levels_n,
              "input_bytes": 12 * n_prims + 8 * (sum(len(w.offsets) - 1 for w in wls) + 1)}
    B = step_bytes(counts, 4)
    return {"workload": "64 weave patches, 100-20,000 fibers x 256 segments, 256^3-2048^3, full pyramids, K=4",
            "fibers": int(sum(len(w.offsets) - 1 for w in wls)), "pairs": n_pairs, "voxels_per_level": levels_n,
            "graph_replay_ms": batch_ms, "pairs_per_s": n_pairs / (batch_ms * 1e-3),
            "single_instance_graphs_sum_ms": single_ms, "speedup_vs_single": single_ms / batch_ms,
            "algorithmic_bytes": B, "hbm_frac": round(B / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "tuning": tuning.as_dict() if tuning is not None else "default"}


def occupancy_timing(vx, args):
    """Sub-voxel occupancy (Sec. 3.5, Sec. 4.2) of the full pyramids of the brushed-metal surface
    (13 levels) and of the plain weave (11 levels): the pass regenerates the pairs, builds every
    pair's 512-bit sub-cell mask and the masks and counts of all levels."""
    import torch
    import synth
    out = {}
    for name in ("brushed_metal", "plain_weave"):
        wl = synth.brushed_metal() if name == "brushed_metal" else synth.plain_weave()
        kind = 0 if name == "brushed_metal" else 1
        data = torch.as_tensor(wl.tris if kind == 0 else wl.pts).cuda()
        offs = None if kind == 0 else torch.as_tensor(wl.offsets).cuda()
        radius = 0.0 if kind == 0 else wl.radius
        plan = vx.VoxelizePlan(kind, wl.grid, data, offsets=offs, radius=radius).run()
        leaf = plan.check()
        cal = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], wl.levels).run()
        caps = [max(v.n, 1) for v in cal.check()[1:]]
        del cal
        lod = vx.LodPlan(wl.grid, leaf, plan.stats[2:3], wl.levels, caps=caps).run()
        lod.check()
        occ = vx.OccupancyPlan(kind, wl.grid, data, lod, offsets=offs, radius=radius)
        for _ in range(max(1, args.warmup)):
            occ.run()
        torch.cuda.synchronize()
        vx.timing_reset()
        vx.timing_filter(None)
        vx.timing_enable(True)
        occ.run()
        vx.timing_enable(False)
        kt = vx.timing_collect()
        steps = max(1, min(args.steps, 5))
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record()
            occ.run()
            b.record()
        torch.cuda.synchronize()
        levels = occ.check()
        ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        lv0 = levels[0].numpy()
        out[name] = {"pass_ms": ms, "pairs": occ.n_pairs, "leaf_voxels": leaf.n,
                     "pairs_per_s": occ.n_pairs / (ms * 1e-3),
                     "leaf_mean_occupancy": float(lv0["hits"].mean() / 512.0),
                     "leaf_mean_density_xy_xz_yz": [float(lv0[f].mean() / 64.0) for f in ("xy", "xz", "yz")],
                     "kernels_ms": {k: round(v[0], 4) for k, v in sorted(kt.items(), key=lambda x: -x[1][0])}}
        del occ, lod, plan, leaf, data, offs
        torch.cuda.empty_cache()
    return out


def sggxh_timing(vx, args, d_lod_ms):
    """The paper's SGGX-H reduction (Sec. 4.4: 5000 samples per lobe, 5^3 histograms, Wasserstein
    merges) over the 13-level pyramid of the brushed-metal surface with K = 4, against the moment
    metric's Ward + Lloyd clustering of the same pyramid: time, and at level 1 (both reduce the
    same leaf lobes) the share of voxels merged alike and the projected-area error of the K lobes
    against the unmerged children (64 directions)."""
    import torch
    import synth
    from paper_2604_13191_amd import autotune
    wl = synth.brushed_metal()
    tris = torch.as_tensor(wl.tris).cuda()
    grid, levels = wl.grid, wl.levels
    del wl
    tuned = autotune.load("brushed_metal")
    plan = vx.VoxelizePlan(0, grid, tris, tuning=tuned).run()
    leaf = plan.check()
    cal = vx.LodPlan(grid, leaf, plan.stats[2:3], levels, tuning=tuned).run()
    caps = [max(v.n, 1) for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(grid, leaf, plan.stats[2:3], levels, K=4, iters=2, caps=caps, tuning=tuned).run()
    lod.check()
    sh = vx.SggxhPlan(lod, K=4, samples=5000)
    sh.run()
    sh.check()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    vx.timing_reset()
    vx.timing_filter(None)
    vx.timing_enable(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        sh.run()
        b.record()
    torch.cuda.synchronize()
    vx.timing_enable(False)
    kt = vx.timing_collect()
    hl = sh.check()
    ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    # level 1: both methods reduce the same leaf lobes
    n0, n1 = leaf.n, lod.out[0].n
    lk = leaf.keys[:n0].long()
    pk = lod.out[0].keys[:n1].long()
    parent = torch.searchsorted(pk, lk >> 3)
    inputs = torch.zeros(n1, dtype=torch.int64, device=lk.device).index_add_(
        0, parent, (leaf.w[:n0] > 0).long())
    from synth import fibonacci_dirs
    dirs = torch.as_tensor(fibonacci_dirs(64), dtype=torch.float64, device=lk.device)
    S0 = leaf.S[:, :n0].double()
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    q0 = (S0[0][:, None] * x * x + S0[1][:, None] * y * y + S0[2][:, None] * z * z
          + 2 * (S0[3][:, None] * x * y + S0[4][:, None] * x * z + S0[5][:, None] * y * z))
    # a lobe's projected area along v: w sqrt(v^T (S / w) v) = sqrt(w v^T S v)
    w0 = leaf.w[:n0].double()[:, None]
    ref = torch.zeros(n1, 64, dtype=torch.float64, device=lk.device).index_add_(
        0, parent, torch.sqrt((w0 * q0).clamp_min(0)))
    reduced = inputs > 4
    out = {"workload": "brushed_metal 13-level pyramid, K=4, 5000 samples per lobe", "build_ms": ms,
           "moment_metric_lod_ms": d_lod_ms,
           "kernels_ms": {k: round(v[0] / steps, 3) for k, v in kt.items()},
           "level1_voxels": n1, "level1_reduced": int(reduced.sum())}
    errs = {}
    for name, lb in (("sggx_h", hl[0]), ("moment_ward_lloyd", lod.lobes[0])):
        Sk = lb.S[:, :, :n1].double()                           # [6, K, n]
        x2 = (Sk[0][..., None] * x * x + Sk[1][..., None] * y * y + Sk[2][..., None] * z * z
              + 2 * (Sk[3][..., None] * x * y + Sk[4][..., None] * x * z + Sk[5][..., None] * y * z))
        wk = lb.w[:, :n1].double()[..., None]                   # [K, n, 1]
        prof = torch.sqrt((wk * x2).clamp_min(0)).sum(0)        # [n, 64]
        e = (prof - ref).abs().max(1).values / ref.max(1).values.clamp_min(1e-30)
        errs[name] = e[reduced]
        out[name + "_level1_profile_error"] = {"mean": float(errs[name].mean()), "p99": float(errs[name].quantile(0.99)),
                                               "max": float(errs[name].max())}
    wa = torch.sort(hl[0].w[:, :n1].double(), dim=0).values
    wb = torch.sort(lod.lobes[0].w[:, :n1].double(), dim=0).values
    same = ((wa - wb).abs() <= 1e-5 * wa.sum(0).clamp_min(1e-30)).all(0)
    out["level1_same_partition_share"] = float(same[reduced].double().mean())
    del sh, lod, plan, leaf, tris
    torch.cuda.empty_cache()
    return out


def _leaf_error(exact, ex_n, samp, s_n):
    """Relative L1 distance of the sampled leaf from the exact one (weights and moments, summed
    over the union of their voxels) and the share of the exact voxels of positive area that the
    sampler reached."""
    import torch
    ek, sk = exact.keys[:ex_n].long(), samp.keys[:s_n].long()
    ew, sw = exact.w[:ex_n].double(), samp.w[:s_n].double()
    eS, sS = exact.S[:, :ex_n].double(), samp.S[:, :s_n].double()
    idx = torch.searchsorted(ek, sk).clamp_max(max(ex_n - 1, 0))
    hit = ek[idx] == sk
    m = torch.zeros(ex_n, dtype=torch.bool, device=ek.device)
    m[idx[hit]] = True
    dw = (sw[hit] - ew[idx[hit]]).abs().sum() + sw[~hit].sum() + ew[~m].sum()
    dS = ((sS[:, hit] - eS[:, idx[hit]]).abs().sum() + sS[:, ~hit].abs().sum() + eS[:, ~m].abs().sum())
    pos = ew > 0
    return {"w_rel_l1": float(dw / ew.sum()), "S_rel_l1": float(dS / eS.abs().sum()),
            "exact_area_voxels_reached": float((m & pos).sum() / pos.sum()), "voxels": int(s_n)}


def sampling_timing(vx, args, exact_ms):
    """The paper's sampling voxelizer (Sec. 3.2-3.3) on the headline surface, feeding the same
    13-level pyramid with K = 4 lobes: whole steps (sample + pyramid) for N = 4, 16 and 64 samples
    on the largest triangle, against the exact step, with the sampled leaf's distance from the
    exact one."""
    import torch
    import synth
    from paper_2604_13191_amd import autotune
    wl = synth.brushed_metal()
    tris = torch.as_tensor(wl.tris).cuda()
    grid, levels = wl.grid, wl.levels
    del wl
    tuned = autotune.load("brushed_metal")
    ex = vx.VoxelizePlan(0, grid, tris, tuning=tuned).run()
    exact = ex.check()
    out = {"workload": "brushed_metal, sampled voxelizer + 13-level pyramid, K=4", "exact_step_ms": exact_ms,
           "runs": {}}
    steps = max(1, min(args.steps, 5))
    for N in (4, 16, 64):
        sp = vx.SamplePlan(0, grid, tris, N=N)
        sp.run()
        leaf = sp.check()
        cal = vx.LodPlan(grid, leaf, sp.stats[2:3], levels, tuning=tuned).run()
        caps = [max(v.n, 1) for v in cal.check()[1:]]
        del cal
        lod = vx.LodPlan(grid, leaf, sp.stats[2:3], levels, K=4, iters=2, caps=caps, tuning=tuned)
        for _ in range(max(1, args.warmup)):
            sp.run()
            lod.run()
        torch.cuda.synchronize()
        vx.timing_reset()
        vx.timing_filter(None)
        vx.timing_enable(True)
        sp.run()
        lod.run()
        vx.timing_enable(False)
        kt = vx.timing_collect()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for a, b, c in ev:
            a.record()
            sp.run()
            b.record()
            lod.run()
            c.record()
        torch.cuda.synchronize()
        sp.check()
        lod.check()
        smp = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
        lb = sum(b.elapsed_time(c) for _, b, c in ev) / steps
        r = {"samples": sp.n_samples, "sample_ms": smp, "lod_build_ms": lb, "step_ms": smp + lb,
             "samples_per_s": sp.n_samples / (smp * 1e-3), "step_over_exact": (smp + lb) / exact_ms,
             "kernels_ms": {k: round(v[0], 4) for k, v in sorted(kt.items(), key=lambda x: -x[1][0])
                            if k.startswith("sample") or k.startswith("radix")}}
        r.update(_leaf_error(exact, exact.n, leaf, leaf.n))
        out["runs"][str(N)] = r
        del sp, lod, leaf
        torch.cuda.empty_cache()
    del ex, exact, tris
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the headline workload
# ------------------------------------------------------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(window=1025, repeats=3):
    """The oracle (FP64, std::thread over primitive chunks) on the first `window` x `window`
    vertices of the brushed-metal field (1/16 of it at 1025): voxelize + 13-level pyramid + K = 4
    lobe clustering, single-threaded and on every host core the process may use, median of
    `repeats` runs each."""
    import oracle
    import synth
    wl = synth.brushed_metal(window=window)
    nall = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    res = {}
    for nth in (1, nall):
        ts, pairs = [], 0
        for _ in range(repeats):
            t0 = time.perf_counter()
            ref = oracle.voxelize_triangles(wl.grid, wl.tris, nthreads=nth)
            lod = oracle.build_lod(ref, wl.levels)
            oracle.cluster_pyramid(lod, 4, 2, nthreads=nth)
            ts.append(time.perf_counter() - t0)
            pairs = ref.n_pairs
        res[nth] = (statistics.median(ts), pairs)
    t_all, pairs = res[nall]
    t_one, _ = res[1]
    return {"value": pairs / t_all, "unit": "pairs/s", "cores": nall, "kind": "oracle",
            "sample": f"brushed metal, first {window}x{window} vertices ({wl.tris.shape[0]} triangles, {pairs} pairs): "
                      f"voxelize + {wl.levels}-level pyramid + K=4 clustering in FP64, median of {repeats} runs: "
                      f"{t_all:.2f} s on {nall} threads, {t_one:.2f} s on 1 thread",
            "single_thread_value": pairs / t_one, "cpu_model": cpu_model(), "nproc": os.cpu_count()}


# ------------------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-weave", action="store_true")
    ap.add_argument("--no-compact", action="store_true")
    ap.add_argument("--no-sampling", action="store_true")
    ap.add_argument("--no-occupancy", action="store_true")
    ap.add_argument("--no-sggxh", action="store_true")
    ap.add_argument("--probe", action="store_true", help="end with a plain copy of known size (counter scaling)")
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

    # ---- headline: brushed metal ---------------------------------------------------------------
    tuned = autotune.load("brushed_metal")
    wl = synth.brushed_metal()
    tris = torch.as_tensor(wl.tris).cuda()
    grid, levels, n_tris = wl.grid, wl.levels, wl.tris.shape[0]
    del wl
    head, plan, lod, leaf = single_section(vx, 0, grid, tris, levels, 4, args, "brushed_metal",
                                           input_bytes=36 * n_tris, tuning=tuned)
    del plan, lod, leaf, tris
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": head["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": "brushed_metal: 4096x4096 vertex height field (33,538,050 triangles), 4096^3, "
                               "13 levels, K=4", "n_pairs": head["n_pairs"], "n_leaf_voxels": head["n_leaf_voxels"],
                   "level_voxels": head["level_voxels"], "tuning": tuned.as_dict() if tuned is not None else "default"},
        "voxelize_ms": head["voxelize_ms"], "lod_build_ms": head["lod_build_ms"],
        "graph_ms_per_step": head.get("graph_ms_per_step"), "graph_pairs_per_s": head.get("graph_pairs_per_s"),
        "roofline": head["roofline"], "kernels": head["kernels"],
    }

    if not args.no_sampling:
        out["sampling"] = sampling_timing(vx, args, head["ms_per_step"])
        torch.cuda.empty_cache()
    if not args.no_occupancy:
        out["occupancy"] = occupancy_timing(vx, args)
        torch.cuda.empty_cache()
    if not args.no_sggxh:
        out["sggx_h"] = sggxh_timing(vx, args, head["lod_build_ms"])
        torch.cuda.empty_cache()

    # ---- plain weave, fit, compact -------------------------------------------------------------
    if not args.no_weave or not args.no_fit or not args.no_compact:
        tw = autotune.load("plain_weave")
        ww = synth.plain_weave()
        pts = torch.as_tensor(ww.pts).cuda()
        offs = torch.as_tensor(ww.offsets).cuda()
        sec, plan, lod, leaf = single_section(vx, 1, ww.grid, pts, ww.levels, 1, args, "plain_weave", offs,
                                              ww.radius, input_bytes=12 * ww.pts.shape[0] + 8 * len(ww.offsets),
                                              tuning=tw)
        sec["workload"] = "plain_weave: 2000 fibers x 256 segments, radius 0.5 voxel, 1024^3, 11 levels, K=1"
        sec["tuning"] = tw.as_dict() if tw is not None else "default"
        if not args.no_weave:
            out["plain_weave"] = sec
        if not args.no_fit:
            out["fit"] = fit_timing(vx, ww, pts, offs, args, sec["ms_per_step"])
        if not args.no_compact:
            out["sggx_compact"] = compact_timing(vx, leaf, args)
        del plan, lod, leaf, pts, offs
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batch_timing(vx, args)
        torch.cuda.empty_cache()
    if args.probe:
        # a plain copy of known size, for scaling the HBM byte counters of a profiler run
        probe = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")
        probe2 = torch.empty_like(probe)
        torch.neg(probe.view(torch.float32), out=probe2.view(torch.float32))
        torch.cuda.synchronize()
        del probe, probe2
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
