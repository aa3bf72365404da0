"""Batched patches (vx_batch_build) through the C ABI.

* A batch of uneven patches gives, patch by patch, exactly what the single-instance path gives
  for that patch alone: the same kernels run, every voxel sums its pairs (and parents their
  children) in the same order, so keys, counts, masks, w, S and lobes are bit-identical.
* Each patch of a small batch agrees with the FP64 oracle (keys/counts/masks exact, w and S
  to the bar of tests/parity.py, lobes as in the clustering tests).
* A captured graph replays to the eager result, replay after replay, with eager work between.
* Other tunings (tile edge, unit budget, launch grids: the autotuner's knobs) do not change a bit
  of the result.
* At the full uneven workload (64 patches, 100 .. 20,000 fibers, 256^3 .. 2048^3, K = 4) the
  batched build equals the 64 single-instance builds, and its two smallest patches match the
  oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_level, compare_lobes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _patches(vx, wls):
    import torch
    return [vx.Patch(w.grid, torch.as_tensor(w.pts).cuda(), torch.as_tensor(w.offsets), w.radius) for w in wls]


def _small_batch(seed):
    """Seven patches: weave patches on 2^5 .. 2^7 grids, a random-walk patch with points
    leaving the grid, an empty patch, a patch of one-point fibers, and a patch whose grid
    does not start at the origin."""
    wls = synth.weave_patches(n_patches=3, seed=seed, fibers=(3, 40), log2_res=(5, 7), n_points=33)
    wls.append(synth.random_fibers(12, 20, 6, seed=seed + 1, step=1.5, margin=2.0))
    e = synth.random_fibers(1, 1, 4, seed=0)
    wls.append(synth.FiberWorkload("empty", e.grid, np.zeros((0, 3), np.float32), np.zeros(1, np.int64),
                                   0.5, e.levels, 1))
    one = synth.random_fibers(5, 1, 5, seed=seed + 2)
    wls.append(one)
    sh = synth.random_fibers(6, 16, 5, seed=seed + 3, inset=2.0)
    g = synth.Grid((-7.25, 3.5, 100.0), 32.0, 5)
    wls.append(synth.FiberWorkload("shifted", g, (sh.pts + np.array([-7.25, 3.5, 100.0], np.float32)),
                                   sh.offsets, 0.75, 6, 1))
    return wls


def _single(vx, wl, K):
    """The single-instance path for one patch: voxelize + full pyramid with K lobes (level caps
    from a K = 1 counting build)."""
    import torch
    pts = torch.as_tensor(wl.pts).cuda()
    offs = torch.as_tensor(wl.offsets).cuda()
    if wl.pts.shape[0] == 0:
        return None, None
    plan = vx.VoxelizePlan(1, wl.grid, pts, offsets=offs, radius=wl.radius)
    plan.run()
    leaf = plan.check()
    levels = wl.grid.log2_res + 1
    n_dev = plan.stats[2:3]
    cal = vx.LodPlan(wl.grid, leaf, n_dev, levels).run()
    caps = [max(v.n, 1) for v in cal.check()[1:]]
    del cal
    lod = vx.LodPlan(wl.grid, leaf, n_dev, levels, K=K, iters=2, caps=caps).run()
    out = lod.check()
    out[0].plan = plan
    return out, lod.lobes


def _u64(t):
    import torch
    return t.to(torch.int64) & 0xFFFFFFFF if t.dtype == torch.int32 else t


def _same(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a, b)


def _check_patch_vs_single(plan, p, lv, lobes, what):
    """Bit-exact comparison on the GPU of patch p's levels with the single-instance levels."""
    import torch
    n_lv = len(lv)
    tb = plan.table
    M = (1 << 33) - 1
    if lv[-1].n == 0:                # no pairs at all: the patch owns no voxel on any level
        assert np.all(tb[:, p] == tb[:, p + 1]), what
        return
    for L in range(plan.levels):
        a, b = int(tb[L, p]), int(tb[L, p + 1])
        o = plan.out[L]
        src = min(L, n_lv - 1)       # a shallow patch keeps its root above its own pyramid
        s = lv[src]
        if L >= n_lv:
            assert b - a == 1 and s.n == 1, (what, L, a, b, s.n)
            assert int(o.keys[a]) & M == 0, (what, L)
            assert int(o.count[a]) == int(s.count[0]) and float(o.w[a]) == float(s.w[0]), (what, L)
            assert torch.equal(o.S[:, a], s.S[:, 0]), (what, L)
            assert int(o.mask[a]) == 1, (what, L)
            if plan.lobes:
                lb = plan.lobes[L - 1]
                sw = float(s.w[0])
                assert abs(float(lb.w[:, a].double().sum()) - sw) <= 1e-5 * max(sw, 1e-2), (what, L)
            continue
        n = s.n
        assert b - a == n, (what, L, b - a, n)
        assert _same(o.keys[a:b] & M, _u64(s.keys[:n])), (what, L, "keys")
        assert _same(o.count[a:b], s.count[:n]), (what, L, "count")
        assert _same(o.w[a:b], s.w[:n]), (what, L, "w")
        assert _same(o.S[:, a:b], s.S[:, :n]), (what, L, "S")
        if L > 0:
            assert _same(o.mask[a:b], s.mask[:n]), (what, L, "mask")
            if plan.lobes:
                gb, sb = plan.lobes[L - 1], lobes[L - 1]
                assert _same(gb.nl[a:b], sb.nl[:n]), (what, L, "nl")
                assert _same(gb.w[:, a:b], sb.w[:, :n]), (what, L, "lobe w")
                assert _same(gb.S[:, :, a:b], sb.S[:, :, :n]), (what, L, "lobe S")


def _check_patch_vs_oracle(plan, p, wl, K, what):
    ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius)
    levels = wl.grid.log2_res + 1
    lod = oracle.build_lod(ref, levels)
    olobes = oracle.cluster_pyramid(lod, K, 2) if K > 1 else None
    for L in range(levels):
        d = plan.patch_level(p, L)
        o = lod[L]
        compare_level(d, o.keys, o.count, o.w, o.S, o.mask if L > 0 else None, what=f"{what} L{L}")
        if L > 0 and olobes is not None:
            g = {"nl": d["nl"], "w": d["lw"], "S": d["lS"]}
            compare_lobes(g, olobes[L], o.w, o.S, K, what=f"{what} lobes L{L}")


@pytest.mark.parametrize("K", [1, 4])
def test_small_batch_vs_single_and_oracle(vx, K):
    wls = _small_batch(21)
    say(f"case: small uneven batch of {len(wls)} patches, K={K}")
    plan = vx.BatchPlan(_patches(vx, wls), K=K, iters=2)
    plan.run()
    plan.check()
    assert plan.levels == max(w.grid.log2_res for w in wls) + 1
    for p, wl in enumerate(wls):
        lv, lobes = _single(vx, wl, K)
        if lv is None:
            assert np.all(plan.table[:, p] == plan.table[:, p + 1]), "empty patch owns voxels"
            continue
        _check_patch_vs_single(plan, p, lv, lobes, f"patch {p}")
        _check_patch_vs_oracle(plan, p, wl, K, f"patch {p}")
    say("pairs", plan.n_pairs, "voxels per level", [v.n for v in plan.out])


def test_graph_replay_matches_eager(vx):
    import torch
    wls = _small_batch(5)
    say("case: small uneven batch, graph capture and 3 replays")
    plan = vx.BatchPlan(_patches(vx, wls), K=4, iters=2)
    plan.run()
    plan.check()
    ref = [(v.keys[:v.n].clone(), v.count[:v.n].clone(), v.w[:v.n].clone(), v.S[:, :v.n].clone()) for v in plan.out]
    ref_lobes = [(lb.nl[:lb.n].clone(), lb.w[:, :lb.n].clone(), lb.S[:, :, :lb.n].clone()) for lb in plan.lobes]
    table = plan.table.copy()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = plan.capture(stream)
    other = synth.random_fibers(8, 30, 6, seed=99)
    for rep in range(3):
        # eager work between replays: clear the outputs and run an unrelated single-instance build
        for v in plan.out:
            v.keys.zero_()
            v.w.zero_()
            v.S.zero_()
        for lb in plan.lobes:
            lb.w.zero_()
        vx.voxelize_fibers(torch.as_tensor(other.pts).cuda(), torch.as_tensor(other.offsets).cuda(), 0.5,
                           other.grid)
        torch.cuda.synchronize()
        g.replay(stream)
        stream.synchronize()
        plan.check()
        assert np.array_equal(plan.table, table), rep
        for L, (v, r) in enumerate(zip(plan.out, ref)):
            assert v.n == r[0].numel(), (rep, L)
            assert torch.equal(v.keys[:v.n], r[0]) and torch.equal(v.count[:v.n], r[1]), (rep, L)
            assert torch.equal(v.w[:v.n], r[2]) and torch.equal(v.S[:, :v.n], r[3]), (rep, L)
        for L, (lb, r) in enumerate(zip(plan.lobes, ref_lobes)):
            assert torch.equal(lb.nl[:lb.n], r[0]) and torch.equal(lb.w[:, :lb.n], r[1]), (rep, L)
            assert torch.equal(lb.S[:, :, :lb.n], r[2]), (rep, L)
        say("replay", rep, "ok")
    del g


def test_tunings_do_not_change_results(vx):
    """Tile edge, unit budget and launch grids change the decomposition, never a bit of the result:
    a small uneven batch (fibers) and a brushed-metal window (triangles, 64-bit keys, K = 4)."""
    import torch
    import synth
    wls = _small_batch(8)
    say("case: small uneven batch and a brushed-metal window under other tunings")
    tunings = [vx.Tuning(3, 1024, (64, 64, 64, 64, 64)), vx.Tuning(4, 1536, (4096, 256, 16384, 512, 2048)),
               vx.Tuning(2, 2048, (0, 0, 0, 0, 0)), vx.Tuning(4, 3072, (128, 8192, 256, 16384, 64))]
    plan = vx.BatchPlan(_patches(vx, wls), K=4, iters=2)
    plan.run()
    plan.check()
    ref = [(v.keys[:v.n].clone(), v.w[:v.n].clone(), v.S[:, :v.n].clone()) for v in plan.out]
    ref_l = [lb.S[:, :, :lb.n].clone() for lb in plan.lobes]
    for t in tunings:
        p2 = vx.BatchPlan(_patches(vx, wls), K=4, iters=2, tuning=t)
        p2.run()
        p2.check()
        for v, r in zip(p2.out, ref):
            assert torch.equal(v.keys[:v.n], r[0]) and torch.equal(v.w[:v.n], r[1])
            assert torch.equal(v.S[:, :v.n], r[2])
        for lb, r in zip(p2.lobes, ref_l):
            assert torch.equal(lb.S[:, :, :lb.n], r)
        say("batch", t, "ok")
    wl = synth.brushed_metal(window=96)
    tris = torch.as_tensor(wl.tris).cuda()
    base = vx.voxelize_triangles(tris, wl.grid)
    lod0, lobes0 = vx.build_lod(wl.grid, base, 6, K=4, return_lobes=True)
    for t in tunings:
        v = vx.voxelize_triangles(tris, wl.grid, tuning=t)
        assert v.n == base.n
        for name in ("keys", "count", "w", "S"):
            assert torch.equal(getattr(v, name)[..., :v.n], getattr(base, name)[..., :v.n]), (t, name)
        lod, lobes = vx.build_lod(wl.grid, v, 6, K=4, return_lobes=True, tuning=t)
        for a, b in zip(lod[1:], lod0[1:]):
            assert torch.equal(a.w[:a.n], b.w[:b.n]) and torch.equal(a.S[:, :a.n], b.S[:, :b.n])
        for a, b in zip(lobes, lobes0):
            assert torch.equal(a.S[:, :, :a.n], b.S[:, :, :b.n])
        say("triangles", t, "ok")
    with pytest.raises(vx.VxError):
        vx.voxelize_triangles(tris, wl.grid, tuning=vx.Tuning(0, 1000))


def test_batch_errors(vx):
    import torch
    wls = _small_batch(3)[:2]
    say("case: batch argument errors")
    pats = _patches(vx, wls)
    plan = vx.BatchPlan(pats, K=1)
    L = vx.load()
    cp = plan._cp
    good = cp[1].pt_begin
    cp[1].pt_begin = good + 1                # ranges must tile the point array
    with pytest.raises(vx.VxError):
        plan.run()
    cp[1].pt_begin = good
    lr = cp[0].grid.log2_res
    cp[0].grid.log2_res = 12                 # above the 33-bit Morton field
    with pytest.raises(vx.VxError):
        plan.run()
    cp[0].grid.log2_res = lr
    plan.run()
    plan.check()
    assert L.vx_batch_workspace_size(0, 10, 10, 10, 10) == 0


@pytest.mark.timeout(900)
def test_full_uneven_batch_equals_single_runs(vx):
    """64 patches, fiber counts log-uniform in [100, 20000], grids 256^3 .. 2048^3, K = 4."""
    import torch
    wls = synth.weave_patches()
    say(f"case: full uneven batch, {len(wls)} patches, {sum(len(w.offsets) - 1 for w in wls)} fibers")
    plan = vx.BatchPlan(_patches(vx, wls), K=4, iters=2)
    plan.run()
    plan.check()
    say("pairs", plan.n_pairs, "leaf voxels", plan.out[0].n)
    for p, wl in enumerate(wls):
        lv, lobes = _single(vx, wl, 4)
        _check_patch_vs_single(plan, p, lv, lobes, f"patch {p}")
        del lv, lobes
        if p % 16 == 15:
            say("patches up to", p, "equal")
            torch.cuda.empty_cache()
    sizes = [len(w.offsets) * (1 << w.grid.log2_res) for w in wls]
    for p in np.argsort(sizes)[:2]:
        say("oracle parity for patch", int(p), "fibers", len(wls[p].offsets) - 1, "R", 1 << wls[p].grid.log2_res)
        _check_patch_vs_oracle(plan, int(p), wls[p], 4, f"patch {int(p)}")
