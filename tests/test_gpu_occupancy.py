"""GPU parity of the sub-voxel occupancy (Sec. 3.5 occupancy and projections, Sec. 4.2 coarser
levels) against its oracle, through the C ABI: masks, hit counts and the XY / XZ / YZ cell counts
bit-exact at every level."""
import sys

import numpy as np
import pytest

import oracle
from oracle.occupancy import occupancy_fibers, occupancy_triangles
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _pyramid(vx, kind, grid, data, levels, offsets=None, radius=0.0):
    plan = vx.VoxelizePlan(kind, grid, data, offsets=offsets, radius=radius).run()
    leaf = plan.check()
    lod = vx.LodPlan(grid, leaf, plan.stats[2:3], levels).run()
    lod.check()
    occ = vx.OccupancyPlan(kind, grid, data, lod, offsets=offsets, radius=radius).run()
    return lod, occ.check(), occ


def compare(lod, occ, ref, what, upto=None):
    levels = [lod.leaf] + lod.out
    for L in range(len(ref) if upto is None else upto):
        keys = levels[L].numpy()["keys"].astype(np.uint64)
        g = occ[L].numpy()
        r = ref[L]
        assert np.array_equal(keys, r.keys), f"{what} L{L}: keys"
        if not np.array_equal(g["mask"], r.mask):
            bad = np.flatnonzero((g["mask"] != r.mask).any(1))[:4]
            raise AssertionError(f"{what} L{L}: masks differ at {bad.tolist()}: {g['mask'][bad]} vs {r.mask[bad]}")
        for f in ("hits", "xy", "xz", "yz"):
            assert np.array_equal(g[f], getattr(r, f)), f"{what} L{L}: {f}"
    return {"levels": len(ref), "leaf_voxels": len(ref[0].keys), "mean_hits": float(ref[0].hits.mean())}


def test_icosphere_all_levels(vx):
    wl = synth.icosphere()
    say("case: occupancy, icosphere 20480 tris, 64^3, 7 levels")
    lod, occ, _ = _pyramid(vx, 0, wl.grid, _dev(wl.tris), wl.levels)
    say(compare(lod, occ, occupancy_triangles(wl.grid, wl.tris, wl.levels), "icosphere"))


@pytest.mark.parametrize("seed", [1, 2])
def test_random_triangles_and_fibers(vx, seed):
    tw = synth.random_triangles(60, 4, seed=seed, scale=3.0, margin=1.5)
    say(f"case: occupancy, random triangles 60 (seed {seed}), 16^3, 5 levels")
    lod, occ, _ = _pyramid(vx, 0, tw.grid, _dev(tw.tris), 5)
    compare(lod, occ, occupancy_triangles(tw.grid, tw.tris, 5), "random triangles")
    fw = synth.random_fibers(5, 14, 4, seed=seed, step=1.4, margin=1.0)
    say(f"case: occupancy, random fibers 5 x 14 (seed {seed}), radius 0.7, 16^3, 5 levels")
    lod, occ, _ = _pyramid(vx, 1, fw.grid, _dev(fw.pts), 5, _dev(fw.offsets), 0.7)
    compare(lod, occ, occupancy_fibers(fw.grid, fw.pts, fw.offsets, 0.7, 5), "random fibers")


def test_lattice_aligned_cases(vx):
    """Flat triangles on a sub-cell boundary and on a voxel face, and a fiber along a sub-cell
    edge with a radius of whole sub-cells: every closed-box tie at once."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    tris = np.array([[[0.75, 1.125, 2.5], [6.25, 1.125, 2.5], [0.75, 5.375, 2.5]],
                     [[1.5, 0.5, 3.0], [7.0, 0.5, 3.0], [1.5, 6.0, 3.0]],
                     [[2.25, 2.0, 0.5], [2.25, 6.0, 0.5], [2.25, 2.0, 7.25]]], np.float32)
    say("case: occupancy, lattice-aligned triangles and fiber, 8^3, 4 levels")
    lod, occ, _ = _pyramid(vx, 0, grid, _dev(tris), 4)
    compare(lod, occ, occupancy_triangles(grid, tris, 4), "aligned triangles")
    pts = np.array([[1.25, 3.25, 4.5], [6.5, 3.25, 4.5], [6.5, 5.125, 2.0]], np.float32)
    lod, occ, _ = _pyramid(vx, 1, grid, _dev(pts), 4, _dev(np.array([0, 3])), 0.375)
    compare(lod, occ, occupancy_fibers(grid, pts, [0, 3], 0.375, 4), "aligned fiber")


def test_weave_small(vx):
    wl = synth.plain_weave(n_fibers=16, seed=5)
    say("case: occupancy, plain weave 16 fibers x 256 segments, radius 0.5, 1024^3, 4 levels")
    lod, occ, _ = _pyramid(vx, 1, wl.grid, _dev(wl.pts), 4, _dev(wl.offsets), wl.radius)
    say(compare(lod, occ, occupancy_fibers(wl.grid, wl.pts, wl.offsets, wl.radius, 4), "weave16"))


def test_brushed_metal_window(vx):
    wl = synth.brushed_metal(window=96)
    say("case: occupancy, brushed metal 96^2 window, 4096^3, 5 levels")
    lod, occ, _ = _pyramid(vx, 0, wl.grid, _dev(wl.tris), 5)
    say(compare(lod, occ, occupancy_triangles(wl.grid, wl.tris, 5), "brushed window"))


def test_brushed_metal_full_sampled_regions(vx):
    """The full surface: levels 0-3 inside sampled 32 x 32 columns (aligned to 8 voxels, so a
    coarse voxel's children all lie inside) against the oracle over the triangles reaching them."""
    wl = synth.brushed_metal()
    say("case: occupancy, brushed metal full size, levels 0-3 in sampled regions")
    lod, occ, _ = _pyramid(vx, 0, wl.grid, _dev(wl.tris), 4)
    levels = [lod.leaf] + lod.out
    gk = [lv.numpy()["keys"].astype(np.uint64) for lv in levels]
    go = [o.numpy() for o in occ]
    gc = [oracle.demorton(gk[L], wl.grid.log2_res - L) << L for L in range(4)]
    t = wl.tris
    lo_t, hi_t = t.min(1), t.max(1)
    rng = np.random.default_rng(4)
    for x0, y0 in (rng.integers(0, 4096 // 8 - 4, size=(3, 2)) * 8):
        sel = np.flatnonzero((hi_t[:, 0] >= x0) & (lo_t[:, 0] <= x0 + 32) & (hi_t[:, 1] >= y0) &
                             (lo_t[:, 1] <= y0 + 32))
        ref = occupancy_triangles(wl.grid, t[sel], 4)
        for L in range(4):
            sz = 1 << L

            def inside(c):
                return (c[:, 0] >= x0) & (c[:, 0] + sz <= x0 + 32) & (c[:, 1] >= y0) & (c[:, 1] + sz <= y0 + 32)
            mg = inside(gc[L])
            mr = inside(oracle.demorton(ref[L].keys, wl.grid.log2_res - L) << L)
            assert np.array_equal(gk[L][mg], ref[L].keys[mr]), (x0, y0, L)
            assert np.array_equal(go[L]["mask"][mg], ref[L].mask[mr]), (x0, y0, L)
            for f in ("hits", "xy", "xz", "yz"):
                assert np.array_equal(go[L][f][mg], getattr(ref[L], f)[mr]), (x0, y0, L, f)
        say(f"region ({x0}, {y0}): {int(mg.sum())} level-3 voxels, {len(sel)} triangles")


def test_errors(vx):
    a = synth.random_triangles(20, 4, seed=3, scale=2.0)
    b = synth.random_triangles(20, 4, seed=4, scale=2.0)
    grid = a.grid
    plan = vx.VoxelizePlan(0, grid, _dev(a.tris)).run()
    leaf = plan.check()
    lod = vx.LodPlan(grid, leaf, plan.stats[2:3], 3).run()
    lod.check()
    with pytest.raises(vx.VxError) as e:                # occupancy of other triangles than the leaf's
        o = vx.OccupancyPlan(0, grid, _dev(b.tris), lod).run()
        o.check()
    assert e.value.status == 6
    big = synth.Grid((0.0, 0.0, 0.0), 16.0, 18)
    with pytest.raises(vx.VxError):                     # log2_res above 17
        vx.OccupancyPlan(0, big, _dev(a.tris), lod)
