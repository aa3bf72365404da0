"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Keys, counts and child masks bit-exact; w and S within the bar in tests/parity.py.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_level, compare_pyramid

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _levels(vx, grid, leaf, levels):
    return vx.build_lod(grid, leaf, levels)


def test_icosphere_64(vx):
    wl = synth.icosphere()
    say("case: icosphere 20480 tris, 64^3, 7 levels")
    leaf = vx.voxelize_triangles(_dev(wl.tris), wl.grid)
    ref = oracle.voxelize_triangles(wl.grid, wl.tris)
    assert leaf.plan.n_pairs == ref.n_pairs
    pyr = _levels(vx, wl.grid, leaf, wl.levels)
    reps = compare_pyramid(pyr, oracle.build_lod(ref, wl.levels), "icosphere")
    say(reps[0])


def test_weave_small(vx):
    wl = synth.plain_weave(n_fibers=96, seed=5)
    say("case: plain weave 96 fibers x 256 segments, 1024^3, 11 levels")
    leaf = vx.voxelize_fibers(_dev(wl.pts), _dev(wl.offsets), wl.radius, wl.grid)
    ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius)
    assert leaf.plan.n_pairs == ref.n_pairs
    pyr = _levels(vx, wl.grid, leaf, wl.levels)
    reps = compare_pyramid(pyr, oracle.build_lod(ref, wl.levels), "weave96")
    say(reps[0])


def test_weave_full_sampled_regions(vx):
    """The measured workload at full size: GPU result on sampled 32^3 regions against the oracle
    restricted to the same regions, plus conservation of length and of the moment."""
    wl = synth.plain_weave()
    say("case: plain weave 2000 fibers full size, sampled regions")
    leaf = vx.voxelize_fibers(_dev(wl.pts), _dev(wl.offsets), wl.radius, wl.grid)
    g = leaf.numpy()
    coords = oracle.demorton(g["keys"].astype(np.uint64), wl.grid.log2_res)
    rng = np.random.default_rng(7)
    regions = [(0, 0, 496), (992, 992, 496), (480, 480, 500)]
    regions += [tuple(int(v) for v in rng.integers(0, 1024 - 32, 2)) + (int(rng.integers(496, 500)),) for _ in range(5)]
    for (x0, y0, z0) in regions:
        lo = np.array([x0, y0, z0])
        hi = lo + 32
        ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius, region=np.concatenate([lo, hi]))
        sel = np.all((coords >= lo) & (coords < hi), axis=1)
        sub = {k: v[sel] for k, v in g.items()}
        rep = compare_level(sub, ref.keys, ref.count, ref.w, ref.S, what=f"region {lo.tolist()}")
        assert rep["n"] > 0 or z0 > 510
    # every point lies inside the grid, so the length is conserved (FP32 sums vs FP64 total)
    q = oracle.snap(wl.grid, wl.pts).reshape(2000, 257, 3).astype(np.float64)
    d = (q[:, 1:] - q[:, :-1]).reshape(-1, 3) / float(1 << (23 - wl.grid.log2_res))
    L = np.linalg.norm(d, axis=1)
    assert abs(g["w"].astype(np.float64).sum() - L.sum()) <= 1e-5 * L.sum()
    assert np.allclose(g["S"][:, :3].sum(1), 2 * g["w"], rtol=1e-5, atol=1e-6)


def test_weave_full_every_voxel_all_levels(vx):
    """The plain weave at full size (2,000 fibers x 256 segments, 1024^3): every voxel of the leaf
    and of all 10 levels above it against the oracle's full build (keys, counts and masks exact,
    w and S to the 1e-5 bar), and the pair count."""
    wl = synth.plain_weave()
    say("case: plain weave 2000 fibers full size, every voxel of all 11 levels")
    leaf = vx.voxelize_fibers(_dev(wl.pts), _dev(wl.offsets), wl.radius, wl.grid)
    pyr = _levels(vx, wl.grid, leaf, wl.levels)
    ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius)
    assert leaf.plan.n_pairs == ref.n_pairs
    reps = compare_pyramid(pyr, oracle.build_lod(ref, wl.levels), "weave full")
    say("levels:", [r["n"] for r in reps], "worst w/S:", max(r["max_rel_w"] for r in reps),
        max(r["max_rel_S"] for r in reps))


def test_brushed_metal_window_64bit_keys(vx):
    wl = synth.brushed_metal(n=4096, window=96)
    say("case: brushed metal 96x96 window, 4096^3 (64-bit keys), 13 levels")
    leaf = vx.voxelize_triangles(_dev(wl.tris), wl.grid)
    ref = oracle.voxelize_triangles(wl.grid, wl.tris)
    assert leaf.plan.n_pairs == ref.n_pairs
    pyr = _levels(vx, wl.grid, leaf, wl.levels)
    compare_pyramid(pyr, oracle.build_lod(ref, wl.levels), "brushed96")


def _adversarial_triangles(seed, R, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        kind = i % 5
        if kind == 0:
            t = rng.integers(-2, 2 * R + 3, size=(3, 3)) / 2.0
        elif kind == 1:
            t = rng.integers(0, 2 * R + 1, size=(3, 3)) / 2.0
            t[:, i % 3] = rng.integers(0, R + 1)
        elif kind == 2:
            a = rng.integers(0, 2 * R, size=3) / 2.0
            d = rng.integers(-2, 3, size=3) / 2.0
            t = np.stack([a, a + d, a + 2 * d])
        elif kind == 3:
            t = rng.uniform(-0.9 * R, 1.9 * R, size=(3, 3))
        else:
            t = np.clip(rng.uniform(0, R, size=(1, 3)) + rng.normal(0, 1.5, size=(3, 3)), -0.9 * R, 1.9 * R)
        out.append(t)
    return np.array(out, dtype=np.float32)


@pytest.mark.parametrize("log2_res", [2, 4, 6])
def test_adversarial_triangles(vx, log2_res):
    R = 1 << log2_res
    grid = synth.Grid((0.0, 0.0, 0.0), float(R), log2_res)
    tris = _adversarial_triangles(100 + log2_res, R, 600)
    say(f"case: adversarial triangles R={R}")
    leaf = vx.voxelize_triangles(_dev(tris), grid)
    ref = oracle.voxelize_triangles(grid, tris)
    compare_level(leaf.numpy(), ref.keys, ref.count, ref.w, ref.S, what=f"adv tris R{R}")


def _adversarial_fibers(seed, R, n_fib):
    """Axis-parallel runs on half-voxel positions (distance ties with r = 0.5), zero-length
    segments and random walks, some leaving the grid."""
    rng = np.random.default_rng(seed)
    pts, offs = [], [0]
    for f in range(n_fib):
        kind = f % 4
        if kind == 0:
            a = rng.integers(0, 2 * R, size=3) / 2.0
            axis = rng.integers(0, 3)
            k = rng.integers(2, 6)
            p = np.repeat(a[None], k, 0)
            p[:, axis] += np.arange(k) * rng.integers(1, 4) / 2.0
        elif kind == 1:
            a = rng.integers(0, 2 * R, size=3) / 2.0
            p = np.stack([a, a, a + np.array([0.5, 0.0, 0.0])])
        elif kind == 2:
            p = rng.uniform(-0.5 * R, 1.5 * R, size=(4, 3))
        else:
            p = np.clip(rng.uniform(0, R, size=(1, 3)) + np.cumsum(rng.normal(0, 1.0, size=(6, 3)), 0),
                        -0.9 * R, 1.9 * R)
        pts.append(p)
        offs.append(offs[-1] + len(p))
    return np.concatenate(pts).astype(np.float32), np.array(offs, dtype=np.int64)


@pytest.mark.parametrize("log2_res,radius", [(3, 0.5), (5, 0.5), (5, 0.0), (6, 1.25)])
def test_adversarial_fibers(vx, log2_res, radius):
    R = 1 << log2_res
    grid = synth.Grid((0.0, 0.0, 0.0), float(R), log2_res)
    pts, offs = _adversarial_fibers(200 + log2_res, R, 400)
    say(f"case: adversarial fibers R={R} r={radius}")
    leaf = vx.voxelize_fibers(_dev(pts), _dev(offs), radius, grid)
    ref = oracle.voxelize_fibers(grid, pts, offs, radius)
    compare_level(leaf.numpy(), ref.keys, ref.count, ref.w, ref.S, what=f"adv fibers R{R} r{radius}")


def test_crowded_voxels(vx):
    """Voxels touched by more primitives than a unit holds (summed in streaming order), siblings
    of such voxels, and a crowded corner whose tile splits down to single cells and sibling
    groups; next to large primitives spanning many tiles."""
    R = 64
    grid = synth.Grid((0.0, 0.0, 0.0), float(R), 6)
    rng = np.random.default_rng(41)

    def tiny(n, lo, hi):
        c = rng.uniform(lo, hi, size=(n, 1, 3))
        return c + rng.uniform(-0.05, 0.05, size=(n, 3, 3))

    tris = np.concatenate([
        tiny(5000, 20.1, 20.9),                                            # one voxel, 5000 triangles
        tiny(3500, 20.1, 20.9) + np.array([1.0, 0.0, 0.0]),               # its sibling, 3500
        tiny(2500, 16.1, 19.9),                                            # a crowded 4^3 corner
        rng.uniform(0.0, R, size=(40, 3, 3)),                              # large triangles
    ]).astype(np.float32)
    say("case: crowded voxels, triangles R=64")
    leaf = vx.voxelize_triangles(_dev(tris), grid)
    ref = oracle.voxelize_triangles(grid, tris)
    assert leaf.plan.n_pairs == ref.n_pairs
    compare_pyramid(vx.build_lod(grid, leaf, 7), oracle.build_lod(ref, 7), "crowded tris")
    # fibers: 4000 short segments inside one voxel, random walks around them
    a = rng.uniform(30.2, 30.8, size=(4000, 1, 3))
    seg = np.concatenate([a, a + rng.uniform(-0.15, 0.15, size=(4000, 1, 3))], 1)
    walks = np.clip(30.5 + np.cumsum(rng.normal(0, 1.5, size=(300, 8, 3)), 1), 0.0, R)
    pts = np.concatenate([seg.reshape(-1, 3), walks.reshape(-1, 3)]).astype(np.float32)
    offs = np.concatenate([np.arange(0, 8001, 2), 8000 + np.arange(1, 301) * 8]).astype(np.int64)
    say("case: crowded voxels, fibers R=64 r=0.5")
    leaf = vx.voxelize_fibers(_dev(pts), _dev(offs), 0.5, grid)
    ref = oracle.voxelize_fibers(grid, pts, offs, 0.5)
    assert leaf.plan.n_pairs == ref.n_pairs
    compare_pyramid(vx.build_lod(grid, leaf, 7), oracle.build_lod(ref, 7), "crowded fibers")


@pytest.mark.parametrize("log2_res", [10, 11, 20])
def test_resolution_limits(vx, log2_res):
    """The last 32-bit-key grid, the first 64-bit one and the finest grid (8 lattice units per
    voxel): small primitives scattered over the whole grid, the full pyramid."""
    R = 1 << log2_res
    grid = synth.Grid((-0.5 * R, 0.25 * R, 3.0), float(R), log2_res)
    rng = np.random.default_rng(300 + log2_res)
    c = np.array(grid.bmin) + rng.uniform(0, R, size=(400, 1, 3))
    tris = (c + rng.normal(0, 1.5, size=(400, 3, 3))).astype(np.float32)
    say(f"case: triangles at R=2^{log2_res}")
    leaf = vx.voxelize_triangles(_dev(tris), grid)
    ref = oracle.voxelize_triangles(grid, tris)
    assert leaf.plan.n_pairs == ref.n_pairs
    compare_pyramid(vx.build_lod(grid, leaf, log2_res + 1), oracle.build_lod(ref, log2_res + 1), f"tris 2^{log2_res}")
    start = np.array(grid.bmin) + rng.uniform(0, R, size=(150, 1, 3))
    pts = (start + np.cumsum(rng.normal(0, 1.2, size=(150, 6, 3)), 1)).reshape(-1, 3).astype(np.float32)
    offs = np.arange(0, 151) * 6
    say(f"case: fibers at R=2^{log2_res}")
    leaf = vx.voxelize_fibers(_dev(pts), _dev(offs), 0.5, grid)
    ref = oracle.voxelize_fibers(grid, pts, offs, 0.5)
    assert leaf.plan.n_pairs == ref.n_pairs
    compare_pyramid(vx.build_lod(grid, leaf, log2_res + 1), oracle.build_lod(ref, log2_res + 1), f"fibers 2^{log2_res}")


def test_empty_and_outside(vx):
    grid = synth.Grid((0.0, 0.0, 0.0), 16.0, 4)
    say("case: empty input, all outside the grid")
    leaf = vx.voxelize_triangles(_dev(np.zeros((0, 3, 3), np.float32)), grid)
    assert leaf.n == 0
    tris = np.array([[[20, 20, 20], [21, 20, 20], [20, 21, 20]]], dtype=np.float32)
    leaf = vx.voxelize_triangles(_dev(tris), grid)
    assert leaf.n == 0 and leaf.plan.n_pairs == 0
    pts = np.array([[-3, 1, 1], [-2, 1, 1], [5, 5, 5]], dtype=np.float32)
    leaf = vx.voxelize_fibers(_dev(pts), _dev(np.array([0, 2, 3])), 0.5, grid)   # one segment outside, one 1-point fiber
    assert leaf.n == 0
    pyr = vx.build_lod(grid, leaf, 5)
    assert all(l.n == 0 for l in pyr)


def test_errors(vx):
    import torch
    grid = synth.Grid((0.0, 0.0, 0.0), 16.0, 4)
    say("case: error paths")
    tris = np.array([[[1, 1, 1], [2, 1, 1], [1, np.nan, 1]]], dtype=np.float32)
    with pytest.raises(vx.VxError) as e:
        vx.voxelize_triangles(_dev(tris), grid)
    assert e.value.status == 4
    far = np.array([[[1, 1, 1], [2, 1, 1], [1, 40, 1]]], dtype=np.float32)     # beyond one grid of margin
    with pytest.raises(vx.VxError) as e:
        vx.voxelize_triangles(_dev(far), grid)
    assert e.value.status == 4
    with pytest.raises(vx.VxError) as e:                                          # offsets not ending at n_pts
        vx.voxelize_fibers(_dev(np.zeros((4, 3), np.float32) + 1), _dev(np.array([0, 2, 3])), 0.5, grid)
    assert e.value.status == 4
    # capacity: the library reports the required size and refuses to write beyond the buffers
    wl = synth.icosphere(subdiv=2)
    t = _dev(wl.tris)
    plan = vx.VoxelizePlan(0, wl.grid, t)
    plan.run()
    n_vox = plan.check().n
    # each capacity one short: records, units, leaf voxels
    for kw, idx, need in (({"max_records": plan.max_records - 1}, vx.STAT_RECORDS, plan.max_records),
                          ({"max_units": plan.max_units - 1}, vx.STAT_UNITS, plan.max_units),
                          ({"out_cap": n_vox - 1}, vx.STAT_VOXELS, n_vox)):
        args = {"max_records": plan.max_records, "max_units": plan.max_units, "out_cap": n_vox}
        args.update(kw)
        small = vx.VoxelizePlan(0, wl.grid, t, **args)
        small.run()
        with pytest.raises(vx.VxError) as e:
            small.check()
        assert e.value.status == 2, kw
        assert int(small.stats[idx].item()) == need, kw
    plan.run()
    v = plan.check()
    ref = oracle.voxelize_triangles(wl.grid, wl.tris)
    compare_level(v.numpy(), ref.keys, ref.count, ref.w, ref.S, what="after capacity error")
    # host-checked arguments
    L = vx.load()
    assert L.vx_voxelize_workspace_size(0, 1 << 32, 10, 10, 10, 4) == 0
    assert L.vx_voxelize_workspace_size(2, 10, 10, 10, 10, 4) == 0
    bad = vx.CGrid((vx.ctypes.c_double * 3)(0, 0, 0), -1.0, 4)
    st = L.vx_voxelize_triangles(vx.ctypes.byref(bad), vx._ptr(t), 1, 0, 0, None, 0, None, vx._ptr(plan.stats), None,
                                 None)
    assert st == 1
    torch.cuda.synchronize()


def test_repeat_runs_identical(vx):
    """Deterministic: every voxel sums its pairs in primitive order whatever order the work is
    done in, so repeated runs give identical bits."""
    wl = synth.plain_weave(n_fibers=64, seed=9)
    say("case: repeatability")
    plan = vx.VoxelizePlan(1, wl.grid, _dev(wl.pts), offsets=_dev(wl.offsets), radius=wl.radius)
    a = plan.run().check().numpy()
    b = plan.run().check().numpy()
    for k in a:
        assert np.array_equal(a[k], b[k])
