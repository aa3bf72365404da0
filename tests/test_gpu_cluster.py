"""GPU parity of the Sec. 4.4 lobe clustering (K > 1) against the oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import compare_lobes, compare_pyramid

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _random_leaf(seed, log2_res, n, families=None):
    """Distinct random leaf voxels with fiber-like lobes S = w (I - t t^T); with `families`,
    tangents are drawn near a few directions so that merges are clear."""
    rng = np.random.default_rng(seed)
    R = 1 << log2_res
    coords = rng.choice(R ** 3, size=n, replace=False)
    x, y, z = coords % R, (coords // R) % R, coords // (R * R)
    keys = np.array([oracle.morton(a, b, c, log2_res) for a, b, c in zip(x, y, z)], dtype=np.uint64)
    order = np.argsort(keys)
    keys = keys[order]
    w = rng.uniform(0.1, 2.0, n).astype(np.float32)
    if families is None:
        t = rng.normal(size=(n, 3))
    else:
        base = rng.normal(size=(families, 3))
        t = base[rng.integers(0, families, n)] + 0.05 * rng.normal(size=(n, 3))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    M = np.stack([1 - t[:, 0] ** 2, 1 - t[:, 1] ** 2, 1 - t[:, 2] ** 2, -t[:, 0] * t[:, 1], -t[:, 0] * t[:, 2],
                  -t[:, 1] * t[:, 2]], 1)
    S = (w[:, None] * M).astype(np.float32)
    cnt = rng.integers(1, 5, n).astype(np.uint32)
    return keys, cnt, w, S


def _leaf_to_device(vx, keys, cnt, w, S, log2_res):
    import torch
    n = len(keys)
    v = vx.alloc_voxels(n, log2_res, "cuda", False)
    kd = keys.astype(np.int64) if log2_res > 10 else keys.astype(np.uint32).view(np.int32)
    v.keys.copy_(torch.as_tensor(kd))
    v.count.copy_(torch.as_tensor(cnt.view(np.int32)))
    v.w.copy_(torch.as_tensor(w))
    v.S.copy_(torch.as_tensor(np.ascontiguousarray(S.T)))
    v.n = n
    return v


@pytest.mark.parametrize("K,families", [(2, 2), (4, 3), (4, None), (8, 5)])
def test_cluster_on_given_leaf(vx, K, families):
    """The clustering alone: the same FP32 leaf goes to the GPU and (as FP64) to the oracle."""
    log2_res = 5
    keys, cnt, w, S = _random_leaf(300 + K, log2_res, 6000, families)
    say(f"case: given leaf, 32^3, K={K}, families={families}")
    grid = synth.Grid((0.0, 0.0, 0.0), 32.0, log2_res)
    leaf = _leaf_to_device(vx, keys, cnt, w, S, log2_res)
    pyr, lobes = vx.build_lod(grid, leaf, log2_res + 1, K=K, iters=2, return_lobes=True)
    ref = oracle.Voxels(keys, cnt, w.astype(np.float64), S.astype(np.float64), int(cnt.sum()))
    lod = oracle.build_lod(ref, log2_res + 1)
    compare_pyramid(pyr, lod, f"given leaf K{K}")
    olobes = oracle.cluster_pyramid(lod, K, 2)
    for L in range(1, log2_res + 1):
        rep = compare_lobes(lobes[L - 1].numpy(), olobes[L], lod[L].w, lod[L].S, K, what=f"K{K} L{L}")
        say(L, rep)


def test_cluster_brushed_metal_window(vx):
    wl = synth.brushed_metal(window=128)
    say("case: brushed metal 128x128 window, 4096^3, 13 levels, K=4")
    import torch
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    pyr, lobes = vx.build_lod(wl.grid, leaf, wl.levels, K=4, iters=2, return_lobes=True)
    ref = oracle.voxelize_triangles(wl.grid, wl.tris)
    lod = oracle.build_lod(ref, wl.levels)
    compare_pyramid(pyr, lod, "brushed128")
    olobes = oracle.cluster_pyramid(lod, 4, 2)
    for L in range(1, wl.levels):
        rep = compare_lobes(lobes[L - 1].numpy(), olobes[L], lod[L].w, lod[L].S, 4, what=f"brushed L{L}")
        say(L, rep)


def test_cluster_weave(vx):
    wl = synth.plain_weave(n_fibers=128, seed=12)
    say("case: plain weave 128 fibers, 1024^3, 11 levels, K=4")
    import torch
    leaf = vx.voxelize_fibers(torch.as_tensor(wl.pts).cuda(), torch.as_tensor(wl.offsets).cuda(), wl.radius,
                              wl.grid)
    pyr, lobes = vx.build_lod(wl.grid, leaf, wl.levels, K=4, iters=2, return_lobes=True)
    ref = oracle.voxelize_fibers(wl.grid, wl.pts, wl.offsets, wl.radius)
    lod = oracle.build_lod(ref, wl.levels)
    olobes = oracle.cluster_pyramid(lod, 4, 2)
    for L in range(1, wl.levels):
        rep = compare_lobes(lobes[L - 1].numpy(), olobes[L], lod[L].w, lod[L].S, 4, what=f"weave L{L}")
        say(L, rep)


def test_brushed_metal_full_sampled_regions(vx):
    """The brushed-metal height field at full size (33,538,050 triangles, 4096^3, 64-bit keys,
    13 levels, K = 4): on sampled 32^3 regions the leaf, levels 1-5 and their lobes against the
    oracle restricted to the same regions; over the whole grid, conservation of area."""
    import torch
    from parity import compare_level
    n = 4096
    wl = synth.brushed_metal(n=n)
    say("case: brushed metal full 4096x4096 vertices (33.5M triangles), 4096^3, 13 levels, K=4, sampled regions")
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    pyr, lobes = vx.build_lod(wl.grid, leaf, wl.levels, K=4, iters=2, return_lobes=True)
    torch.cuda.synchronize()
    say("gpu done:", leaf.plan.n_pairs, "pairs,", [p.n for p in pyr[:3]], "voxels in levels 0-2")
    g0 = pyr[0].numpy()
    # every triangle lies inside the grid: the leaf holds the whole area (FP32 sums, FP64 total)
    t = wl.tris.astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]), axis=1).sum()
    assert abs(g0["w"].astype(np.float64).sum() - area) <= 1e-5 * area
    assert abs(pyr[-1].numpy()["w"].astype(np.float64).sum() - area) <= 1e-5 * area
    # surface lobes S = w n n^T: trace w
    assert np.allclose(g0["S"][:, :3].sum(1), g0["w"], rtol=1e-5, atol=1e-6)
    rng = np.random.default_rng(11)
    corners = [(0, 0), (n - 32, n - 32), (n // 2, n // 2)]
    corners += [tuple(int(32 * v) for v in rng.integers(0, n // 32, 2)) for _ in range(3)]
    levels_gpu = [p.numpy() for p in pyr[:6]]
    lobes_gpu = [lb.numpy() for lb in lobes[:5]]
    for r, (x0, y0) in enumerate(corners):
        # the surface lies within 2 voxels of z = n / 2, a block boundary: take both sides
        z0 = n // 2 - 32 if r % 2 else n // 2
        lo = np.array([x0, y0, z0])
        hi = lo + 32
        # the triangles of the cells around the region (the oracle clips to the region itself)
        i0, i1 = max(x0 - 2, 0), min(x0 + 34, n - 1)
        j0, j1 = max(y0 - 2, 0), min(y0 + 34, n - 1)
        ii, jj = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1), indexing="ij")
        cell = (ii * (n - 1) + jj).ravel()
        sel_t = np.stack([2 * cell, 2 * cell + 1], 1).ravel()
        ref = oracle.voxelize_triangles(wl.grid, wl.tris[sel_t], region=np.concatenate([lo, hi]))
        lod = oracle.build_lod(ref, 6)
        olobes = oracle.cluster_pyramid(lod, 4, 2)
        for L in range(6):
            g = levels_gpu[L]
            c = oracle.demorton(g["keys"].astype(np.uint64), wl.grid.log2_res - L)
            sel = np.all((c >= (lo >> L)) & (c < (hi >> L)), axis=1)
            sub = {k: v[sel] for k, v in g.items()}
            o = lod[L]
            rep = compare_level(sub, o.keys, o.count, o.w, o.S, o.mask if L > 0 else None,
                                what=f"brushed full region {lo.tolist()} L{L}")
            assert rep["n"] > 0
            if L > 0:
                gl = {k: v[sel] for k, v in lobes_gpu[L - 1].items()}
                compare_lobes(gl, olobes[L], o.w, o.S, 4, what=f"brushed full region {lo.tolist()} L{L}")
        say("region", lo.tolist(), "ok:", rep)


def _stepwise(pyr, lobes, lod, K, what, min_checked_from_level3=1):
    """Every level clustered again by the oracle from the GPU's own lobes of the level below."""
    from parity import compare_lobes_stepwise, gpu_lobes_as_oracle, leaf_as_oracle_lobes
    child = leaf_as_oracle_lobes(pyr[0].numpy())
    deep = 0
    for L in range(1, len(pyr)):
        g = lobes[L - 1].numpy()
        rep = compare_lobes_stepwise(g, child, lod[L].child_start, K, what=f"{what} L{L}")
        say(what, "level", L, rep)
        if L >= 3:
            deep += rep["checked_exactly_merging"]
        child = gpu_lobes_as_oracle(g)
    assert deep >= min_checked_from_level3, (what, deep)


def test_cluster_levels_stepwise_brushed(vx):
    """Brushed metal 256x256 window, K = 4: each level's merges checked on that level's inputs."""
    import torch
    wl = synth.brushed_metal(window=256)
    say("case: brushed metal 256x256 window, stepwise clustering check, K=4")
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    pyr, lobes = vx.build_lod(wl.grid, leaf, wl.levels, K=4, iters=2, return_lobes=True)
    ref = oracle.voxelize_triangles(wl.grid, wl.tris)
    lod = oracle.build_lod(ref, wl.levels)
    _stepwise(pyr, lobes, lod, 4, "brushed256", min_checked_from_level3=100)


@pytest.mark.parametrize("K", [2, 4, 8])
def test_cluster_levels_stepwise_given_leaf(vx, K):
    keys, cnt, w, S = _random_leaf(500 + K, 6, 40000, None)
    say(f"case: given leaf, 64^3, stepwise clustering check, K={K}")
    grid = synth.Grid((0.0, 0.0, 0.0), 64.0, 6)
    leaf = _leaf_to_device(vx, keys, cnt, w, S, 6)
    pyr, lobes = vx.build_lod(grid, leaf, 7, K=K, iters=2, return_lobes=True)
    ref = oracle.Voxels(keys, cnt, w.astype(np.float64), S.astype(np.float64), int(cnt.sum()))
    lod = oracle.build_lod(ref, 7)
    _stepwise(pyr, lobes, lod, K, f"given K{K}", min_checked_from_level3=10)
