"""GPU parity of the paper's SGGX-H lobe reduction (Sec. 4.4) against its oracle, level by level:
each level is reduced again by the oracle from the GPU's own lobes of the level below.  Both sides
draw the same samples (counter-based SplitMix64, decisions in IEEE double), so the number of lobes
is equal and every lobe's weight and moment agree within the FP32 sums of its members:
    |w - w_ref| <= 1e-5 max(w_ref, 1e-2),  max |S - S_ref| <= 1e-5 max(tr S_ref, 1e-2)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import gpu_lobes_as_oracle, leaf_as_oracle_lobes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare(g, ref, what):
    assert np.array_equal(g["nl"].astype(np.int32), ref.nl), f"{what}: lobe counts"
    K = ref.w.shape[1]
    gw, gS = g["w"].astype(np.float64), g["S"].astype(np.float64)
    ew = np.abs(gw - ref.w) / np.maximum(ref.w, 1e-2)
    tr = ref.S[:, :, :3].sum(-1)
    eS = np.abs(gS - ref.S).max(-1) / np.maximum(tr, 1e-2)
    valid = np.arange(K)[None, :] < ref.nl[:, None]
    assert np.all(gw[~valid] == 0) and np.all(gS[~valid] == 0), f"{what}: unused slots"
    rep = {"n": len(ref.nl), "reduced": int((ref.nl == K).sum()), "max_rel_w": float(ew.max(initial=0)),
           "max_rel_S": float(eS.max(initial=0))}
    assert rep["max_rel_w"] <= 1e-5 and rep["max_rel_S"] <= 1e-5, f"{what}: {rep}"
    return rep


def _stepwise(vx, grid, leaf_plan_leaf, lodp, K, N, what, levels=None):
    sh = vx.SggxhPlan(lodp, K=K, samples=N).run()
    lobes = sh.check()
    pyr = [lodp.leaf] + lodp.out
    keys = [p.numpy()["keys"].astype(np.uint64) for p in pyr]
    child = leaf_as_oracle_lobes(pyr[0].numpy())
    for L in range(1, len(pyr) if levels is None else levels):
        pk = keys[L]
        ck = keys[L - 1]
        cs = np.searchsorted(ck >> np.uint64(3), pk).astype(np.int64)
        cs = np.append(cs, len(ck))
        ref = oracle.sggxh_level(child, cs, pk, L, K, N)
        g = lobes[L - 1].numpy()
        say(what, "level", L, _compare(g, ref, f"{what} L{L}"))
        child = gpu_lobes_as_oracle(g)


@pytest.mark.parametrize("K", [2, 4])
def test_brushed_metal_window_stepwise(vx, K):
    import torch
    wl = synth.brushed_metal(window=64)
    say(f"case: SGGX-H, brushed metal 64^2 window, K = {K}, 500 samples")
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    lodp = vx.LodPlan(wl.grid, leaf, leaf.plan.stats[2:3], wl.levels).run()
    lodp.check()
    _stepwise(vx, wl.grid, leaf, lodp, K, 500, f"brushed64 K{K}")


def test_weave_small_stepwise_paper_samples(vx):
    """A small weave with the paper's 5000 samples per lobe, K = 4, levels 1-4."""
    import torch
    wl = synth.plain_weave(n_fibers=8, seed=5)
    say("case: SGGX-H, plain weave 8 fibers, K = 4, 5000 samples, levels 1-4")
    leaf = vx.voxelize_fibers(torch.as_tensor(wl.pts).cuda(), torch.as_tensor(wl.offsets).cuda(), wl.radius,
                              wl.grid)
    lodp = vx.LodPlan(wl.grid, leaf, leaf.plan.stats[2:3], 5).run()
    lodp.check()
    _stepwise(vx, wl.grid, leaf, lodp, 4, 5000, "weave8", levels=5)


@pytest.mark.parametrize("K", [1, 8])
def test_given_leaf_extreme_caps(vx, K):
    """Random fiber-like leaf lobes: K = 1 (everything merges) and K = 8 (64 lobes per voxel)."""
    import torch
    rng = np.random.default_rng(40 + K)
    log2_res = 4
    R = 16
    n = 2500
    coords = rng.choice(R ** 3, size=n, replace=False)
    keys = np.sort(np.array([oracle.morton(c % R, (c // R) % R, c // (R * R), log2_res) for c in coords],
                            dtype=np.uint64))
    w = rng.uniform(0.1, 2.0, n).astype(np.float32)
    t = rng.normal(size=(n, 3))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    M = np.stack([1 - t[:, 0] ** 2, 1 - t[:, 1] ** 2, 1 - t[:, 2] ** 2, -t[:, 0] * t[:, 1], -t[:, 0] * t[:, 2],
                  -t[:, 1] * t[:, 2]], 1)
    S = (w[:, None] * M).astype(np.float32)
    w[::97] = 0.0                               # a few empty voxels
    S[::97] = 0.0
    leaf = vx.alloc_voxels(n, log2_res, "cuda", False)
    leaf.keys.copy_(torch.as_tensor(keys.astype(np.uint32).view(np.int32)))
    leaf.count.copy_(torch.ones(n, dtype=torch.int32))
    leaf.w.copy_(torch.as_tensor(w))
    leaf.S.copy_(torch.as_tensor(np.ascontiguousarray(S.T)))
    leaf.n = n
    grid = synth.Grid((0.0, 0.0, 0.0), 16.0, log2_res)
    nd = torch.tensor([n], dtype=torch.int64, device="cuda")
    lodp = vx.LodPlan(grid, leaf, nd, 5).run()
    lodp.check()
    say(f"case: SGGX-H, given leaf 2500 voxels, 16^3, K = {K}, 300 samples")
    _stepwise(vx, grid, leaf, lodp, K, 300, f"given K{K}")


def test_errors(vx):
    import torch
    wl = synth.icosphere(subdiv=2)
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    lodp = vx.LodPlan(wl.grid, leaf, leaf.plan.stats[2:3], wl.levels).run()
    lodp.check()
    for K, N in ((0, 10), (9, 10), (4, 0), (4, 70000)):
        with pytest.raises(vx.VxError):
            vx.SggxhPlan(lodp, K=K, samples=N).run()


def test_brushed_metal_full_sampled_parents(vx):
    """The bench's configuration (the full 33.5 M-triangle surface, 13 levels, K = 4, 5000 samples
    per lobe): at every level, 200 sampled parents reduced again by the oracle from the GPU's own
    lobes of the level below."""
    import torch
    wl = synth.brushed_metal()
    say("case: SGGX-H, brushed metal full size, K = 4, 5000 samples, 200 sampled parents per level")
    leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    lodp = vx.LodPlan(wl.grid, leaf, leaf.plan.stats[2:3], wl.levels).run()
    lodp.check()
    lobes = vx.SggxhPlan(lodp, K=4, samples=5000).run().check()
    pyr = [lodp.leaf] + lodp.out
    rng = np.random.default_rng(21)
    child = leaf_as_oracle_lobes(pyr[0].numpy())
    ck = pyr[0].numpy()["keys"].astype(np.uint64)
    for L in range(1, len(pyr)):
        pk = pyr[L].numpy()["keys"].astype(np.uint64)
        g = lobes[L - 1].numpy()
        sel = np.sort(rng.choice(len(pk), size=min(200, len(pk)), replace=False))
        lo = np.searchsorted(ck >> np.uint64(3), pk[sel])
        hi = np.searchsorted(ck >> np.uint64(3), pk[sel], side="right")
        rows = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
        cs = np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.int64)
        sub = oracle.Lobes(child.nl[rows], child.w[rows], child.S[rows], np.zeros(len(rows)), np.zeros(len(rows)))
        ref = oracle.sggxh_level(sub, cs, pk[sel], L, 4, 5000)
        gs = {k: v[sel] for k, v in g.items()}
        say("level", L, _compare(gs, ref, f"full L{L}"))
        child = gpu_lobes_as_oracle(g)
        ck = pk
