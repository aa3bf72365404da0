"""The allocation-free pyramid entry point, vx_build_lod_noalloc, against vx_build_lod (the same
kernels with a caller workspace): two calls in a row on one GPU, the second with a smaller leaf
(so the library's scratch array still holds the first call's contents), each compared bit for
bit with the workspace entry point on every level and lobe; and the capacity limit reported as
an error before any launch."""
import sys

import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _leaf(vx, wl, kind):
    import torch
    if kind == 1:
        leaf = vx.voxelize_fibers(torch.as_tensor(wl.pts).cuda(), torch.as_tensor(wl.offsets).cuda(), wl.radius,
                                  wl.grid)
    else:
        leaf = vx.voxelize_triangles(torch.as_tensor(wl.tris).cuda(), wl.grid)
    return leaf


def _same(a, b, n):
    import torch
    return torch.equal(a[..., :n], b[..., :n])


def _compare(ref, na):
    assert ref.n_levels.cpu().tolist() == na.n_levels.cpu().tolist()
    for L, (r, g) in enumerate(zip(ref.out, na.out), start=1):
        n = r.n
        assert g.n == n, L
        for name in ("keys", "count", "w", "S", "mask"):
            assert _same(getattr(r, name), getattr(g, name), n), (L, name)
    for L, (r, g) in enumerate(zip(ref.lobes, na.lobes), start=1):
        n = ref.out[L - 1].n
        for name in ("nl", "w", "S"):
            assert _same(getattr(r, name), getattr(g, name), n), (L, "lobes", name)


@pytest.mark.parametrize("K", [1, 4])
def test_noalloc_equals_workspace_entry_point_twice(vx, K):
    cases = [("plain weave, 300 fibers", synth.plain_weave(n_fibers=300, seed=21), 1),
             ("brushed metal, 40x40 window (64-bit keys)", synth.brushed_metal(window=40), 0)]
    sizes = []
    for what, wl, kind in cases:
        say("case: build_lod_noalloc vs build_lod,", what, "K =", K)
        leaf = _leaf(vx, wl, kind)
        sizes.append(leaf.n)
        n_dev = leaf.plan.stats[2:3]
        ref = vx.LodPlan(wl.grid, leaf, n_dev, wl.levels, K=K, iters=2).run()
        ref.check()
        na = vx.LodPlan(wl.grid, leaf, n_dev, wl.levels, K=K, iters=2, noalloc=True).run()
        na.check()
        assert na.ws is None
        _compare(ref, na)
        say("  levels", ref.n_levels.cpu().tolist()[:-1], "identical")
    assert sizes[1] < sizes[0]                       # the second call is the smaller one


def test_noalloc_capacity_limit(vx):
    import torch
    say("case: build_lod_noalloc with a leaf capacity above the limit")
    grid = synth.Grid((0.0, 0.0, 0.0), 1.0, 6)
    leaf = vx.alloc_voxels(vx.NOALLOC_MAX_LEAF + 1, grid.log2_res, "cuda", False)
    leaf.n = 0
    n_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan = vx.LodPlan(grid, leaf, n_dev, 3, K=1, caps=[16, 16], noalloc=True)
    with pytest.raises(vx.VxError) as e:
        plan.run()
    assert e.value.status == 2
    torch.cuda.synchronize()
