"""GPU parity of the sampling voxelizer (Sec. 3.2-3.3) against its FP64 oracle, through the C ABI.

Keys and counts bit-exact (both sides place every sample with the same FP64 operations); w and
S per voxel within
    tol_i = 1e-5 + (n_i + 4) * 2^-24
of the oracle, relative to max(w, 1e-2) and max(tr S, 1e-2): the GPU rounds each sample's
weight and moment to FP32 (a few units in the last place) and sums the voxel's n_i samples in
FP32 in sample order, whose rounding error is at most (n_i - 1) * 2^-24 of the sum of the terms'
magnitudes (the standard bound for recursive summation); the oracle sums in FP64.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def compare_samples(g, ref, what):
    gk = g["keys"].astype(np.uint64)
    assert len(gk) == len(ref.keys), f"{what}: {len(gk)} voxels vs oracle {len(ref.keys)}"
    if not np.array_equal(gk, ref.keys):
        bad = np.flatnonzero(gk != ref.keys)[:5]
        raise AssertionError(f"{what}: keys differ at {bad.tolist()}: {gk[bad]} vs {ref.keys[bad]}")
    n = ref.count.astype(np.float64)
    assert np.array_equal(g["count"].astype(np.uint64), ref.count.astype(np.uint64)), f"{what}: counts"
    tol = 1e-5 + (n + 4) * 2.0 ** -24
    ew = np.abs(g["w"].astype(np.float64) - ref.w) / np.maximum(ref.w, 1e-2)
    tr = ref.S[:, 0] + ref.S[:, 1] + ref.S[:, 2]
    eS = np.abs(g["S"].astype(np.float64) - ref.S).max(axis=1) / np.maximum(tr, 1e-2) if len(tr) else ew
    rep = {"n": len(gk), "max_count": int(n.max(initial=0)), "max_w_err/tol": float((ew / tol).max(initial=0)),
           "max_S_err/tol": float((eS / tol).max(initial=0))}
    assert rep["max_w_err/tol"] <= 1 and rep["max_S_err/tol"] <= 1, f"{what}: {rep}"
    return rep


def _fibers(vx, wl, chords, per, **kw):
    p = vx.SamplePlan(1, wl.grid, _dev(wl.pts), offsets=_dev(wl.offsets), chords=chords, per_chord=per, **kw)
    p.run()
    v = p.check()
    return p, v.numpy()


def _tris(vx, grid, tris, N, **kw):
    p = vx.SamplePlan(0, grid, _dev(tris), N=N, **kw)
    p.run()
    v = p.check()
    return p, v.numpy()


@pytest.mark.parametrize("log2_res,chords,per", [(5, 4, 3), (12, 7, 5)])
def test_random_fibers(vx, log2_res, chords, per):
    """Random walks leaving the grid on every side (samples outside dropped); 32- and 64-bit keys."""
    R = 1 << log2_res
    wl = synth.random_fibers(12, 40, log2_res, seed=log2_res, step=max(1.0, R / 64), margin=3.0 * R / 32)
    say(f"case: sampled random fibers 12 x 40 points, R = {R}, {chords} chords x {per}")
    p, g = _fibers(vx, wl, chords, per)
    ref = oracle.sample_fibers(wl.grid, wl.pts, wl.offsets, chords, per)
    assert p.n_samples == 12 * 39 * chords * per and p.n_inside == ref.n_pairs < p.n_samples
    say(compare_samples(g, ref, "random fibers"))


@pytest.mark.parametrize("N", [1, 7, 64])
def test_random_triangles(vx, N):
    """Triangles of mixed sizes, some leaving the grid and one degenerate (one sample, zero weight)."""
    wl = synth.random_triangles(300, 6, seed=11, scale=4.0, margin=2.0)
    tris = wl.tris.copy()
    tris[17, 2] = tris[17, 0]                                 # a zero-area triangle
    say(f"case: sampled random triangles 300, 64^3, N = {N}")
    p, g = _tris(vx, wl.grid, tris, N)
    ref = oracle.sample_triangles(wl.grid, tris, N)
    assert p.n_inside == ref.n_pairs
    say(compare_samples(g, ref, f"random triangles N={N}"))


def test_plain_weave_small(vx):
    wl = synth.plain_weave(n_fibers=96, seed=5)
    say("case: sampled plain weave 96 fibers x 256 segments, 1024^3, 6 chords x 4")
    p, g = _fibers(vx, wl, 6, 4)
    ref = oracle.sample_fibers(wl.grid, wl.pts, wl.offsets, 6, 4)
    say(compare_samples(g, ref, "weave96"))


def test_brushed_metal_window(vx):
    wl = synth.brushed_metal(window=384)
    say("case: sampled brushed metal 384^2 window, 4096^3, N = 16")
    p, g = _tris(vx, wl.grid, wl.tris, 16)
    ref = oracle.sample_triangles(wl.grid, wl.tris, 16)
    say(compare_samples(g, ref, "brushed window"))


def test_brushed_metal_full_sampled_regions(vx):
    """The full surface (33.5 M triangles, N = 16): the GPU result inside sampled 24^2 columns
    against the oracle over the triangles that reach them (plus the largest triangles, which fix
    the sample counts), and the total weight against the total area."""
    wl = synth.brushed_metal()
    say("case: sampled brushed metal full size, N = 16, sampled regions")
    p, g = _tris(vx, wl.grid, wl.tris, 16)
    t = wl.tris.astype(np.float64)
    c = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    q = (c * c).sum(1)
    top = np.argsort(q)[-8:]
    assert abs(g["w"].astype(np.float64).sum() - 0.5 * np.sqrt(q).sum()) <= 1e-5 * 0.5 * np.sqrt(q).sum()
    coords = oracle.demorton(g["keys"].astype(np.uint64), wl.grid.log2_res)
    lo_t = t.min(1)
    hi_t = t.max(1)
    rng = np.random.default_rng(9)
    for x0, y0 in rng.integers(0, 4096 - 24, size=(3, 2)):
        sel = np.flatnonzero((hi_t[:, 0] >= x0) & (lo_t[:, 0] <= x0 + 24) & (hi_t[:, 1] >= y0) &
                             (lo_t[:, 1] <= y0 + 24))
        sub = np.union1d(sel, top)
        ref = oracle.sample_triangles(wl.grid, wl.tris[sub], 16)
        rc = oracle.demorton(ref.keys, wl.grid.log2_res)
        inr = lambda cc: (cc[:, 0] >= x0) & (cc[:, 0] < x0 + 24) & (cc[:, 1] >= y0) & (cc[:, 1] < y0 + 24)
        mg, mr = inr(coords), inr(rc)
        gg = {k: v[mg] for k, v in g.items()}
        r = oracle.Voxels(ref.keys[mr], ref.count[mr], ref.w[mr], ref.S[mr], int(ref.count[mr].sum()))
        say(compare_samples(gg, r, f"region ({x0}, {y0})"))


def test_edge_cases(vx):
    """Empty input; fibers of one point and empty fibers between others; everything outside."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    p, g = _tris(vx, grid, np.zeros((0, 3, 3), np.float32), 8)
    assert p.out.n == 0 and p.n_samples == 0
    pts = np.array([[1.2, 1.3, 1.4], [2.5, 2.2, 1.9], [3.1, 3.7, 2.2], [4.4, 4.1, 3.3], [5.0, 5.5, 4.0],
                    [6.1, 6.2, 6.3]], np.float32)
    offs = np.array([0, 0, 1, 4, 4, 6], np.int64)            # empty, one point, three, empty, two
    wl = synth.FiberWorkload("edge", grid, pts, offs, 0.0, 4, 1)
    p, g = _fibers(vx, wl, 3, 2)
    ref = oracle.sample_fibers(grid, pts, offs, 3, 2)
    assert p.n_samples == 3 * 3 * 2
    compare_samples(g, ref, "edge fibers")
    far = np.array([[[20.0, 20.0, 20.0], [21.0, 20.0, 20.0], [20.0, 21.0, 20.0]]], np.float32)
    p, g = _tris(vx, grid, far, 4)
    assert p.out.n == 0 and p.n_inside == 0 and p.n_samples == 4


def test_errors(vx):
    import torch
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    tris = np.array([[[1.0, 1.0, 1.0], [5.0, 1.5, 2.0], [2.0, 6.0, 3.0]]], np.float32)
    with pytest.raises(vx.VxError):                                   # too few samples allowed
        p = vx.SamplePlan(0, grid, _dev(tris), N=16, max_samples=15, out_cap=64)
        p.run()
        p.check()
    with pytest.raises(vx.VxError):                                   # too few voxels allowed
        p = vx.SamplePlan(0, grid, _dev(tris), N=16, max_samples=16, out_cap=1)
        p.run()
        p.check()
    bad = tris.copy()
    bad[0, 1, 2] = np.nan
    with pytest.raises(vx.VxError):
        vx.SamplePlan(0, grid, _dev(bad), N=4)
    pts = np.array([[1.0, 1.0, 1.0], [2.0, 2.0, 2.0], [3.0, 3.0, 3.0]], np.float32)
    with pytest.raises(vx.VxError):                                   # offsets not ending at n_pts
        vx.SamplePlan(1, grid, _dev(pts), offsets=torch.tensor([0, 2]), chords=2, per_chord=2)
    with pytest.raises(vx.VxError):                                   # decreasing offsets
        vx.SamplePlan(1, grid, _dev(pts), offsets=torch.tensor([0, 2, 1, 3]), chords=2, per_chord=2)
    with pytest.raises(vx.VxError):                                   # N out of range (host check)
        vx.SamplePlan(0, grid, _dev(tris), N=0)
