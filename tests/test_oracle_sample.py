"""Pins of the sampling-voxelizer oracle (Sec. 3.2): Heitz's triangle map by its definition and
its uniformity, the area-proportional sample counts in exact rationals, a hand-worked fiber, the
conservation of length and area, the single-direction moments, and convergence of the sampled
weights to the exact clipped measures of the exact oracle as the sample count grows."""
from fractions import Fraction

import numpy as np

import oracle
import synth


def test_heitz_map_corners_and_uniformity():
    assert np.allclose(oracle.heitz_map(0.2, 0.6), [0.1, 0.5])      # u2 > u1: b0 = u1 / 2, b1 = u2 - b0
    assert np.allclose(oracle.heitz_map(0.6, 0.2), [0.5, 0.1])      # else: b1 = u2 / 2, b0 = u1 - b1
    assert np.allclose(oracle.heitz_map(1.0, 0.0), [1.0, 0.0])      # vertex 0
    assert np.allclose(oracle.heitz_map(0.0, 1.0), [0.0, 1.0])      # vertex 1
    assert np.allclose(oracle.heitz_map(0.0, 0.0), [0.0, 0.0])      # vertex 2
    # area-preserving: a uniform grid over the square lands uniformly in the triangle (the four
    # corner sub-triangles of the midpoint subdivision get a quarter each)
    n = 200
    u = (np.arange(n) + 0.5) / n
    b = np.array([oracle.heitz_map(a, c) for a in u for c in u])
    assert (b >= 0).all() and (b.sum(1) <= 1 + 1e-12).all()
    b2 = 1 - b.sum(1)
    quarters = [(b[:, 0] > 0.5).mean(), (b[:, 1] > 0.5).mean(), (b2 > 0.5).mean()]
    assert np.allclose(quarters, 0.25, atol=0.01), quarters


def test_sample_counts_in_exact_rationals():
    rng = np.random.default_rng(3)
    for _ in range(300):
        qmax = float(rng.uniform(0.1, 10.0))
        q = float(rng.uniform(0, qmax))
        N = int(rng.integers(1, 70))
        # floor(N sqrt(q / qmax)) = the largest k with k^2 qmax <= N^2 q (on the FP64 products)
        qq, qm = Fraction(q), Fraction(qmax)
        k = 0
        while Fraction((k + 1) ** 2) * qm <= Fraction(N * N) * qq:
            k += 1
        assert oracle.tri_sample_count(q, qmax, N) == max(1, k)
    assert oracle.tri_sample_count(4.0, 4.0, 16) == 16                  # the largest triangle
    assert oracle.tri_sample_count(1.0, 4.0, 16) == 8                   # a quarter of the area
    assert oracle.tri_sample_count(0.0, 4.0, 16) == 1                   # never fewer than one


def test_fiber_by_hand():
    """One straight segment from x = 0.25 to 1.75 (grid [0, 2]^3, R = 2), one chord, two
    samples at fractions 1/4 and 3/4: x = 0.625 (voxel 0) and 1.375 (voxel 1), 0.75 each."""
    grid = synth.Grid((0.0, 0.0, 0.0), 2.0, 1)
    pts = np.array([[0.25, 0.5, 0.5], [1.75, 0.5, 0.5]], np.float32)
    v = oracle.sample_fibers(grid, pts, [0, 2], 1, 2)
    assert [tuple(c) for c in oracle.demorton(v.keys, 1)] == [(0, 0, 0), (1, 0, 0)]
    assert list(v.count) == [1, 1] and np.allclose(v.w, [0.75, 0.75], atol=1e-15)
    assert np.allclose(v.S / v.w[:, None], [[0, 1, 1, 0, 0, 0]] * 2, atol=1e-15)   # I - x x^T
    assert v.n_pairs == 2


def test_conservation_and_moments():
    wl = synth.random_fibers(6, 9, 5, seed=7, step=1.5, inset=12.0)
    v = oracle.sample_fibers(wl.grid, wl.pts, wl.offsets, 4, 3)
    assert v.n_pairs == 6 * 8 * 4 * 3                                     # every sample inside the grid
    # total weight = total chord length of the subdivided spans (the chords re-measured here)
    g = (wl.pts.astype(np.float64) - np.asarray(wl.grid.bmin)) * (wl.grid.res / wl.grid.extent)
    total = 0.0
    for f in range(len(wl.offsets) - 1):
        a, b = wl.offsets[f], wl.offsets[f + 1]
        for i in range(a, b - 1):
            P = [g[max(i - 1, a)], g[i], g[i + 1], g[min(i + 2, b - 1)]]
            c0 = P[1]
            c1 = 0.5 * (P[2] - P[0])
            c2 = ((P[0] - 2.5 * P[1]) + 2.0 * P[2]) - 0.5 * P[3]
            c3 = 0.5 * (P[3] - P[0]) + 1.5 * (P[1] - P[2])
            C = [((c3 * t + c2) * t + c1) * t + c0 for t in np.arange(5) / 4.0]
            total += sum(np.linalg.norm(C[j + 1] - C[j]) for j in range(4))
    assert abs(v.w.sum() - total) <= 1e-9 * total
    assert np.allclose(v.S[:, :3].sum(1), 2 * v.w, rtol=1e-12)            # tr S = 2 w for fibers
    tw = synth.random_triangles(40, 4, seed=8, scale=3.0)
    tw.tris[:] = np.clip(tw.tris, 0.5 / 16, 15.5 / 16)                     # every sample inside the grid
    t = oracle.sample_triangles(tw.grid, tw.tris, 32)
    gt = (tw.tris.astype(np.float64) - np.asarray(tw.grid.bmin)) * (tw.grid.res / tw.grid.extent)
    area = 0.5 * np.linalg.norm(np.cross(gt[:, 1] - gt[:, 0], gt[:, 2] - gt[:, 0]), axis=1).sum()
    assert abs(t.w.sum() - area) <= 1e-9 * area
    assert np.allclose(t.S[:, :3].sum(1), t.w, rtol=1e-12)                 # tr S = w for surfaces


def _dense_w(v, bits):
    out = {}
    for k, w in zip(v.keys, v.w):
        out[int(k)] = w
    return out


def test_weights_converge_to_the_exact_measures():
    """Sampled weights approach the exact clipped measures of the exact oracle: fibers (straight,
    equally spaced control points: the Catmull-Rom spans are the straight segments) and
    triangles, the error falling as the sample count grows."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    d = np.array([0.83, 0.41, 0.37])
    pts = (np.array([1.13, 2.07, 1.61]) + np.arange(7)[:, None] * d).astype(np.float32)
    exact = _dense_w(oracle.voxelize_fibers(grid, pts, [0, 7], 0.0), 3)
    errs = []
    for per in (2, 16, 128, 1024):
        s = _dense_w(oracle.sample_fibers(grid, pts, [0, 7], 1, per), 3)
        errs.append(max(abs(s.get(k, 0.0) - exact[k]) for k in exact))
    assert errs[-1] < 2e-3 and errs[-1] < errs[1] < errs[0], errs
    tris = np.array([[[0.3, 0.4, 0.5], [6.7, 1.2, 2.9], [2.2, 7.1, 5.3]],
                     [[1.1, 6.6, 0.4], [5.9, 6.1, 7.2], [3.3, 0.7, 3.8]]], np.float32)
    exact = _dense_w(oracle.voxelize_triangles(grid, tris), 3)
    tot = sum(exact.values())
    errs = []
    for N in (16, 256, 4096):
        s = _dense_w(oracle.sample_triangles(grid, tris, N), 3)
        errs.append(sum(abs(s.get(k, 0.0) - exact[k]) for k in exact) / tot)
    assert errs[-1] < 0.05 and errs[-1] < errs[1] < errs[0], errs
