"""Pins for the FP64 oracle: it is checked against things other than itself.

* exact-rational brute force with different methods (oracle/brute.py) on tiny grids, with
  adversarial inputs built on the lattice so that touching cases are exact ties;
* closed forms (axis-aligned fiber, flat triangle in a voxel face plane);
* conservation laws and SGGX properties on the icosphere and on random fibers;
* the pyramid against direct grouped sums of the leaf;
* the lobe distance against quadrature, Ward against a from-scratch SSE greedy, Lloyd's
  objective, and the special cases of the clustering.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def G(log2_res, extent=None):
    return synth.Grid((0.0, 0.0, 0.0), float(extent if extent is not None else (1 << log2_res)), log2_res)


# ------------------------------------------------------------------------------------------------
# Sec. 3.1 transform and Morton keys
# ------------------------------------------------------------------------------------------------

def test_snap_matches_independent_lattice():
    rng = np.random.default_rng(10)
    grid = synth.Grid((-1.5, 0.25, 3.0), 4.0, 2)
    # anywhere inside the accepted margin of one grid on every side
    p = (np.asarray(grid.bmin) + rng.uniform(-3.99, 7.99, size=(4000, 3))).astype(np.float32)
    # points exactly half-way between two lattice values (round half to even decides them)
    k = rng.integers(0, 1 << 20, size=(1000, 3))
    half = ((2 * k + 1) * 2.0 ** -22).astype(np.float32) + np.float32(0.0)
    grid0 = G(2, 4.0)
    assert np.array_equal(oracle.snap(grid0, half), brute.lattice(grid0, half))
    assert np.array_equal(oracle.snap(grid, p), brute.lattice(grid, p))


def test_snap_rejects_bad_input():
    grid = G(2, 4.0)
    with pytest.raises(oracle.OracleError):
        oracle.snap(grid, np.array([[0.0, np.nan, 0.0]]))
    with pytest.raises(oracle.OracleError):
        oracle.snap(grid, np.array([[0.0, 8.01, 0.0]]))      # more than one grid beyond the bounds
    with pytest.raises(oracle.OracleError):
        oracle.snap(grid, np.array([[-4.01, 0.0, 0.0]]))
    oracle.snap(grid, np.array([[-4.0, 8.0, 0.0]]))           # the margin itself is accepted


def test_morton_roundtrip_and_parent():
    rng = np.random.default_rng(11)
    bits = 10
    c = rng.integers(0, 1 << bits, size=(200, 3))
    keys = np.array([oracle.morton(x, y, z, bits) for x, y, z in c], dtype=np.uint64)
    assert np.array_equal(oracle.demorton(keys, bits), c)
    assert np.array_equal(oracle.demorton(keys >> np.uint64(3), bits - 1), c >> 1)
    # the bit layout itself: x at bit 3b, y at 3b+1, z at 3b+2
    assert oracle.morton(1, 0, 0, 4) == 1 and oracle.morton(0, 1, 0, 4) == 2 and oracle.morton(0, 0, 1, 4) == 4
    assert oracle.morton(2, 0, 0, 4) == 8 and oracle.morton(0, 0, 8, 4) == 1 << 11


# ------------------------------------------------------------------------------------------------
# predicates and measures vs brute force
# ------------------------------------------------------------------------------------------------

def _adversarial_triangles(rng, n, R):
    """Vertices on a half-voxel lattice (ties with faces, edges, corners), plus flat, collinear,
    point-like and partly-outside triangles."""
    out = []
    for i in range(n):
        kind = i % 6
        if kind == 0:
            t = rng.integers(-1, 2 * R + 2, size=(3, 3)) / 2.0
        elif kind == 1:                          # flat on a voxel face plane
            t = rng.integers(0, 2 * R + 1, size=(3, 3)) / 2.0
            t[:, i % 3] = rng.integers(0, R + 1)
        elif kind == 2:                          # collinear
            a = rng.integers(0, 2 * R, size=3) / 2.0
            d = rng.integers(-2, 3, size=3) / 2.0
            t = np.stack([a, a + d, a + 2 * d])
        elif kind == 3:                          # a point
            t = np.repeat(rng.integers(0, 2 * R + 1, size=(1, 3)) / 2.0, 3, axis=0)
        elif kind == 4:                          # generic, small
            c = rng.uniform(0, R, size=(1, 3))
            t = c + rng.normal(0, 0.7, size=(3, 3))
        else:                                    # partly outside the grid
            t = rng.uniform(-0.5 * R, 1.5 * R, size=(3, 3))
        out.append(t)
    return np.array(out, dtype=np.float32)


def test_triangle_predicates_vs_brute():
    rng = np.random.default_rng(12)
    R, grid = 4, G(2)
    s = brute.voxel_size(grid)
    tris = _adversarial_triangles(rng, 60, R)
    q = brute.lattice(grid, tris.reshape(-1, 3)).reshape(-1, 3, 3)
    L = oracle.lib()
    n_touch = 0
    for t in q:
        qa = np.ascontiguousarray(t, dtype=np.int64)
        for x in range(-1, R + 1):
            for y in range(-1, R + 1):
                for z in range(-1, R + 1):
                    lo = np.array([x * s, y * s, z * s], dtype=np.int64)
                    tb = brute.tri_touch(t, lo, s)
                    to = bool(L.vxo_tri_touch(oracle._ptr(qa), oracle._ptr(lo), s))
                    assert tb == to, (t.tolist(), lo.tolist())
                    n_touch += tb
                    if tb:
                        ab = brute.tri_area(t, lo, s)
                        ao = L.vxo_tri_area(oracle._ptr(qa), oracle._ptr(lo), s)
                        assert abs(ab - ao) <= 1e-12 * max(1.0, ab), (t.tolist(), lo.tolist(), ab, ao)
    assert n_touch > 300


def _adversarial_segments(rng, n, R, s):
    """Segments and radii with exact distance ties: axis-parallel segments at distance exactly
    rho from a face, an edge (3-4-5 offsets) or a corner (1-2-2 offsets); degenerate segments;
    random segments.  Coordinates in lattice units."""
    out = []
    u = s // 8
    for i in range(n):
        kind = i % 6
        base = rng.integers(0, R, size=3) * s
        if kind == 0:                            # parallel to x at distance rho = s/2 of a face
            a = base + np.array([rng.integers(-s, s), s // 2 * 3, s // 2])
            b = a + np.array([rng.integers(1, 3 * s), 0, 0])
            rho = s // 2
        elif kind == 1:                          # parallel to z, 3-4-5 distance from a vertical edge
            a = base + np.array([-3 * u, -4 * u, rng.integers(-s, s)])
            b = a + np.array([0, 0, rng.integers(0, 2 * s)])
            rho = 5 * u
        elif kind == 2:                          # a point at 1-2-2 distance from a corner
            a = base + np.array([-u, -2 * u, -2 * u])
            b = a.copy()
            rho = 3 * u - (i % 12 == 2)          # once at the tie, once just short of it
        elif kind == 3:                          # zero radius, on the lattice of half voxels
            a = rng.integers(0, 2 * R + 1, size=3) * (s // 2)
            b = rng.integers(0, 2 * R + 1, size=3) * (s // 2)
            rho = 0
        elif kind == 4:                          # generic
            a = rng.integers(0, R * s, size=3)
            b = a + rng.integers(-2 * s, 2 * s, size=3)
            rho = int(rng.integers(0, s))
        else:                                    # oblique through an edge neighbourhood
            a = base + np.array([-s, -u, s // 2])
            b = base + np.array([2 * s, -u + rng.integers(-1, 2), s // 2])
            rho = u
        out.append((np.asarray(a, np.int64), np.asarray(b, np.int64), int(rho)))
    return out


def test_capsule_predicates_vs_brute():
    rng = np.random.default_rng(13)
    R, grid = 4, G(2)
    s = brute.voxel_size(grid)
    L = oracle.lib()
    n_touch = 0
    for a, b, rho in _adversarial_segments(rng, 60, R, s):
        a = np.ascontiguousarray(a)
        b = np.ascontiguousarray(b)
        for x in range(-1, R + 1):
            for y in range(-1, R + 1):
                for z in range(-1, R + 1):
                    lo = np.array([x * s, y * s, z * s], dtype=np.int64)
                    tb = brute.cap_touch(a, b, lo, s, rho)
                    to = bool(L.vxo_cap_touch(oracle._ptr(a), oracle._ptr(b), oracle._ptr(lo), s, rho))
                    assert tb == to, (a.tolist(), b.tolist(), lo.tolist(), rho)
                    n_touch += tb
                    lb = brute.seg_length(a, b, lo, s)
                    lo_ = L.vxo_seg_length(oracle._ptr(a), oracle._ptr(b), oracle._ptr(lo), s)
                    assert abs(lb - lo_) <= 1e-12 * max(1.0, lb)
    assert n_touch > 200


@pytest.mark.parametrize("seed", [20, 21])
def test_voxelize_triangles_vs_brute(seed):
    rng = np.random.default_rng(seed)
    grid = G(2, 4.0) if seed == 20 else G(3, 2.0)
    tris = _adversarial_triangles(rng, 12, grid.res) * np.float32(grid.extent / grid.res)
    o = oracle.voxelize_triangles(grid, tris)
    bk, bc, bw, bS = brute.voxelize_triangles(grid, tris)
    assert np.array_equal(o.keys, bk) and np.array_equal(o.count, bc)
    assert np.abs(o.w - bw).max() <= 1e-11 and np.abs(o.S - bS).max() <= 1e-11
    assert o.n_pairs == int(bc.sum())


@pytest.mark.parametrize("seed", [30, 31])
def test_voxelize_fibers_vs_brute(seed):
    f = synth.random_fibers(3, 4, 2 if seed == 30 else 3, seed=seed, step=1.2, radius=0.5 if seed == 30 else 0.75,
                            margin=0.5)
    o = oracle.voxelize_fibers(f.grid, f.pts, f.offsets, f.radius)
    bk, bc, bw, bS = brute.voxelize_fibers(f.grid, f.pts, f.offsets, f.radius)
    assert np.array_equal(o.keys, bk) and np.array_equal(o.count, bc)
    assert np.abs(o.w - bw).max() <= 1e-11 and np.abs(o.S - bS).max() <= 1e-11


# ------------------------------------------------------------------------------------------------
# closed forms
# ------------------------------------------------------------------------------------------------

def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_axis_aligned_fiber_closed_form():
    g = _load("axis_fiber.json")
    grid = G(g["log2_res"])
    pts = np.array(g["points"], dtype=np.float32)
    o = oracle.voxelize_fibers(grid, pts, np.array([0, len(pts)]), g["radius"])
    got = {tuple(c): (int(n), float(w)) for c, n, w in zip(oracle.demorton(o.keys, grid.log2_res).tolist(),
                                                           o.count, o.w)}
    want = {tuple(v["voxel"]): (v["count"], v["w"]) for v in g["voxels"]}
    assert set(got) == set(want)
    for k in want:
        assert got[k][0] == want[k][0] and abs(got[k][1] - want[k][1]) < 1e-12, k
    # a single direction t = x: the normalised SGGX is I - t t^T = diag(0, 1, 1)
    m = o.w > 0
    Sb = o.S[m] / o.w[m, None]
    assert np.allclose(Sb, [0, 1, 1, 0, 0, 0], atol=1e-15)
    assert o.S[~m].max() == 0.0


def test_flat_triangle_ownership():
    g = _load("flat_triangle.json")
    grid = G(g["log2_res"])
    tri = np.array([g["triangle"]], dtype=np.float32)
    o = oracle.voxelize_triangles(grid, tri)
    c = oracle.demorton(o.keys, grid.log2_res)
    assert sorted(set(c[:, 2].tolist())) == g["touched_layers"]
    assert np.all(o.w[c[:, 2] != g["owner_layer"]] == 0)
    assert abs(o.w.sum() - g["area"]) < 1e-12
    m = o.w > 0
    assert np.allclose(o.S[m] / o.w[m, None], [0, 0, 1, 0, 0, 0], atol=1e-15)


# ------------------------------------------------------------------------------------------------
# conservation and SGGX properties
# ------------------------------------------------------------------------------------------------

def _psd_sym(S, w, scale):
    M = np.zeros((len(S), 3, 3))
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for c, (i, j) in enumerate(idx):
        M[:, i, j] = S[:, c]
        M[:, j, i] = S[:, c]
    ev = np.linalg.eigvalsh(M)
    assert ev.min() >= -1e-12 * max(1.0, scale)


def test_icosphere_conservation():
    wl = synth.icosphere()
    o = oracle.voxelize_triangles(wl.grid, wl.tris)
    q = brute.lattice(wl.grid, wl.tris.reshape(-1, 3)).reshape(-1, 3, 3).astype(np.float64)
    s = float(brute.voxel_size(wl.grid))
    n = np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0]) / s ** 2
    area = 0.5 * np.linalg.norm(n, axis=1)
    nn = n / np.linalg.norm(n, axis=1, keepdims=True)
    M = np.stack([nn[:, 0] ** 2, nn[:, 1] ** 2, nn[:, 2] ** 2, nn[:, 0] * nn[:, 1], nn[:, 0] * nn[:, 2],
                  nn[:, 1] * nn[:, 2]], 1)
    assert abs(o.w.sum() - area.sum()) <= 1e-9 * area.sum()
    assert np.abs(o.S.sum(0) - (area[:, None] * M).sum(0)).max() <= 1e-9 * area.sum()
    assert np.abs(o.S[:, :3].sum(1) - o.w).max() <= 1e-12 * o.w.max()      # tr S = w for surfaces
    _psd_sym(o.S, o.w, o.w.max())
    # a sphere's normals are spread evenly: the root SGGX is close to (A / 3) I
    assert np.allclose(o.S.sum(0)[:3], area.sum() / 3, rtol=2e-3)
    assert 4 * 20480 < o.n_pairs < 5 * 20480


def test_fiber_conservation():
    f = synth.random_fibers(40, 30, 6, seed=40, step=1.3, radius=0.5, inset=20.0)
    o = oracle.voxelize_fibers(f.grid, f.pts, f.offsets, f.radius)
    q = brute.lattice(f.grid, f.pts).astype(np.float64).reshape(40, 30, 3)
    assert q.min() > 0 and q.max() < (1 << 23)                              # no clamping happened
    s = float(brute.voxel_size(f.grid))
    d = (q[:, 1:] - q[:, :-1]).reshape(-1, 3) / s
    ln = np.linalg.norm(d, axis=1)
    # all points stay inside the grid, so every bit of length is owned by some voxel
    assert abs(o.w.sum() - ln.sum()) <= 1e-9 * ln.sum()
    t = d / ln[:, None]
    M = np.stack([1 - t[:, 0] ** 2, 1 - t[:, 1] ** 2, 1 - t[:, 2] ** 2, -t[:, 0] * t[:, 1], -t[:, 0] * t[:, 2],
                  -t[:, 1] * t[:, 2]], 1)
    assert np.abs(o.S.sum(0) - (ln[:, None] * M).sum(0)).max() <= 1e-9 * ln.sum()
    assert np.abs(o.S[:, :3].sum(1) - 2 * o.w).max() <= 1e-12 * o.w.max()   # tr S = 2 w for fibers
    _psd_sym(o.S, o.w, o.w.max())


def test_pyramid_against_grouped_leaf_sums():
    wl = synth.icosphere()
    o = oracle.voxelize_triangles(wl.grid, wl.tris)
    lod = oracle.build_lod(o, wl.levels)
    assert len(lod[-1].keys) == 1 and lod[-1].keys[0] == 0
    coords = oracle.demorton(o.keys, wl.grid.log2_res)
    for L in range(1, wl.levels):
        g = o.keys >> np.uint64(3 * L)
        uk, inv = np.unique(g, return_inverse=True)
        assert np.array_equal(uk, lod[L].keys)
        S = np.zeros((len(uk), 6))
        np.add.at(S, inv, o.S)
        assert np.abs(S - lod[L].S).max() <= 1e-12 * max(1.0, np.abs(S).max())
        cnt = np.zeros(len(uk), np.int64)
        np.add.at(cnt, inv, o.count.astype(np.int64))
        assert np.array_equal(cnt, lod[L].count.astype(np.int64))
        # child mask: which octants of the parent hold data one level down
        child = (coords >> (L - 1)) & 1
        octant = child[:, 0] | child[:, 1] << 1 | child[:, 2] << 2
        mask = np.zeros(len(uk), np.int64)
        np.bitwise_or.at(mask, inv, (1 << octant).astype(np.int64))
        assert np.array_equal(mask.astype(np.uint8), lod[L].mask)
    # the parent's normalised SGGX is the weight-averaged child SGGX
    p = lod[1]
    for i in range(0, len(p.keys), 97):
        a, b = p.child_start[i], p.child_start[i + 1]
        avg = (lod[0].w[a:b, None] * (lod[0].S[a:b] / lod[0].w[a:b, None])).sum(0) / lod[0].w[a:b].sum()
        assert np.allclose(p.S[i] / p.w[i], avg, atol=1e-12)


# ------------------------------------------------------------------------------------------------
# Sec. 4.4 lobe merging
# ------------------------------------------------------------------------------------------------

def _fib_dirs(n):
    k = np.arange(n)
    z = 1 - (2 * k + 1) / n
    phi = k * math.pi * (3 - math.sqrt(5))
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def _mat(v):
    return np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])


def test_lobe_distance_is_quadrature_of_projected_area_squared():
    rng = np.random.default_rng(50)
    W = _fib_dirs(20000)
    for _ in range(5):
        A, B = rng.normal(size=6), rng.normal(size=6)
        D = _mat(A - B)
        quad = 15.0 * np.mean(np.einsum("ni,ij,nj->n", W, D, W) ** 2)   # (15 / 4 pi) * integral
        assert abs(oracle.lobe_dist(A, B) - quad) <= 1e-4 * quad


def _random_lobes(rng, n):
    w = rng.uniform(0.2, 2.0, n)
    S = []
    for i in range(n):
        t = rng.normal(size=3)
        t /= np.linalg.norm(t)
        M = np.eye(3) - np.outer(t, t)
        S.append(w[i] * np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]]))
    return w, np.array(S)


def _one_parent(w, S, K, iters):
    n = len(w)
    child = oracle.Lobes(np.ones(n, np.int32), w.reshape(n, 1), S.reshape(n, 1, 6), np.full(n, np.inf),
                         np.full(n, np.inf), np.full(n, np.inf), np.full(n, np.inf))
    return oracle.cluster_level(child, np.array([0, n]), K, iters)


def _norm2(X):
    return oracle.lobe_dist(X, np.zeros(6))


def _sse(members, w, S):
    W = w[members].sum()
    c = S[members].sum(0) / W
    return sum(w[m] * oracle.lobe_dist(S[m] / w[m], c) for m in members)


def test_ward_matches_greedy_sse_from_scratch():
    rng = np.random.default_rng(51)
    for trial in range(20):
        n = int(rng.integers(3, 9))
        K = int(rng.integers(1, min(4, n)))
        w, S = _random_lobes(rng, n)
        out = _one_parent(w, S, K, 0)
        clusters = [[i] for i in range(n)]
        while len(clusters) > K:
            best = None
            for i in range(len(clusters)):
                for j in range(i + 1, len(clusters)):
                    inc = _sse(clusters[i] + clusters[j], w, S) - _sse(clusters[i], w, S) - _sse(clusters[j], w, S)
                    if best is None or inc < best[0]:
                        best = (inc, i, j)
            _, i, j = best
            clusters[i] = clusters[i] + clusters[j]
            del clusters[j]
        ws = sorted([w[c].sum() for c in clusters], reverse=True)
        assert out.nl[0] == K
        assert np.allclose(out.w[0, :K], ws, rtol=1e-12)
        got = sorted(map(tuple, np.round(out.S[0, :K], 9)))
        want = sorted(map(tuple, np.round([S[c].sum(0) for c in clusters], 9)))
        assert got == want


def test_lloyd_objective_never_increases_and_sums_are_kept():
    rng = np.random.default_rng(52)
    total_norm = None
    for trial in range(20):
        n = int(rng.integers(5, 17))
        w, S = _random_lobes(rng, n)
        const = sum(w[m] * _norm2(S[m] / w[m]) for m in range(n))
        prev = None
        for it in range(4):
            out = _one_parent(w, S, 3, it)
            k = out.nl[0]
            J = const - sum(out.w[0, i] * _norm2(out.S[0, i] / out.w[0, i]) for i in range(k))
            assert np.isclose(out.w[0, :k].sum(), w.sum()) and np.allclose(out.S[0, :k].sum(0), S.sum(0))
            assert np.all(np.diff(out.w[0, :k]) <= 0)                     # sorted by weight
            if prev is not None:
                assert J <= prev + 1e-9 * const
            prev = J


def test_clustering_special_cases():
    rng = np.random.default_rng(53)
    w, S = _random_lobes(rng, 4)
    out = _one_parent(w, S, 4, 2)                                         # count <= K: unchanged
    order = np.argsort(-w, kind="stable")
    assert out.nl[0] == 4 and np.array_equal(out.w[0], w[order]) and np.array_equal(out.S[0], S[order])
    assert np.isinf(out.gap_rel[0])
    out = _one_parent(w, S, 1, 2)                                         # K = 1: the total
    assert out.nl[0] == 1 and np.isclose(out.w[0, 0], w.sum()) and np.allclose(out.S[0, 0], S.sum(0))
    # two well separated families (fibers along x and along z) are recovered with K = 2
    wx = np.array([1.0, 0.5, 0.7])
    wz = np.array([0.9, 0.3, 1.1])
    Sx = wx[:, None] * np.array([0.02, 1, 0.98, 0.01, 0, 0])
    Sz = wz[:, None] * np.array([1, 0.97, 0.03, 0, 0.01, 0])
    w6 = np.concatenate([wx[:1], wz[:1], wx[1:], wz[1:]])
    S6 = np.concatenate([Sx[:1], Sz[:1], Sx[1:], Sz[1:]])
    out = _one_parent(w6, S6, 2, 2)
    assert out.nl[0] == 2
    got = {round(out.w[0, 0], 12), round(out.w[0, 1], 12)}
    assert got == {round(wx.sum(), 12), round(wz.sum(), 12)}
    # identical lobes are merged first (zero cost)
    w3 = np.array([1.0, 1.0, 1.0])
    S3 = np.array([[1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0]], dtype=float)
    out = _one_parent(w3, S3, 2, 0)
    assert np.allclose(out.S[0, 0], [2, 0, 0, 0, 0, 0]) and np.allclose(out.S[0, 1], [0, 1, 0, 0, 0, 0])
    # an exact tie between the pairs (0, 2) and (1, 3) goes to the lexicographically first pair
    w4 = np.ones(4)
    S4 = np.array([[1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 1, 0, 0, 0, 0]], dtype=float)
    out = _one_parent(w4, S4, 3, 0)
    assert out.gap_rel[0] == 0.0
    assert np.allclose(out.S[0, 0], [2, 0, 0, 0, 0, 0]) and np.allclose(out.S[0, 1:3].sum(0), [0, 2, 0, 0, 0, 0])


def test_cluster_pyramid_keeps_k1_sums():
    wl = synth.brushed_metal(n=4096, window=48)
    o = oracle.voxelize_triangles(wl.grid, wl.tris)
    lod = oracle.build_lod(o, wl.levels)
    lobes = oracle.cluster_pyramid(lod, 4, 2)
    for L in range(1, wl.levels):
        lb = lobes[L]
        assert lb.nl.max() <= 4
        assert np.allclose(lb.w.sum(1), lod[L].w, rtol=1e-12)
        assert np.allclose(lb.S.sum(1), lod[L].S, rtol=1e-12, atol=1e-12 * lod[L].w.max())
