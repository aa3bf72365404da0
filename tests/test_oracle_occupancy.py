"""Pins of the sub-voxel occupancy oracle (Sec. 3.5 occupancy equation and projections, Sec. 4.2
projections for the coarser levels).

The oracle takes the sub-cells from the voxelizer run at 8x the resolution and the coarser levels
by shifting keys; the pins check it against other routes: voxelizations at the other
resolutions themselves, exact-rational brute force per sub-cell, closed forms for an axis-aligned
fiber and for flat right triangles (on a sub-cell boundary, on a voxel face, inside a layer), and
the projections counted from dense boolean grids built from those closed forms.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.occupancy import occupancy_fibers, occupancy_from_fine, occupancy_triangles
import synth


def G(log2_res, extent=None):
    R = 1 << log2_res
    return synth.Grid((0.0, 0.0, 0.0), float(R if extent is None else extent), log2_res)


def dense_cells(lvl, log2_res):
    """{(voxel coords), (i, j, k)} -> set of global sub-cell coordinates (8 per voxel axis)."""
    vc = oracle.demorton(lvl.keys, log2_res)
    out = set()
    for v, words in zip(vc.tolist(), lvl.mask):
        for w in range(8):
            x = int(words[w])
            while x:
                b = (x & -x).bit_length() - 1
                x &= x - 1
                m = 64 * w + b
                i = sum(((m >> (3 * t)) & 1) << t for t in range(3))
                j = sum(((m >> (3 * t + 1)) & 1) << t for t in range(3))
                k = sum(((m >> (3 * t + 2)) & 1) << t for t in range(3))
                out.add((8 * v[0] + i, 8 * v[1] + j, 8 * v[2] + k))
    return out


def projections_from_cells(cells, lvl, log2_res):
    """(hits, xy, xz, yz) per voxel of lvl, counted on dense 8^3 boolean blocks."""
    vc = oracle.demorton(lvl.keys, log2_res)
    index = {tuple(v): n for n, v in enumerate(vc.tolist())}
    blocks = np.zeros((len(vc), 8, 8, 8), bool)
    for (x, y, z) in cells:
        blocks[index[(x >> 3, y >> 3, z >> 3)], x & 7, y & 7, z & 7] = True
    return (blocks.sum((1, 2, 3)), blocks.any(3).sum((1, 2)), blocks.any(2).sum((1, 2)),
            blocks.any(1).sum((1, 2)))


def check_projections(lvl, log2_res):
    cells = dense_cells(lvl, log2_res)
    h, xy, xz, yz = projections_from_cells(cells, lvl, log2_res)
    assert np.array_equal(h, lvl.hits) and np.array_equal(xy, lvl.xy)
    assert np.array_equal(xz, lvl.xz) and np.array_equal(yz, lvl.yz)


def test_levels_match_voxelizations_at_every_resolution():
    """Level L's voxels are the voxelization at R / 2^L and its sub-cells the voxelization at
    8 R / 2^L (a closed box is the union of its halves' closed boxes); every voxel holds a hit."""
    tw = synth.random_triangles(30, 4, seed=5, scale=2.5, margin=1.0)
    fw = synth.random_fibers(4, 12, 4, seed=6, step=1.3, margin=1.0)
    for kind, wl in (("tri", tw), ("fib", fw)):
        levels = 4
        if kind == "tri":
            occ = occupancy_triangles(wl.grid, wl.tris, levels)
            vox = lambda g: oracle.voxelize_triangles(g, wl.tris)
        else:
            occ = occupancy_fibers(wl.grid, wl.pts, wl.offsets, 0.7, levels)
            vox = lambda g: oracle.voxelize_fibers(g, wl.pts, wl.offsets, 0.7)
        lod = oracle.build_lod(vox(wl.grid), levels)
        for L in range(levels):
            assert np.array_equal(occ[L].keys, lod[L].keys), (kind, L)
            assert occ[L].hits.min() >= 1
            # the level's sub-cells straight from the voxelizer at 8 R / 2^L
            direct = occupancy_from_fine(vox(G(wl.grid.log2_res + 3 - L, wl.grid.extent)).keys, 1)[0]
            assert np.array_equal(direct.keys, occ[L].keys) and np.array_equal(direct.mask, occ[L].mask), (kind, L)
            check_projections(occ[L], wl.grid.log2_res - L)


def test_brute_force_every_sub_cell():
    """R = 2: every sub-cell of every voxel against exact-rational clipping (triangles) and the
    Minkowski decomposition (a capsule)."""
    grid = G(1, 2.0)
    tris = np.array([[[0.13, 0.27, 0.61], [1.71, 0.44, 1.05], [0.52, 1.83, 0.33]],
                     [[1.0, 0.25, 1.5], [1.0, 1.75, 1.5], [1.0, 0.25, 0.125]]], np.float32)
    pts = np.array([[0.2, 0.9, 1.3], [1.85, 1.1, 0.7]], np.float32)
    s = brute.voxel_size(grid) // 8
    q = brute.lattice(grid, tris.reshape(-1, 3)).reshape(-1, 3, 3)
    a, b = brute.lattice(grid, pts)
    rho = int(np.rint(np.float32(0.3) * (8388608.0 / grid.extent)))
    for kind in ("tri", "fib"):
        occ = (occupancy_triangles(grid, tris, 1) if kind == "tri"
               else occupancy_fibers(grid, pts, [0, 2], 0.3, 1))[0]
        got = dense_cells(occ, 1)
        want = set()
        for x in range(16):
            for y in range(16):
                for z in range(16):
                    lo = (x * s, y * s, z * s)
                    if kind == "tri":
                        hit = any(brute.tri_touch(t, lo, s) for t in q)
                    else:
                        hit = brute.cap_touch(a, b, lo, s, rho)
                    if hit:
                        want.add((x, y, z))
        assert got == want, kind


def test_axis_aligned_fiber_closed_form():
    """A fiber along x at (y0, z0): sub-cell (I, J, K) is hit when the distance from the segment
    to its closed box, dx^2 + d_yz^2 in lattice units, is at most the radius squared."""
    grid = G(3)                                  # 8 voxels, lattice 2^20 per voxel, sub-cell 2^17
    sub = 1 << 17
    x0, x1, y0, z0 = 1.3125, 6.5, 3.25, 4.5      # z0 on a sub-cell boundary, y0 inside one
    r = 0.375
    pts = np.array([[x0, y0, z0], [x1, y0, z0]], np.float32)
    occ = occupancy_fibers(grid, pts, [0, 2], r, 4)
    L = 1 << 20
    X0, X1, Y0, Z0, RR = int(x0 * L), int(x1 * L), int(y0 * L), int(z0 * L), int(r * L)

    def gap(c, lo, hi):
        return max(lo - c, 0, c - hi)

    want = set()
    for I in range(64):
        for J in range(64):
            for K in range(64):
                dx = max(I * sub - X1, 0, X0 - (I + 1) * sub)
                dy = gap(Y0, J * sub, (J + 1) * sub)
                dz = gap(Z0, K * sub, (K + 1) * sub)
                if dx * dx + dy * dy + dz * dz <= RR * RR:
                    want.add((I, J, K))
    assert dense_cells(occ[0], 3) == want
    check_projections(occ[0], 3)
    # coarser levels: the same rule on sub-cells twice, four, eight times as large
    for lev in range(1, 4):
        S = sub << lev
        wl = set()
        for I in range(64):
            for J in range(64):
                for K in range(64):
                    dx = max(I * S - X1, 0, X0 - (I + 1) * S)
                    dy = gap(Y0, J * S, (J + 1) * S)
                    dz = gap(Z0, K * S, (K + 1) * S)
                    if I * S < 8 * L and J * S < 8 * L and K * S < 8 * L and dx * dx + dy * dy + dz * dz <= RR * RR:
                        wl.add((I, J, K))
        assert dense_cells(occ[lev], 3 - lev) == wl, lev


@pytest.mark.parametrize("c,layers", [(2.4375, None), (2.5, "sub"), (3.0, "voxel")])
def test_flat_right_triangle_closed_form(c, layers):
    """Right triangle in the plane z = c with legs along x and y: the closed square [X0, X1] x
    [Y0, Y1] meets it when X1 >= x0, Y1 >= y0 and its corner nearest the right angle satisfies
    b (X - x0) + a (Y - y0) <= a b; the closed z-range must hold c (two layers of sub-cells
    when c lies on a sub-cell boundary, and on a voxel face two voxels' layers)."""
    grid = G(3)
    sub = 1 << 17
    x0, y0, a, b = 0.75, 1.125, 5.5, 4.25
    tri = np.array([[[x0, y0, c], [x0 + a, y0, c], [x0, y0 + b, c]]], np.float32)
    occ = occupancy_triangles(grid, tri, 1)[0]
    L = 1 << 20
    X0, Y0, A, B, C = int(x0 * L), int(y0 * L), int(a * L), int(b * L), int(c * L)
    want = set()
    for I in range(64):
        for J in range(64):
            for K in range(64):
                if not (K * sub <= C <= (K + 1) * sub):
                    continue
                xl, xh, yl, yh = I * sub, (I + 1) * sub, J * sub, (J + 1) * sub
                if xh < X0 or yh < Y0 or xl > X0 + A or yl > Y0 + B:
                    continue
                X, Y = max(xl, X0), max(yl, Y0)
                if B * (X - X0) + A * (Y - Y0) <= A * B:
                    want.add((I, J, K))
    got = dense_cells(occ, 3)
    assert got == want
    nlayers = len({k for (_, _, k) in got})
    assert nlayers == (1 if layers is None else 2)
    check_projections(occ, 3)
    # a voxel whose whole square the triangle covers: 64 cells per layer
    full = [n for n, h in enumerate(occ.hits) if occ.xy[n] == 64]
    assert full and all(occ.hits[n] == 64 * (1 if layers != "sub" else 2) for n in full
                        if layers != "voxel")
    for n in full:
        assert occ.xz[n] == 8 * (occ.hits[n] // 64) and occ.yz[n] == occ.xz[n]
