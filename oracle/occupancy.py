"""Sub-voxel occupancy and projected densities -- TEST INFRASTRUCTURE (only tests/, smoke() and
bench.py's CPU baseline may use it).

Sec. 3.5 measures the occupancy O of a voxel on a finer third level of 8 cells per axis inside it:
the share of those cells that hold something, and a density per axis from the cells' projections
onto the XY, XZ and YZ planes; Sec. 4.2 gives the coarser levels the same projections.

Reading (exact-measure, like the rest of the oracle): a sub-cell is hit when a primitive touches
its closed box, with the voxel level's touch predicate on the same snapped geometry.  The
sub-cells of all voxels of a grid of resolution R are then exactly the voxels of the grid of
resolution 8 R, and this module takes them from the oracle voxelizer run at log2 R + 3:

    fine key K  ->  voxel key K >> 9,  sub-cell index K & 511 (its 3-bit Morton coordinates)

A level-L voxel keeps 8^3 sub-cells of its own size / 8; a closed box is the union of the closed
boxes of its eight halves, so such a sub-cell is hit exactly when one of the fine sub-cells inside
it is, and level L's sub-cells are the fine keys shifted right by 3 L.

Per voxel (every level): mask = the 512 sub-cell bits (bit m of word m >> 6 for sub-cell Morton
index m), hits = popcount (O = hits / 512), and xy, xz, yz = the number of the 64 cells of the
XY, XZ, YZ plane whose column (along z, y, x) holds a hit (the densities are those / 64).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import voxelize_fibers, voxelize_triangles

SUB_BITS = 3          # 8 sub-cells per axis


@dataclass
class OccLevel:
    keys: np.ndarray      # uint64 [n] voxel keys, sorted
    mask: np.ndarray      # uint64 [n, 8] sub-cell bits
    hits: np.ndarray      # int64 [n] hit sub-cells (0..512)
    xy: np.ndarray        # int64 [n] covered cells of the XY plane (0..64), projection along z
    xz: np.ndarray        # int64 [n] ... of the XZ plane, along y
    yz: np.ndarray        # int64 [n] ... of the YZ plane, along x


@dataclass
class _Grid:
    bmin: tuple
    extent: float
    log2_res: int


def _fine_grid(grid):
    if grid.log2_res + SUB_BITS > 20:
        raise ValueError("occupancy needs log2_res <= 17 (sub-cells of a grid of at most 2^20 per axis)")
    return _Grid(tuple(grid.bmin), float(grid.extent), int(grid.log2_res) + SUB_BITS)


def _sub_coords(m):
    """3-bit Morton index -> (i, j, k) sub-cell coordinates, x at bits 0, 3, 6."""
    m = np.asarray(m, dtype=np.int64)
    i = (m & 1) | ((m >> 2) & 2) | ((m >> 4) & 4)
    j = ((m >> 1) & 1) | ((m >> 3) & 2) | ((m >> 5) & 4)
    k = ((m >> 2) & 1) | ((m >> 4) & 2) | ((m >> 6) & 4)
    return i, j, k


def _level(sub_keys) -> OccLevel:
    K = np.unique(np.asarray(sub_keys, dtype=np.uint64))
    vox = K >> np.uint64(9)
    m = (K & np.uint64(511)).astype(np.int64)
    keys, idx = np.unique(vox, return_inverse=True)
    n = len(keys)
    mask = np.zeros((n, 8), dtype=np.uint64)
    np.bitwise_or.at(mask, (idx, m >> 6), np.uint64(1) << (m & 63).astype(np.uint64))
    hits = np.bincount(idx, minlength=n).astype(np.int64)
    i, j, k = _sub_coords(m)

    def covered(a, b):
        cell = np.unique(idx * 64 + a * 8 + b)
        return np.bincount(cell // 64, minlength=n).astype(np.int64)

    return OccLevel(keys, mask, hits, covered(i, j), covered(i, k), covered(j, k))


def occupancy_from_fine(fine_keys, levels: int):
    """Levels 0 .. levels-1 from the voxel keys of the 8x finer grid."""
    K = np.asarray(fine_keys, dtype=np.uint64)
    return [_level(K >> np.uint64(3 * L)) for L in range(levels)]


def occupancy_triangles(grid, tris, levels: int, nthreads=None):
    fine = voxelize_triangles(_fine_grid(grid), tris, nthreads=nthreads)
    return occupancy_from_fine(fine.keys, levels)


def occupancy_fibers(grid, pts, offsets, radius, levels: int, nthreads=None):
    fine = voxelize_fibers(_fine_grid(grid), pts, offsets, radius, nthreads=nthreads)
    return occupancy_from_fine(fine.keys, levels)
