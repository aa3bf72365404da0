"""Exact-rational brute force for tiny grids -- TEST INFRASTRUCTURE that pins the oracle.

Every voxel of the grid is tested against every primitive (no candidate ranges), with
Python ``fractions.Fraction`` arithmetic and methods chosen to differ from ``vxo.cpp``:

* triangle touches closed box  <=>  Sutherland-Hodgman clipping of the triangle by the six
  closed half-spaces leaves a point (``vxo.cpp`` uses a separating-axis test instead);
* triangle weight = area of the exact rational clipped polygon, with the half-open rule for
  triangles lying in an axis plane (Sec. 3.3 gathering; the ownership reading);
* capsule touches closed box  <=>  the segment meets the Minkowski sum box + ball(r),
  decomposed into 3 slab boxes, 12 edge cylinders and 8 corner balls (``vxo.cpp`` minimises
  the piecewise-quadratic distance instead);
* segment weight = exact Liang-Barsky parameter interval times the segment length.

Lattice coordinates come from ``lattice()`` below, an independent numpy statement of the
Sec. 3.1 transform.
"""
from __future__ import annotations

from fractions import Fraction as Fr
import math

import numpy as np


def lattice(grid, pts) -> np.ndarray:
    """Sec. 3.1: P_volume = (P - bmin) / extent * R, on the lattice of 2^-(23 - log2 R) voxel.
    numpy float64 subtract and multiply round correctly, np.rint rounds half to even."""
    p = np.asarray(pts, dtype=np.float32).reshape(-1, 3).astype(np.float64)
    inv = 8388608.0 / float(grid.extent)
    return np.rint((p - np.asarray(grid.bmin, dtype=np.float64)) * inv).astype(np.int64)


def voxel_size(grid) -> int:
    return 1 << (23 - grid.log2_res)


# ------------------------------------------------------------------------------------------------
# triangles
# ------------------------------------------------------------------------------------------------

def _clip(poly, axis, bound, keep_ge):
    """Clip a convex polygon (list of Fraction 3-tuples) by x[axis] >= bound (or <= bound)."""
    out = []
    n = len(poly)
    for i in range(n):
        P, Q = poly[i], poly[(i + 1) % n]
        dp = (P[axis] - bound) if keep_ge else (bound - P[axis])
        dq = (Q[axis] - bound) if keep_ge else (bound - Q[axis])
        if dp >= 0:
            out.append(P)
        if (dp >= 0) != (dq >= 0):
            t = dp / (dp - dq)
            out.append(tuple(P[c] + t * (Q[c] - P[c]) for c in range(3)))
    return out


def tri_touch(q, lo, s) -> bool:
    poly = [tuple(Fr(int(v)) for v in q[i]) for i in range(3)]
    for a in range(3):
        poly = _clip(poly, a, Fr(int(lo[a])), True)
        if not poly:
            return False
        poly = _clip(poly, a, Fr(int(lo[a]) + s), False)
        if not poly:
            return False
    return True


def tri_area(q, lo, s) -> float:
    """Area (voxel units) of the triangle inside [lo, lo + s)^3."""
    poly = [tuple(Fr(int(v)) for v in q[i]) for i in range(3)]
    for a in range(3):
        col = [int(q[i][a]) for i in range(3)]
        if col[0] == col[1] == col[2]:
            if not (lo[a] <= col[0] < lo[a] + s):
                return 0.0
            continue
        poly = _clip(poly, a, Fr(int(lo[a])), True)
        poly = _clip(poly, a, Fr(int(lo[a]) + s), False)
        if len(poly) < 3:
            return 0.0
    ax = [Fr(0)] * 3
    n = len(poly)
    for i in range(n):
        P, Q = poly[i], poly[(i + 1) % n]
        ax[0] += P[1] * Q[2] - P[2] * Q[1]
        ax[1] += P[2] * Q[0] - P[0] * Q[2]
        ax[2] += P[0] * Q[1] - P[1] * Q[0]
    a2 = ax[0] ** 2 + ax[1] ** 2 + ax[2] ** 2          # (2 * area)^2 in lattice units^4
    return math.sqrt(a2) / 2.0 / float(s) ** 2


def tri_moment(q) -> np.ndarray:
    e0 = [int(q[1][a]) - int(q[0][a]) for a in range(3)]
    e1 = [int(q[2][a]) - int(q[0][a]) for a in range(3)]
    n = [e0[1] * e1[2] - e0[2] * e1[1], e0[2] * e1[0] - e0[0] * e1[2], e0[0] * e1[1] - e0[1] * e1[0]]
    l2 = sum(x * x for x in n)
    if l2 == 0:
        return np.zeros(6)
    nn = [Fr(x) for x in n]
    return np.array([float(nn[0] * nn[0] / l2), float(nn[1] * nn[1] / l2), float(nn[2] * nn[2] / l2),
                     float(nn[0] * nn[1] / l2), float(nn[0] * nn[2] / l2), float(nn[1] * nn[2] / l2)])


# ------------------------------------------------------------------------------------------------
# capsules
# ------------------------------------------------------------------------------------------------

def _slab_interval(A, d, axis, lo, hi, t0, t1):
    """Restrict [t0, t1] to the parameters where lo <= A + t d <= hi on one axis (closed)."""
    if d[axis] == 0:
        return (t0, t1) if lo <= A[axis] <= hi else None
    ta = (lo - A[axis]) / d[axis]
    tb = (hi - A[axis]) / d[axis]
    if ta > tb:
        ta, tb = tb, ta
    t0, t1 = max(t0, ta), min(t1, tb)
    return (t0, t1) if t0 <= t1 else None


def _min_quad_on(A, d, axes, centre, t0, t1):
    """min over t in [t0, t1] of sum over axes of (A + t d - centre)^2, exactly."""
    dd = sum(d[a] * d[a] for a in axes)
    if dd == 0:
        t = t0
    else:
        t = -sum((A[a] - centre[a]) * d[a] for a in axes) / dd
        t = min(max(t, t0), t1)
    return sum((A[a] + t * d[a] - centre[a]) ** 2 for a in axes)


def cap_touch(a, b, lo, s, rho) -> bool:
    A = [Fr(int(x)) for x in a]
    d = [Fr(int(b[k]) - int(a[k])) for k in range(3)]
    lo = [Fr(int(x)) for x in lo]
    hi = [x + s for x in lo]
    r2 = Fr(int(rho)) ** 2
    rho = Fr(int(rho))
    # three slab boxes: the box grown by rho along one axis
    for g in range(3):
        iv = (Fr(0), Fr(1))
        for k in range(3):
            ext = rho if k == g else 0
            iv = _slab_interval(A, d, k, lo[k] - ext, hi[k] + ext, *iv)
            if iv is None:
                break
        if iv is not None:
            return True
    # twelve edge cylinders: axis k of the edge, the two others fixed at a corner value
    for k in range(3):
        u, v = [x for x in range(3) if x != k]
        iv = _slab_interval(A, d, k, lo[k], hi[k], Fr(0), Fr(1))
        if iv is None:
            continue
        for cu in (lo[u], hi[u]):
            for cv in (lo[v], hi[v]):
                c = [None] * 3
                c[u], c[v] = cu, cv
                if _min_quad_on(A, d, (u, v), c, *iv) <= r2:
                    return True
    # eight corner balls
    for cx in (lo[0], hi[0]):
        for cy in (lo[1], hi[1]):
            for cz in (lo[2], hi[2]):
                if _min_quad_on(A, d, (0, 1, 2), (cx, cy, cz), Fr(0), Fr(1)) <= r2:
                    return True
    return False


def seg_length(a, b, lo, s) -> float:
    """Length (voxel units) of the segment inside [lo, lo + s)^3."""
    A = [Fr(int(x)) for x in a]
    d = [Fr(int(b[k]) - int(a[k])) for k in range(3)]
    t0, t1 = Fr(0), Fr(1)
    for k in range(3):
        if d[k] == 0:
            if not (lo[k] <= A[k] < lo[k] + s):
                return 0.0
            continue
        ta = (lo[k] - A[k]) / d[k]
        tb = (lo[k] + s - A[k]) / d[k]
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
    if t1 <= t0:
        return 0.0
    return float(t1 - t0) * math.sqrt(sum(int(x) ** 2 for x in d)) / float(s)


def seg_moment(a, b) -> np.ndarray:
    d = [int(b[k]) - int(a[k]) for k in range(3)]
    l2 = sum(x * x for x in d)
    if l2 == 0:
        return np.zeros(6)
    f = [Fr(x) for x in d]
    return np.array([float(1 - f[0] * f[0] / l2), float(1 - f[1] * f[1] / l2), float(1 - f[2] * f[2] / l2),
                     float(-f[0] * f[1] / l2), float(-f[0] * f[2] / l2), float(-f[1] * f[2] / l2)])


# ------------------------------------------------------------------------------------------------
# dense voxelization
# ------------------------------------------------------------------------------------------------

def _morton(x, y, z, bits):
    k = 0
    for b in range(bits):
        k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return k


def _collect(grid, prims, touch, weight, moment):
    R = grid.res
    s = voxel_size(grid)
    acc = {}
    for prim in prims:
        M = moment(prim)
        for z in range(R):
            for y in range(R):
                for x in range(R):
                    lo = (x * s, y * s, z * s)
                    if not touch(prim, lo, s):
                        continue
                    w = weight(prim, lo, s)
                    k = _morton(x, y, z, grid.log2_res)
                    c, ww, S = acc.get(k, (0, 0.0, np.zeros(6)))
                    acc[k] = (c + 1, ww + w, S + w * M)
    keys = np.array(sorted(acc), dtype=np.uint64)
    return (keys, np.array([acc[int(k)][0] for k in keys], dtype=np.uint32),
            np.array([acc[int(k)][1] for k in keys]), np.array([acc[int(k)][2] for k in keys]).reshape(-1, 6))


def voxelize_triangles(grid, tris):
    q = lattice(grid, np.asarray(tris).reshape(-1, 3)).reshape(-1, 3, 3)
    return _collect(grid, list(q), tri_touch, tri_area, tri_moment)


def voxelize_fibers(grid, pts, offsets, radius):
    q = lattice(grid, pts)
    rho = int(np.rint(float(np.float32(radius)) * (8388608.0 / float(grid.extent))))
    segs = [(q[i], q[i + 1]) for f in range(len(offsets) - 1) for i in range(offsets[f], offsets[f + 1] - 1)]
    return _collect(grid, segs,
                    lambda sg, lo, s: cap_touch(sg[0], sg[1], lo, s, rho),
                    lambda sg, lo, s: seg_length(sg[0], sg[1], lo, s),
                    lambda sg: seg_moment(sg[0], sg[1]))
