"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle's tests.

This module only builds geometry (float32 arrays on the host).  It holds none of the
voxelization arithmetic: no snapping, no intersection tests, no clipping, no moments.

The paper measures on fabric, mesh, hair and vegetation datasets that are not
available (Sec. 5, Tab. 3); these generators stand in for them with the same kinds
of input the method's Sec. 3.1 names: triangle soups with non-shared vertices, and
explicit fiber polylines (node collections).  All generation is float64 numpy with
``numpy.random.default_rng(seed)``; the arrays handed out are float32.

Workloads (sizes and recipes are stated once here and in the design notes):

* ``icosphere``      -- 5x subdivided icosahedron (20,480 triangles), radius 0.45,
  centre (0.5, 0.5, 0.5), N(0, 1e-3) jitter per unique vertex, unit-cube bounds, 64^3.
* ``plain_weave``    -- 2,000 fibers x 257 points (256 segments), warp along x and weft
  along y, sinusoidal crimp (period 64 voxels, amplitude 4), helix twist U(-5, 5) deg,
  N(0, 0.3^2) per-point jitter, radius 0.5 voxel, bounds [0, 1024]^3 at 1024^3.
* ``weave_patches``  -- 64 plain-weave patches of uneven size: fiber counts log-uniform in
  [100, 20000], grids 2^(8..11), the plain-weave recipe in voxel units with R/32 yarns per
  direction and 256 segments per fiber (a batched workload of many small and large jobs).
* ``brushed_metal``  -- height field, two triangles per cell, ridge wavelength about 8
  cells along x and about 256 along y, amplitude 2 voxels, 4096^3 (a window of it for tests).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Grid:
    """Cubic grid bounds: R = 2**log2_res voxels per axis cover [bmin, bmin + extent)^3."""
    bmin: tuple
    extent: float
    log2_res: int

    @property
    def res(self) -> int:
        return 1 << self.log2_res


@dataclass
class TriangleWorkload:
    name: str
    grid: Grid
    tris: np.ndarray          # float32 [n, 3, 3]
    levels: int
    K: int


@dataclass
class FiberWorkload:
    name: str
    grid: Grid
    pts: np.ndarray           # float32 [m, 3]
    offsets: np.ndarray       # int64 [F + 1], CSR row starts into pts
    radius: float
    levels: int
    K: int


# ----------------------------------------------------------------------------------------------
# icosphere (small triangle case)
# ----------------------------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def _subdivide(v, f):
    edges = {}
    verts = [row for row in v]
    new_f = []

    def mid(a, b):
        key = (a, b) if a < b else (b, a)
        if key not in edges:
            m = verts[a] + verts[b]
            verts.append(m / np.linalg.norm(m))
            edges[key] = len(verts) - 1
        return edges[key]

    for a, b, c in f:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        new_f += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
    return np.array(verts), np.array(new_f, dtype=np.int64)


def icosphere(subdiv: int = 5, radius: float = 0.45, centre=(0.5, 0.5, 0.5), jitter: float = 1e-3,
              seed: int = 0, log2_res: int = 6, levels: int = 7) -> TriangleWorkload:
    rng = np.random.default_rng(seed)
    v, f = _icosahedron()
    for _ in range(subdiv):
        v, f = _subdivide(v, f)
    p = np.asarray(centre, dtype=np.float64) + radius * v
    p = p + rng.normal(0.0, jitter, size=p.shape)
    tris = p[f].astype(np.float32)                       # soup: non-shared vertices
    return TriangleWorkload("icosphere", Grid((0.0, 0.0, 0.0), 1.0, log2_res), tris, levels, 1)


# ----------------------------------------------------------------------------------------------
# plain-weave fabric (fiber case; the measured workload)
# ----------------------------------------------------------------------------------------------

def plain_weave(n_fibers: int = 2000, n_points: int = 257, res: int = 1024, seed: int = 1,
                pitch: float = 32.0, ellipse=(10.0, 2.5), crimp_amp: float = 4.0,
                twist_deg: float = 5.0, jitter: float = 0.3, radius: float = 0.5,
                levels: int | None = None) -> FiberWorkload:
    """Warp fibers (first half) run along x, weft fibers (second half) along y.

    Yarn j = f mod (res / pitch); yarn centre in the cross direction at pitch/2 + pitch*j.
    Crimp: z = res/2 +/- amp * cos(pi (s - pitch/2) / pitch + pi j) (period 2*pitch),
    warp with +, weft with -, so crossing yarns alternate over and under.
    Each fiber sits at a uniform offset in the yarn's elliptical cross section
    (semi-axes ``ellipse`` = (in-plane, z)) that rotates along the yarn as a helix of
    angle theta ~ U(-twist, twist): d(angle)/ds = tan(theta) / max(rho, 1) with rho the
    offset magnitude in voxels.  Points sit at s = 2 + (res - 4) k / (n_points - 1), and
    every coordinate gets N(0, jitter^2) noise.
    """
    rng = np.random.default_rng(seed)
    n_yarn = max(1, int(round(res / pitch)))
    half = n_fibers // 2
    k = np.arange(n_points, dtype=np.float64)
    s = 2.0 + (res - 4.0) * k / (n_points - 1)
    pts = np.empty((n_fibers, n_points, 3), dtype=np.float64)
    a_in, a_z = ellipse
    mid = res / 2.0
    for f in range(n_fibers):
        j = f % n_yarn
        centre = pitch / 2.0 + pitch * j
        r = math.sqrt(rng.uniform())
        alpha0 = rng.uniform(0.0, 2.0 * math.pi)
        theta = math.radians(rng.uniform(-twist_deg, twist_deg))
        rho = math.hypot(a_in * r * math.cos(alpha0), a_z * r * math.sin(alpha0))
        alpha = alpha0 + s * math.tan(theta) / max(rho, 1.0)
        off_in = a_in * r * np.cos(alpha)
        off_z = a_z * r * np.sin(alpha)
        phase = math.pi * (s - pitch / 2.0) / pitch + math.pi * j
        if f < half:            # warp: axis x
            pts[f, :, 0] = s
            pts[f, :, 1] = centre + off_in
            pts[f, :, 2] = mid + crimp_amp * np.cos(phase) + off_z
        else:                   # weft: axis y
            pts[f, :, 0] = centre + off_in
            pts[f, :, 1] = s
            pts[f, :, 2] = mid - crimp_amp * np.cos(phase) + off_z
        pts[f] += rng.normal(0.0, jitter, size=(n_points, 3))
    log2_res = int(round(math.log2(res)))
    offsets = np.arange(0, n_fibers * n_points + 1, n_points, dtype=np.int64)
    return FiberWorkload("plain_weave", Grid((0.0, 0.0, 0.0), float(res), log2_res),
                         pts.reshape(-1, 3).astype(np.float32), offsets, radius,
                         levels if levels is not None else log2_res + 1, 1)


def weave_fibers(rng, n_fibers: int, res: int, n_points: int = 257, pitch: float = 32.0,
                 ellipse=(10.0, 2.5), crimp_amp: float = 4.0, twist_deg: float = 5.0,
                 jitter: float = 0.3):
    """The plain-weave recipe (see ``plain_weave``) drawn for all fibers at once: per-fiber
    (r, alpha0, theta) as three vectors, then the point jitter as one [F, n_points, 3] draw.
    Returns float64 points [F, n_points, 3]."""
    n_yarn = max(1, int(round(res / pitch)))
    half = n_fibers // 2
    f = np.arange(n_fibers)
    j = (f % n_yarn)[:, None]
    centre = pitch / 2.0 + pitch * j
    r = np.sqrt(rng.uniform(size=n_fibers))[:, None]
    alpha0 = rng.uniform(0.0, 2.0 * math.pi, size=n_fibers)[:, None]
    theta = np.radians(rng.uniform(-twist_deg, twist_deg, size=n_fibers))[:, None]
    a_in, a_z = ellipse
    s = (2.0 + (res - 4.0) * np.arange(n_points, dtype=np.float64) / (n_points - 1))[None, :]
    rho = np.hypot(a_in * r * np.cos(alpha0), a_z * r * np.sin(alpha0))
    alpha = alpha0 + s * np.tan(theta) / np.maximum(rho, 1.0)
    off_in = a_in * r * np.cos(alpha)
    off_z = a_z * r * np.sin(alpha)
    phase = math.pi * (s - pitch / 2.0) / pitch + math.pi * j
    warp = (f < half)[:, None]
    mid = res / 2.0
    pts = np.empty((n_fibers, n_points, 3), dtype=np.float64)
    pts[:, :, 0] = np.where(warp, s, centre + off_in)
    pts[:, :, 1] = np.where(warp, centre + off_in, s)
    pts[:, :, 2] = mid + np.where(warp, 1.0, -1.0) * crimp_amp * np.cos(phase) + off_z
    pts += rng.normal(0.0, jitter, size=pts.shape)
    return pts


def weave_patches(n_patches: int = 64, seed: int = 3, fibers=(100, 20000), log2_res=(8, 11),
                  n_points: int = 257, radius: float = 0.5, K: int = 4) -> list:
    """Uneven batch: patch p has n_p = round(exp U(ln lo, ln hi)) fibers on a 2^l grid with
    l ~ U{log2_res[0] .. log2_res[1]}, each patch drawn with ``weave_fibers`` in its own voxel
    units (bounds [0, R)^3), full pyramid per patch, K lobes per coarse voxel."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_patches):
        n = int(round(math.exp(rng.uniform(math.log(fibers[0]), math.log(fibers[1])))))
        l2 = int(rng.integers(log2_res[0], log2_res[1] + 1))
        res = 1 << l2
        pts = weave_fibers(rng, n, res, n_points=n_points)
        offsets = np.arange(0, n * n_points + 1, n_points, dtype=np.int64)
        out.append(FiberWorkload(f"weave_patch_{p}", Grid((0.0, 0.0, 0.0), float(res), l2),
                                 pts.reshape(-1, 3).astype(np.float32), offsets, radius, l2 + 1, K))
    return out


# ----------------------------------------------------------------------------------------------
# brushed-metal height field (large triangle case)
# ----------------------------------------------------------------------------------------------

def brushed_metal(n: int = 4096, window: int | None = None, seed: int = 2, amp: float = 2.0,
                  n_waves: int = 16, K: int = 4) -> TriangleWorkload:
    """Vertex (i, j), 0 <= i, j < n: x = i + 1/2, y = j + 1/2, z = n/2 + amp * h / max|h| with
    h = sum_m cos(2 pi (fx_m x + fy_m y) + phi_m), fx_m ~ U(0.9, 1.1) / 8,
    fy_m = +-U(0.5, 1.5) / 256, phi_m ~ U(0, 2 pi).  Two triangles per cell.

    ``window`` keeps only the first ``window`` x ``window`` vertices (the same surface,
    cut), so small test cases are pieces of the full one.  The height normalisation
    max|h| is taken over the full n x n field so that windows agree with it.
    """
    rng = np.random.default_rng(seed)
    fx = rng.uniform(0.9, 1.1, n_waves) / 8.0
    fy = rng.choice([-1.0, 1.0], n_waves) * rng.uniform(0.5, 1.5, n_waves) / 256.0
    ph = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    m = n if window is None else min(window, n)

    def field(ii, jj):
        x = ii + 0.5
        y = jj + 0.5
        h = np.zeros(np.broadcast(x, y).shape, dtype=np.float64)
        for a in range(n_waves):
            h += np.cos(2.0 * math.pi * (fx[a] * x + fy[a] * y) + ph[a])
        return h

    # normalisation over the full field, computed in row blocks to bound memory
    hmax = 0.0
    jj = np.arange(n, dtype=np.float64)[None, :]
    for i0 in range(0, n, 256):
        ii = np.arange(i0, min(n, i0 + 256), dtype=np.float64)[:, None]
        hmax = max(hmax, float(np.abs(field(ii, jj)).max()))
    ii = np.arange(m, dtype=np.float64)[:, None]
    jm = np.arange(m, dtype=np.float64)[None, :]
    z = n / 2.0 + amp * field(ii, jm) / hmax
    xs = np.broadcast_to(ii + 0.5, (m, m))
    ys = np.broadcast_to(jm + 0.5, (m, m))
    V = np.stack([xs, ys, z], axis=-1)                    # [m, m, 3] float64
    v00 = V[:-1, :-1].reshape(-1, 3)
    v10 = V[1:, :-1].reshape(-1, 3)
    v01 = V[:-1, 1:].reshape(-1, 3)
    v11 = V[1:, 1:].reshape(-1, 3)
    ncell = v00.shape[0]
    tris = np.empty((2 * ncell, 3, 3), dtype=np.float32)
    tris[0::2, 0], tris[0::2, 1], tris[0::2, 2] = v00, v10, v11
    tris[1::2, 0], tris[1::2, 1], tris[1::2, 2] = v00, v11, v01
    log2_res = int(round(math.log2(n)))
    return TriangleWorkload("brushed_metal" if window is None else f"brushed_metal_{m}",
                            Grid((0.0, 0.0, 0.0), float(n), log2_res), tris, log2_res + 1, K)


def random_triangles(n: int, log2_res: int, seed: int, scale: float = 1.0, margin: float = 0.0,
                     extent: float = 1.0) -> TriangleWorkload:
    """Uniformly random triangles with edge lengths ~ ``scale`` voxels; vertices may leave the
    grid by up to ``margin`` voxels.  Used for small parity and edge cases."""
    rng = np.random.default_rng(seed)
    R = 1 << log2_res
    c = rng.uniform(-margin, R + margin, size=(n, 1, 3))
    tris = c + rng.normal(0.0, scale, size=(n, 3, 3))
    tris = np.clip(tris, -margin, R + margin) * (extent / R)
    return TriangleWorkload("random_triangles", Grid((0.0, 0.0, 0.0), extent, log2_res),
                            tris.astype(np.float32), log2_res + 1, 1)


def random_fibers(n_fibers: int, n_points: int, log2_res: int, seed: int, step: float = 1.0,
                  radius: float = 0.5, margin: float = 0.0, inset: float = 0.0) -> FiberWorkload:
    """Random-walk polylines (step ``step`` voxels) in a grid of extent R, starting in
    [inset, R - inset]^3 and clamped to [-margin, R + margin]; used for small cases."""
    rng = np.random.default_rng(seed)
    R = 1 << log2_res
    start = rng.uniform(inset, R - inset, size=(n_fibers, 1, 3))
    steps = rng.normal(0.0, step, size=(n_fibers, n_points, 3))
    steps[:, 0] = 0.0
    p = np.clip(start + np.cumsum(steps, axis=1), -margin, R + margin)
    offsets = np.arange(0, n_fibers * n_points + 1, n_points, dtype=np.int64)
    return FiberWorkload("random_fibers", Grid((0.0, 0.0, 0.0), float(R), log2_res),
                         p.reshape(-1, 3).astype(np.float32), offsets, radius, log2_res + 1, 1)


WORKLOADS = {
    "icosphere": icosphere,
    "plain_weave": plain_weave,
    "brushed_metal": brushed_metal,
}


def fibonacci_dirs(n: int = 128) -> np.ndarray:
    """The fit's direction set: n Fibonacci points on the unit sphere, z = 1 - (2k+1)/n,
    phi = k pi (3 - sqrt 5), computed in FP64 and rounded once to float32 (the values both the
    GPU path and the oracle then evaluate with)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * (np.pi * (3.0 - np.sqrt(5.0)))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1).astype(np.float32)
