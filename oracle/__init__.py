"""FP64 CPU oracle for sparse SGGX voxelization and LoD pyramids -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
import this package.  The product path (``paper_2604_13191_amd``) never calls it, and the
two share no code: the oracle is a separate C++ file built with g++ plus the numpy below.

Functions and the passages they follow:

* ``voxelize_triangles`` / ``voxelize_fibers`` -- Sec. 3.1 (grid transform), Sec. 3.3
  (gathering every contribution to a leaf voxel), Sec. 3.4 / Sec. 4.1 (one SGGX matrix per
  voxel).  Exact lattice predicates, FP64 clipped measures and moment sums (``vxo.cpp``).
* ``build_lod`` -- Sec. 4.3: a coarser voxel aggregates its 2x2x2 children; here as sums
  (the parent's normalised SGGX is the weight-averaged child SGGX), plus a child mask.
* ``cluster_pyramid`` -- Sec. 4.4: agglomerative merging of the most similar lobes down to a
  cap of K per voxel, with the deterministic distance and Lloyd refinement in ``vxo.cpp``.
* ``oracle.compact`` (a module of its own, numpy) -- Sec. 4.1 leaf eigen-fit with an
  eigenvalue floor, and Sec. 4.3's 6-byte compact SGGX code and its decoding.
* ``oracle.occupancy`` (numpy over the voxelizer) -- Sec. 3.5 occupancy of 8^3 sub-cells per
  voxel and its XY / XZ / YZ projections, Sec. 4.2 the same for the coarser levels: the
  sub-cells are the voxels of the voxelizer run at 8x the resolution.
* ``sggxh_level`` / ``sggxh_pyramid`` -- Sec. 4.4 SGGX-H: lobes compared through histograms
  of samples drawn from them (counter-based SplitMix64), a Wasserstein distance, and merges of
  the closest pair by pooling samples (``vxo_sggxh.cpp``).
* ``sample_fibers`` / ``sample_triangles`` -- Sec. 3.2 sampling voxelizer: Catmull-Rom spans
  subdivided into chords with equally spaced samples, and Heitz's low-distortion triangle map
  with sample counts in proportion to the triangle's area (``vxo_sample.cpp``).

Pins (tests/test_oracle_*.py): exact-rational brute force (``oracle/brute.py``) on tiny
grids; conservation of area / length / moment; closed forms for axis-aligned fibers and
flat triangles; the quadrature identity of the lobe distance; brute-force merge orders.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "vxo.cpp"), os.path.join(_HERE, "vxo_fit.cpp"), os.path.join(_HERE, "vxo_sample.cpp"),
         os.path.join(_HERE, "vxo_sggxh.cpp")]
# VXO_SANITIZE=1: a separate build under AddressSanitizer and UndefinedBehaviorSanitizer (load it
# with libasan preloaded; tests/test_oracle_sanitized.py does)
_SAN = os.environ.get("VXO_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libvxo_san.so" if _SAN else "libvxo.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
_lib = None

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile vxo.cpp and vxo_fit.cpp with g++ (plain C++17, FP contraction off) into oracle/libvxo.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
                               "-pthread"] + (_SAN_FLAGS if _SAN else []) + _SRCS + ["-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.vxo_snap.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        L.vxo_morton.restype = ctypes.c_uint64
        L.vxo_morton.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int]
        L.vxo_tri_touch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.vxo_tri_area.restype = ctypes.c_double
        L.vxo_tri_area.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.vxo_cap_touch.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int64]
        L.vxo_seg_length.restype = ctypes.c_double
        L.vxo_seg_length.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64]
        L.vxo_voxelize_triangles.restype = ctypes.c_void_p
        L.vxo_voxelize_triangles.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vxo_voxelize_fibers.restype = ctypes.c_void_p
        L.vxo_voxelize_fibers.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vxo_result_size.restype = ctypes.c_int64
        L.vxo_result_size.argtypes = [ctypes.c_void_p]
        L.vxo_result_npairs.restype = ctypes.c_int64
        L.vxo_result_npairs.argtypes = [ctypes.c_void_p]
        L.vxo_result_copy.argtypes = [ctypes.c_void_p] * 5
        L.vxo_result_free.argtypes = [ctypes.c_void_p]
        L.vxo_cluster_level.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int]
        L.vxo_lobe_dist.restype = ctypes.c_double
        L.vxo_lobe_dist.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid_args(grid):
    bmin = (ctypes.c_double * 3)(*[float(x) for x in grid.bmin])
    return bmin, float(grid.extent), int(grid.log2_res)


class OracleError(RuntimeError):
    pass


def _nthreads(n):
    return int(n) if n else (os.cpu_count() or 1)


@dataclass
class Voxels:
    """Leaf voxels, sorted by Morton key: FP64 weight and unnormalised SGGX sums."""
    keys: np.ndarray      # uint64 [n]
    count: np.ndarray     # uint32 [n]
    w: np.ndarray         # float64 [n]
    S: np.ndarray         # float64 [n, 6]  (xx, yy, zz, xy, xz, yz)
    n_pairs: int = 0


def _take(res) -> Voxels:
    L = lib()
    n = L.vxo_result_size(res)
    v = Voxels(np.empty(n, np.uint64), np.empty(n, np.uint32), np.empty(n, np.float64),
               np.empty((n, 6), np.float64), int(L.vxo_result_npairs(res)))
    L.vxo_result_copy(res, _ptr(v.keys), _ptr(v.count), _ptr(v.w), _ptr(v.S))
    L.vxo_result_free(res)
    return v


def _region_arg(region):
    if region is None:
        return None, None
    r = np.ascontiguousarray(np.asarray(region, dtype=np.int64).reshape(6))
    return r, _ptr(r)


def snap(grid, pts) -> np.ndarray:
    """Sec. 3.1 transform snapped to the 2^-(23 - log2 R) voxel lattice: int64 [n, 3]."""
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float32).reshape(-1, 3))
    q = np.empty(p.shape, dtype=np.int64)
    bmin, ext, l2 = _grid_args(grid)
    st = lib().vxo_snap(bmin, ext, l2, _ptr(p), p.shape[0], _ptr(q))
    if st:
        raise OracleError(f"snap failed with status {st}")
    return q


def voxelize_triangles(grid, tris, region=None, nthreads=None) -> Voxels:
    t = np.ascontiguousarray(np.asarray(tris, dtype=np.float32).reshape(-1, 3, 3))
    bmin, ext, l2 = _grid_args(grid)
    r, rp = _region_arg(region)
    st = ctypes.c_int(0)
    res = lib().vxo_voxelize_triangles(bmin, ext, l2, _ptr(t), t.shape[0], rp, _nthreads(nthreads),
                                       ctypes.byref(st))
    if st.value:
        raise OracleError(f"voxelize_triangles failed with status {st.value}")
    return _take(res)


def voxelize_fibers(grid, pts, offsets, radius, region=None, nthreads=None) -> Voxels:
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float32).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    bmin, ext, l2 = _grid_args(grid)
    r, rp = _region_arg(region)
    st = ctypes.c_int(0)
    res = lib().vxo_voxelize_fibers(bmin, ext, l2, _ptr(p), p.shape[0], _ptr(o), o.shape[0] - 1,
                                    float(np.float32(radius)), rp, _nthreads(nthreads), ctypes.byref(st))
    if st.value:
        raise OracleError(f"voxelize_fibers failed with status {st.value}")
    return _take(res)


def morton(x, y, z, bits) -> int:
    return int(lib().vxo_morton(int(x), int(y), int(z), int(bits)))


def demorton(keys, bits):
    """Inverse of the Morton interleave (x at bit 3b, y at 3b+1, z at 3b+2): int64 [n, 3]."""
    k = np.asarray(keys, dtype=np.uint64)
    out = np.zeros((k.shape[0], 3), dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            out[:, a] |= ((k >> np.uint64(3 * b + a)) & np.uint64(1)).astype(np.int64) << b
    return out


# --------------------------------------------------------------------------------------------
# Sec. 4.3: the pyramid of 2x2x2 aggregates (one lobe per voxel).
# --------------------------------------------------------------------------------------------

@dataclass
class Level:
    keys: np.ndarray      # uint64 [n], sorted
    count: np.ndarray     # uint64 [n]: primitive-voxel pairs under the voxel
    mask: np.ndarray      # uint8 [n]: bit b set when child (key << 3 | b) exists (0 at the leaf)
    w: np.ndarray         # float64 [n]
    S: np.ndarray         # float64 [n, 6]
    child_start: np.ndarray = field(default=None)   # int64 [n+1] into the level below


def build_lod(vox: Voxels, levels: int):
    """Level 0 is the leaf; level L voxel u sums the voxels v of level L-1 with v >> 3 == u."""
    out = [Level(vox.keys.copy(), vox.count.astype(np.uint64), np.zeros(len(vox.keys), np.uint8),
                 vox.w.copy(), vox.S.copy(), None)]
    for _ in range(1, levels):
        prev = out[-1]
        pk = prev.keys >> np.uint64(3)
        if len(pk) == 0:
            out.append(Level(pk, pk.astype(np.uint64), np.zeros(0, np.uint8), np.zeros(0), np.zeros((0, 6)),
                             np.zeros(1, np.int64)))
            continue
        starts = np.flatnonzero(np.concatenate([[True], pk[1:] != pk[:-1]]))
        bits = (np.uint64(1) << (prev.keys & np.uint64(7))).astype(np.uint8)
        lvl = Level(pk[starts],
                    np.add.reduceat(prev.count, starts),
                    np.bitwise_or.reduceat(bits, starts).astype(np.uint8),
                    np.add.reduceat(prev.w, starts),
                    np.add.reduceat(prev.S, starts, axis=0),
                    np.append(starts, len(pk)).astype(np.int64))
        out.append(lvl)
    return out


# --------------------------------------------------------------------------------------------
# Sec. 4.4: lobe clustering per coarse voxel.
# --------------------------------------------------------------------------------------------

@dataclass
class Lobes:
    nl: np.ndarray        # int32 [n]
    w: np.ndarray         # float64 [n, K]
    S: np.ndarray         # float64 [n, K, 6]
    gap_rel: np.ndarray   # float64 [n]: least relative margin of a decision taken for the voxel
    gap_abs: np.ndarray   # float64 [n]: least margin relative to the voxel's weight
    tie_gap_rel: np.ndarray = None   # least gap_rel over the voxel and all its descendants
    tie_gap_abs: np.ndarray = None


def lobe_dist(A, B) -> float:
    """D(A, B) = 2 tr(Delta^2) + (tr Delta)^2 for normalised lobes given as (xx, yy, zz, xy, xz, yz)."""
    a = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(B, dtype=np.float64)
    return float(lib().vxo_lobe_dist(_ptr(a), _ptr(b)))


def cluster_level(child: Lobes, child_start, K: int, iters: int, nthreads=None) -> Lobes:
    n_par = len(child_start) - 1
    Kc = child.w.shape[1]
    out = Lobes(np.zeros(n_par, np.int32), np.zeros((n_par, K)), np.zeros((n_par, K, 6)),
                np.zeros(n_par), np.zeros(n_par))
    cs = np.ascontiguousarray(child_start, dtype=np.int64)
    cnl = np.ascontiguousarray(child.nl, dtype=np.int32)
    cw = np.ascontiguousarray(child.w, dtype=np.float64)
    cS = np.ascontiguousarray(child.S, dtype=np.float64)
    lib().vxo_cluster_level(n_par, _ptr(cs), _ptr(cnl), _ptr(cw), _ptr(cS), Kc, int(K), int(iters),
                            _ptr(out.nl), _ptr(out.w), _ptr(out.S), _ptr(out.gap_rel), _ptr(out.gap_abs),
                            _nthreads(nthreads))
    # decision margins inherited from the subtree
    seg_min_rel = np.minimum.reduceat(child.tie_gap_rel, cs[:-1]) if n_par else np.zeros(0)
    seg_min_abs = np.minimum.reduceat(child.tie_gap_abs, cs[:-1]) if n_par else np.zeros(0)
    out.tie_gap_rel = np.minimum(out.gap_rel, seg_min_rel)
    out.tie_gap_abs = np.minimum(out.gap_abs, seg_min_abs)
    return out


def cluster_pyramid(lod, K: int, iters: int = 2, nthreads=None):
    """Per level L >= 1: at most K lobes per voxel, merged from the lobes of its children."""
    leaf = lod[0]
    n0 = len(leaf.keys)
    cur = Lobes((leaf.w > 0).astype(np.int32), leaf.w.reshape(n0, 1).copy(), leaf.S.reshape(n0, 1, 6).copy(),
                np.full(n0, np.inf), np.full(n0, np.inf), np.full(n0, np.inf), np.full(n0, np.inf))
    out = [cur]
    for L in range(1, len(lod)):
        cur = cluster_level(cur, lod[L].child_start, K, iters, nthreads)
        out.append(cur)
    return out


# --------------------------------------------------------------------------------------------
# Differentiable lobe fit (vxo_fit.cpp): loss and analytic gradients in FP64.
# --------------------------------------------------------------------------------------------

FIT_NDIR = 128


def fit_dirs(n=FIT_NDIR):
    """Fibonacci directions: z = 1 - (2k+1)/n, phi = k pi (3 - sqrt 5)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def _fit_lib():
    L = lib()
    if not hasattr(L, "_fit_ready"):
        L.vxo_fit_eval.restype = ctypes.c_double
        L.vxo_fit_eval.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vxo_voxelize_fibers_pairs.restype = ctypes.c_void_p
        L.vxo_voxelize_fibers_pairs.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int)]
        L.vxo_pairs_size.restype = ctypes.c_int64
        L.vxo_pairs_size.argtypes = [ctypes.c_void_p]
        L.vxo_pairs_copy.argtypes = [ctypes.c_void_p] * 3
        L.vxo_pairs_free.argtypes = [ctypes.c_void_p]
        L.vxo_fit_levels.restype = ctypes.c_int
        L.vxo_fit_levels.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_int]
        L._fit_ready = True
    return L


def fit_levels(grid, pts, offsets, radius, hi, nthreads=None):
    """Voxel counts of levels 0..hi of the fibers' pyramid."""
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float32).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n = np.zeros(hi + 1, dtype=np.int64)
    bmin, ext, l2 = _grid_args(grid)
    st = _fit_lib().vxo_fit_levels(bmin, ext, l2, _ptr(p), p.shape[0], _ptr(o), o.shape[0] - 1,
                                   float(np.float32(radius)), int(hi), _ptr(n), _nthreads(nthreads))
    if st:
        raise OracleError(f"fit_levels failed with status {st}")
    return n


def fit_eval(grid, pts_snap, pts_cont, offsets, radius, lo, hi, L_all, grad=True, nthreads=None, dirs=None):
    """Loss of the two-lobe fit at levels lo..hi and, with grad, d loss / d L and d loss / d points.

    pts_snap (float32) fixes which segment touches which voxel; pts_cont (float64) gives the
    weights and tangents.  L_all: float64 [sum of level sizes, 12], levels lo..hi in key order.
    dirs: the 128 directions [128, 3] (any float dtype, evaluated in FP64), or None for the
    Fibonacci set computed in FP64."""
    ps = np.ascontiguousarray(np.asarray(pts_snap, dtype=np.float32).reshape(-1, 3))
    pc = np.ascontiguousarray(np.asarray(pts_cont, dtype=np.float64).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    La = np.ascontiguousarray(np.asarray(L_all, dtype=np.float64).reshape(-1, 12))
    lv = np.zeros(La.shape[0])
    dd = None
    if dirs is not None:
        dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        if dd.shape[0] != 128:
            raise OracleError("fit_eval: the direction set has 128 directions")
    dL = np.zeros_like(La) if grad else None
    dp = np.zeros_like(pc) if grad else None
    st = ctypes.c_int(0)
    bmin, ext, l2 = _grid_args(grid)
    loss = _fit_lib().vxo_fit_eval(bmin, ext, l2, _ptr(ps), _ptr(pc), ps.shape[0], _ptr(o), o.shape[0] - 1,
                                   float(np.float32(radius)), int(lo), int(hi), _ptr(La), _ptr(lv),
                                   _ptr(dL) if grad else None, _ptr(dp) if grad else None,
                                   _ptr(dd) if dd is not None else None, _nthreads(nthreads),
                                   ctypes.byref(st))
    if st.value:
        raise OracleError(f"fit_eval failed with status {st.value}")
    return loss, lv, dL, dp


def fiber_pairs(grid, pts, offsets, radius, nthreads=None):
    """Every touching (segment, leaf voxel) pair: Morton keys and segment ids (first point)."""
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float32).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    st = ctypes.c_int(0)
    bmin, ext, l2 = _grid_args(grid)
    L = _fit_lib()
    r = L.vxo_voxelize_fibers_pairs(bmin, ext, l2, _ptr(p), p.shape[0], _ptr(o), o.shape[0] - 1,
                                    float(np.float32(radius)), _nthreads(nthreads), ctypes.byref(st))
    if st.value:
        raise OracleError(f"fiber_pairs failed with status {st.value}")
    n = L.vxo_pairs_size(r)
    keys = np.zeros(n, np.uint64)
    prim = np.zeros(n, np.int64)
    L.vxo_pairs_copy(r, _ptr(keys), _ptr(prim))
    L.vxo_pairs_free(r)
    return keys, prim


def fit_conditioning(grid, pts, offsets, radius, hi):
    """Per control point: the least normalised projected area squared, min over directions of
    w^T (S / w) w, over every voxel whose sums feed a fitted target and that a segment of the
    point touches (the voxel itself and its ancestors up to level hi - 1).  The target's
    sqrt is ill-conditioned where this is small: its derivative scales as 1 / sqrt of it."""
    v = voxelize_fibers(grid, pts, offsets, radius)
    lod = build_lod(v, hi + 1)
    W = fit_dirs()
    mins = []
    for L in range(hi):
        lv = lod[L]
        m = lv.w > 0
        S = lv.S[m] / lv.w[m, None]
        q = (S[:, 0, None] * W[:, 0] ** 2 + S[:, 1, None] * W[:, 1] ** 2 + S[:, 2, None] * W[:, 2] ** 2
             + 2 * (S[:, 3, None] * W[:, 0] * W[:, 1] + S[:, 4, None] * W[:, 0] * W[:, 2]
                    + S[:, 5, None] * W[:, 1] * W[:, 2]))
        out = np.full(len(lv.w), np.inf)
        out[m] = q.min(1)
        mins.append(out)
    leafk = lod[0].keys
    cond_leaf = np.full(len(leafk), np.inf)
    for L in range(hi):
        idx = np.searchsorted(lod[L].keys, leafk >> np.uint64(3 * L))
        cond_leaf = np.minimum(cond_leaf, mins[L][idx])
    pk, pp = fiber_pairs(grid, pts, offsets, radius)
    vi = np.searchsorted(leafk, pk)
    cond = np.full(len(np.asarray(pts).reshape(-1, 3)), np.inf)
    np.minimum.at(cond, pp, cond_leaf[vi])
    np.minimum.at(cond, pp + 1, cond_leaf[vi])
    return cond

# ------------------------------------------------------------------------------------------------
# the paper's sampling voxelizer (Sec. 3.2)
# ------------------------------------------------------------------------------------------------

def _sample_lib():
    L = lib()
    if not hasattr(L, "_sample_ready"):
        L.vxo_sample_fibers.restype = ctypes.c_void_p
        L.vxo_sample_fibers.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]
        L.vxo_sample_triangles.restype = ctypes.c_void_p
        L.vxo_sample_triangles.argtypes = [_c_dp, ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.vxo_sresult_size.restype = ctypes.c_int64
        L.vxo_sresult_size.argtypes = [ctypes.c_void_p]
        L.vxo_sresult_nsamples.restype = ctypes.c_int64
        L.vxo_sresult_nsamples.argtypes = [ctypes.c_void_p]
        L.vxo_sresult_copy.argtypes = [ctypes.c_void_p] * 5
        L.vxo_sresult_free.argtypes = [ctypes.c_void_p]
        L.vxo_heitz_map.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.vxo_tri_sample_count.restype = ctypes.c_int64
        L.vxo_tri_sample_count.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L._sample_ready = True
    return L


def _take_samples(res) -> Voxels:
    L = _sample_lib()
    n = L.vxo_sresult_size(res)
    v = Voxels(np.empty(n, np.uint64), np.empty(n, np.uint32), np.empty(n, np.float64),
               np.empty((n, 6), np.float64), int(L.vxo_sresult_nsamples(res)))
    L.vxo_sresult_copy(res, _ptr(v.keys), _ptr(v.count), _ptr(v.w), _ptr(v.S))
    L.vxo_sresult_free(res)
    return v


def sample_fibers(grid, pts, offsets, sub, per) -> Voxels:
    """Sampling voxelizer for fibers (Sec. 3.2): per segment the Catmull-Rom span cut into `sub`
    chords, `per` samples per chord; count = samples per voxel, w = summed chord length / per,
    S = sum w (I - t t^T).  n_pairs holds the number of samples inside the grid."""
    p = np.ascontiguousarray(np.asarray(pts, dtype=np.float32).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    bmin, ext, l2 = _grid_args(grid)
    st = ctypes.c_int(0)
    res = _sample_lib().vxo_sample_fibers(bmin, ext, l2, _ptr(p), p.shape[0], _ptr(o), o.shape[0] - 1, int(sub),
                                          int(per), ctypes.byref(st))
    if st.value:
        raise OracleError(f"sample_fibers failed with status {st.value}")
    return _take_samples(res)


def sample_triangles(grid, tris, max_samples) -> Voxels:
    """Sampling voxelizer for triangles (Sec. 3.2): Heitz's triangle map of stratified points,
    max(1, floor(N A / A_max)) samples per triangle; w = summed A / n_T, S = sum w n n^T."""
    t = np.ascontiguousarray(np.asarray(tris, dtype=np.float32).reshape(-1, 3, 3))
    bmin, ext, l2 = _grid_args(grid)
    st = ctypes.c_int(0)
    res = _sample_lib().vxo_sample_triangles(bmin, ext, l2, _ptr(t), t.shape[0], int(max_samples),
                                             ctypes.byref(st))
    if st.value:
        raise OracleError(f"sample_triangles failed with status {st.value}")
    return _take_samples(res)


def heitz_map(u1, u2):
    b = np.zeros(2)
    _sample_lib().vxo_heitz_map(float(u1), float(u2), _ptr(b))
    return b


def tri_sample_count(q, qmax, N) -> int:
    return int(_sample_lib().vxo_tri_sample_count(float(q), float(qmax), int(N)))


# ------------------------------------------------------------------------------------------------
# the paper's SGGX-H lobe reduction (Sec. 4.4)
# ------------------------------------------------------------------------------------------------

SGGXH_SAMPLES = 5000


def _sggxh_lib():
    L = lib()
    if not hasattr(L, "_sggxh_ready"):
        u64 = ctypes.c_uint64
        L.vxo_splitmix_at.restype = u64
        L.vxo_splitmix_at.argtypes = [u64, u64]
        L.vxo_sggxh_lobe_key.restype = u64
        L.vxo_sggxh_lobe_key.argtypes = [ctypes.c_int, u64, ctypes.c_int]
        L.vxo_sggxh_hist.argtypes = [ctypes.c_void_p, ctypes.c_double, u64, ctypes.c_int, ctypes.c_void_p]
        L.vxo_sggxh_samples.restype = ctypes.c_int
        L.vxo_sggxh_samples.argtypes = [ctypes.c_void_p, ctypes.c_double, u64, ctypes.c_int, ctypes.c_void_p]
        L.vxo_sggxh_reduce.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vxo_sggxh_level.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L._sggxh_ready = True
    return L


def splitmix_at(key, c) -> int:
    """SplitMix64 output number c of seed key."""
    return int(_sggxh_lib().vxo_splitmix_at(int(key) & (2**64 - 1), int(c)))


def sggxh_lobe_key(level, voxel_key, slot) -> int:
    return int(_sggxh_lib().vxo_sggxh_lobe_key(int(level), int(voxel_key), int(slot)))


def sggxh_hist(S, w, key, N=SGGXH_SAMPLES) -> np.ndarray:
    """Counts [5, 5, 5] (bins of x, y, z) of N normals sampled from the lobe (w, S)."""
    S6 = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(6))
    h = np.zeros(125, np.int32)
    _sggxh_lib().vxo_sggxh_hist(_ptr(S6), float(w), int(key), int(N), _ptr(h))
    return h.reshape(5, 5, 5)


def sggxh_samples(S, w, key, N=SGGXH_SAMPLES) -> np.ndarray:
    """The unit normals [N, 3] drawn for the lobe (w, S), in sample order."""
    S6 = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(6))
    out = np.zeros((int(N), 3))
    m = _sggxh_lib().vxo_sggxh_samples(_ptr(S6), float(w), int(key), int(N), _ptr(out))
    return out[:m]


def sggxh_reduce(w, S, counts, K):
    """Merge lobes with the given histograms down to K: (nl, w [K], S [K, 6], out_of [n])."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = len(w)
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(n, 6))
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.int32).reshape(n, 125))
    nl = ctypes.c_int(0)
    ow, oS, of = np.zeros(max(K, 1)), np.zeros((max(K, 1), 6)), np.zeros(n, np.int32)
    _sggxh_lib().vxo_sggxh_reduce(n, _ptr(w), _ptr(S), _ptr(c), int(K), ctypes.byref(nl), _ptr(ow), _ptr(oS),
                                  _ptr(of))
    return nl.value, ow[:nl.value], oS[:nl.value], of


def sggxh_level(child: Lobes, child_start, parent_keys, level: int, K: int, N=SGGXH_SAMPLES) -> Lobes:
    n_par = len(child_start) - 1
    Kc = child.w.shape[1]
    out = Lobes(np.zeros(n_par, np.int32), np.zeros((n_par, K)), np.zeros((n_par, K, 6)),
                np.zeros(n_par), np.zeros(n_par))
    pk = np.ascontiguousarray(parent_keys, dtype=np.uint64)
    cs = np.ascontiguousarray(child_start, dtype=np.int64)
    cnl = np.ascontiguousarray(child.nl, dtype=np.int32)
    cw = np.ascontiguousarray(child.w, dtype=np.float64)
    cS = np.ascontiguousarray(child.S, dtype=np.float64)
    _sggxh_lib().vxo_sggxh_level(n_par, _ptr(pk), _ptr(cs), _ptr(cnl), _ptr(cw), _ptr(cS), Kc, int(level), int(K),
                                 int(N), _ptr(out.nl), _ptr(out.w), _ptr(out.S))
    return out


def sggxh_pyramid(lod, K: int, N=SGGXH_SAMPLES):
    """SGGX-H lobes of levels 1 .. len(lod)-1 (index 0 holds the leaf as one lobe per voxel)."""
    leaf = lod[0]
    n0 = len(leaf.keys)
    cur = Lobes((leaf.w > 0).astype(np.int32), leaf.w.reshape(n0, 1).copy(), leaf.S.reshape(n0, 1, 6).copy(),
                np.zeros(n0), np.zeros(n0))
    out = [cur]
    for L in range(1, len(lod)):
        cur = sggxh_level(cur, lod[L].child_start, lod[L].keys, L, K, N)
        out.append(cur)
    return out
