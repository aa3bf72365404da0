"""Comparison helpers for the GPU-vs-oracle parity tests.

Bar (per voxel): keys, counts and child masks bit-exact; for the float sums
    |w_gpu - w_ref|          <= TOL * max(w_ref, FLOOR)
    max_ij |S_gpu - S_ref|   <= TOL * max(tr S_ref, FLOOR)
with TOL = 1e-5 (FP32 accumulation against an FP64 reference) and FLOOR = 1e-2 (voxel^2 for
areas, voxel for lengths): the absolute accuracy FP32 can give sub-1e-2 slivers whose
measures come out of clipping in voxel-local coordinates.
"""
import numpy as np

TOL = 1e-5
FLOOR = 1e-2


def compare_level(g: dict, o_keys, o_count, o_w, o_S, o_mask=None, tol=TOL, floor=FLOOR, what=""):
    """g: dict from Voxels.numpy(); o_*: oracle arrays (FP64).  Returns a small report."""
    gk = g["keys"].astype(np.uint64)
    assert len(gk) == len(o_keys), f"{what}: {len(gk)} voxels vs oracle {len(o_keys)}"
    if not np.array_equal(gk, o_keys):
        bad = np.flatnonzero(gk != o_keys)[:5]
        raise AssertionError(f"{what}: keys differ at {bad.tolist()}: {gk[bad]} vs {o_keys[bad]}")
    assert np.array_equal(g["count"].astype(np.uint64), np.asarray(o_count).astype(np.uint64)), f"{what}: counts"
    if o_mask is not None:
        assert np.array_equal(g["mask"], o_mask), f"{what}: child masks"
    sw = np.maximum(np.abs(o_w), floor)
    tr = o_S[:, 0] + o_S[:, 1] + o_S[:, 2]
    sS = np.maximum(tr, floor)
    ew = np.abs(g["w"].astype(np.float64) - o_w) / sw
    eS = np.abs(g["S"].astype(np.float64) - o_S).max(axis=1) / sS if len(o_S) else np.zeros(0)
    rep = {"n": int(len(o_keys)), "max_rel_w": float(ew.max(initial=0)), "max_rel_S": float(eS.max(initial=0)),
           "at_floor": int(np.sum(tr < floor))}
    assert rep["max_rel_w"] <= tol and rep["max_rel_S"] <= tol, f"{what}: {rep}"
    return rep


def compare_pyramid(levels_gpu, lod_ref, what=""):
    reps = []
    for L, (g, o) in enumerate(zip(levels_gpu, lod_ref)):
        d = g.numpy()
        reps.append(compare_level(d, o.keys, o.count, o.w, o.S, o.mask if L > 0 else None, what=f"{what} L{L}"))
    return reps
