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


def _fib_dirs(n=64):
    k = np.arange(n)
    z = 1 - (2 * k + 1) / n
    phi = k * np.pi * (3 - np.sqrt(5))
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def _quad(S, W):
    """w^T S w for S [..., 6] and directions W [m, 3] -> [..., m]."""
    x, y, z = W[:, 0], W[:, 1], W[:, 2]
    return (S[..., 0, None] * x * x + S[..., 1, None] * y * y + S[..., 2, None] * z * z
            + 2 * (S[..., 3, None] * x * y + S[..., 4, None] * x * z + S[..., 5, None] * y * z))


def mixture_profile(w, S, W):
    """Projected area of the lobe mixture, sum_k w_k sqrt(w^T (S_k / w_k) w) = sum_k sqrt(w_k w^T S_k w)."""
    q = _quad(S, W) * w[..., None]
    return np.sqrt(np.maximum(q, 0)).sum(axis=-2)


DECIDED_REL = 1e-3     # a decision is clear when the runner-up is 0.1 % worse ...
DECIDED_ABS = 1e-6     # ... and the margin is above 1e-6 of the voxel's weight


def compare_lobes(g: dict, ref, lvl_w, lvl_S, K, tol=TOL, floor=FLOOR, prof_tol=1e-4, what=""):
    """g: Lobes.numpy() of one level; ref: oracle.Lobes of the same level; lvl_w / lvl_S: the
    oracle's one-lobe sums of the level (what every lobe set must add up to).
    Voxels whose every decision (in their whole subtree) had a clear margin must match the
    oracle lobe for lobe (after matching lobes by a min-cost assignment); the others -- where
    FP32 rounding may legitimately flip a near-tie -- are checked for the invariants and the
    mixture's projected-area profile."""
    from scipy.optimize import linear_sum_assignment
    n = len(ref.nl)
    assert len(g["nl"]) == n, what
    tr = lvl_S[:, 0] + lvl_S[:, 1] + lvl_S[:, 2]
    scale = np.maximum(tr, floor)
    gw, gS = g["w"].astype(np.float64), g["S"].astype(np.float64)
    # invariants for every voxel
    assert np.all(g["nl"] <= K), what
    assert np.all((g["nl"] > 0) == (lvl_w > 0)), what
    assert np.all(np.abs(gw.sum(1) - lvl_w) <= tol * np.maximum(lvl_w, floor)), what
    assert np.all(np.abs(gS.sum(1) - lvl_S).max(1) <= tol * scale), what
    kk = np.arange(K)[None, :]
    live = kk < g["nl"][:, None]
    assert np.all(gw[live] > 0) and np.all(gw[~live] == 0), what
    decided = (ref.tie_gap_rel >= DECIDED_REL) & (ref.tie_gap_abs >= DECIDED_ABS)
    n_exact = 0
    for i in np.flatnonzero(decided):
        assert g["nl"][i] == ref.nl[i], (what, i, g["nl"][i], ref.nl[i])
        m = ref.nl[i]
        if m == 0:
            continue
        cost = np.abs(gS[i, :m, None, :] - ref.S[i, None, :m, :]).max(-1) + \
            np.abs(gw[i, :m, None] - ref.w[i, None, :m])
        r, c = linear_sum_assignment(cost)
        err = max(np.abs(gw[i, r] - ref.w[i, c]).max(), np.abs(gS[i, r] - ref.S[i, c]).max())
        assert err <= tol * scale[i], (what, i, err, scale[i])
        n_exact += 1
    # near-tie voxels that nevertheless match lobe for lobe (reported, not required)
    n_tie_same = 0
    for i in np.flatnonzero(~decided):
        m = ref.nl[i]
        if m == 0 or g["nl"][i] != m:
            continue
        cost = np.abs(gS[i, :m, None, :] - ref.S[i, None, :m, :]).max(-1) + \
            np.abs(gw[i, :m, None] - ref.w[i, None, :m])
        r, c = linear_sum_assignment(cost)
        err = max(np.abs(gw[i, r] - ref.w[i, c]).max(), np.abs(gS[i, r] - ref.S[i, c]).max())
        n_tie_same += int(err <= tol * scale[i])
    W = _fib_dirs()
    pg = mixture_profile(gw, gS, W)
    po = mixture_profile(ref.w, ref.S, W)
    denom = np.maximum(po.max(1), floor)
    perr = np.abs(pg - po).max(1) / denom
    tie = ~decided & (ref.nl > 0)
    rep = {"n": int(n), "decided": int(decided.sum()), "checked_exactly": n_exact, "near_tie": int(tie.sum()),
           "near_tie_matching_exactly": n_tie_same,
           "near_tie_profile_err_max": float(perr[tie].max(initial=0)),
           "near_tie_profile_err_p99": float(np.percentile(perr[tie], 99)) if tie.any() else 0.0,
           "decided_profile_err_max": float(perr[decided].max(initial=0))}
    assert rep["near_tie_profile_err_max"] <= prof_tol, (what, rep)
    return rep


def compare_lobes_stepwise(g_lobes: dict, child, child_start, K, iters=2, tol=TOL, floor=FLOOR, what=""):
    """One level of the clustering checked on its own inputs: ``child`` holds the GPU's own lobes
    of the level below (as an oracle.Lobes in FP64; the leaf's single lobes at level 1), which
    the oracle clusters again.  Wherever this level's own decisions (Ward merges and Lloyd
    assignments of the voxel, not of its subtree) have a clear margin, the GPU's lobes must match
    the oracle's lobe for lobe; every voxel must keep the sums of its inputs, nl <= K and positive
    weights.  Returns a report with the number of voxels checked lobe for lobe."""
    import oracle
    from scipy.optimize import linear_sum_assignment
    n = len(child_start) - 1
    assert len(g_lobes["nl"]) == n, what
    c = oracle.Lobes(child.nl, child.w, child.S, child.gap_rel, child.gap_abs,
                     np.full(len(child.nl), np.inf), np.full(len(child.nl), np.inf))
    ref = oracle.cluster_level(c, child_start, K, iters)
    # what every parent's lobes must add up to: its children's lobes
    live_c = np.arange(child.w.shape[1])[None, :] < child.nl[:, None]
    cw = np.where(live_c, child.w, 0.0).sum(1)
    cS = np.where(live_c[:, :, None], child.S, 0.0).sum(1)
    starts = np.asarray(child_start[:-1])
    sum_w = np.add.reduceat(cw, starts) if n else np.zeros(0)
    sum_S = np.add.reduceat(cS, starts, axis=0) if n else np.zeros((0, 6))
    gw, gS = g_lobes["w"].astype(np.float64), g_lobes["S"].astype(np.float64)
    scale = np.maximum(sum_S[:, 0] + sum_S[:, 1] + sum_S[:, 2], floor)
    assert np.all(g_lobes["nl"] <= K), what
    assert np.all(np.abs(gw.sum(1) - sum_w) <= tol * np.maximum(sum_w, floor)), what
    assert np.all(np.abs(gS.sum(1) - sum_S).max(1) <= tol * scale), what
    kk = np.arange(K)[None, :]
    live = kk < g_lobes["nl"][:, None]
    assert np.all(gw[live] > 0) and np.all(gw[~live] == 0), what
    merged = ref.nl > 0
    # voxels with more input lobes than K take decisions; the others keep their inputs as they are
    n_in = np.add.reduceat(child.nl.astype(np.int64), starts) if n else np.zeros(0, np.int64)
    decided = (ref.gap_rel >= DECIDED_REL) & (ref.gap_abs >= DECIDED_ABS)
    n_exact, n_dec_merge = 0, 0
    for i in np.flatnonzero(decided & merged):
        assert g_lobes["nl"][i] == ref.nl[i], (what, i, g_lobes["nl"][i], ref.nl[i])
        m = ref.nl[i]
        cost = np.abs(gS[i, :m, None, :] - ref.S[i, None, :m, :]).max(-1) + np.abs(gw[i, :m, None] - ref.w[i, None, :m])
        r, cc = linear_sum_assignment(cost)
        err = max(np.abs(gw[i, r] - ref.w[i, cc]).max(), np.abs(gS[i, r] - ref.S[i, cc]).max())
        assert err <= tol * scale[i], (what, i, err, scale[i])
        n_exact += 1
        n_dec_merge += int(n_in[i] > K)
    return {"n": int(n), "merging": int(np.sum(n_in > K)), "checked_exactly": n_exact,
            "checked_exactly_merging": n_dec_merge, "near_tie": int(np.sum(~decided & merged))}


def gpu_lobes_as_oracle(g_lobes: dict):
    """A GPU level's lobes (Lobes.numpy()) as an oracle.Lobes in FP64 (margins unknown: +inf)."""
    import oracle
    n = len(g_lobes["nl"])
    inf = np.full(n, np.inf)
    return oracle.Lobes(g_lobes["nl"].astype(np.int32), g_lobes["w"].astype(np.float64),
                        g_lobes["S"].astype(np.float64), inf, inf.copy(), inf.copy(), inf.copy())


def leaf_as_oracle_lobes(g_leaf: dict):
    """A GPU leaf (Voxels.numpy()) as one lobe per voxel, present where w > 0."""
    import oracle
    n = len(g_leaf["w"])
    inf = np.full(n, np.inf)
    return oracle.Lobes((g_leaf["w"] > 0).astype(np.int32), g_leaf["w"].astype(np.float64).reshape(n, 1),
                        g_leaf["S"].astype(np.float64).reshape(n, 1, 6), inf, inf.copy(), inf.copy(), inf.copy())
