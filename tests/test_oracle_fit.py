"""Pins of the differentiable lobe fit oracle (FP64): central finite differences of the loss,
closed-form zero-loss case, and the clipped-length gradient away from clip-plane kinks."""
import numpy as np
import pytest

import oracle
import synth


def _lattice_points(grid, pts):
    """Points moved onto the snapping lattice (exact in float32), so snapped = continuous."""
    q = oracle.snap(grid, pts).astype(np.float64)
    return (np.asarray(grid.bmin) + q * (grid.extent / 2.0 ** 23)).astype(np.float32)


def _init_L(grid, pts, offsets, radius, lo, hi, seed):
    """0.5 chol(S/w + 0.05 I) + N(0, 0.01) per voxel and lobe, from the oracle's own pyramid."""
    rng = np.random.default_rng(seed)
    v = oracle.voxelize_fibers(grid, pts, offsets, radius)
    lod = oracle.build_lod(v, hi + 1)
    out = []
    for L in range(lo, hi + 1):
        lv = lod[L]
        for i in range(len(lv.keys)):
            if lv.w[i] > 0:
                S = lv.S[i] / lv.w[i]
                M = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]]) + 0.05 * np.eye(3)
                C = 0.5 * np.linalg.cholesky(M)
            else:
                C = np.zeros((3, 3))
            row = []
            for j in range(2):
                row += [C[0, 0], C[1, 0], C[1, 1], C[2, 0], C[2, 1], C[2, 2]]
            out.append(np.array(row) + rng.normal(0, 0.01, 12))
    return np.array(out)


def _small_fabric():
    wl = synth.plain_weave(n_fibers=16, n_points=33, res=128, seed=41)
    pts = _lattice_points(wl.grid, wl.pts)
    return wl, pts


def _lb_state(A, B, lo):
    """Which constraints fix the clipped interval of segment A-B in [lo, lo+1)^3 (kink detector)."""
    d = B - A
    t0, t1, e0, e1 = 0.0, 1.0, -1, -1
    for a in range(3):
        if d[a] == 0:
            if not (lo[a] <= A[a] < lo[a] + 1):
                return ("empty",)
            continue
        ta, tb = (lo[a] - A[a]) / d[a], (lo[a] + 1 - A[a]) / d[a]
        tin, tout = min(ta, tb), max(ta, tb)
        if tin > t0:
            t0, e0 = tin, a
        if tout < t1:
            t1, e1 = tout, a
    return ("empty",) if t1 <= t0 else (e0, e1)


def _crosses(pts_c, i, offsets, grid, delta):
    """Does moving point i by +-delta change the clipping structure of one of its segments?"""
    vs = grid.res / grid.extent
    segs = [j for j in (i - 1, i) if j >= 0 and j + 1 < len(pts_c)
            and np.searchsorted(offsets, j, "right") == np.searchsorted(offsets, j + 1, "right")]
    for j in segs:
        states = []
        for sgn in (0.0, 1.0, -1.0):
            P = pts_c.copy()
            P[i] += sgn * delta
            A, B = P[j] * vs, P[j + 1] * vs
            lo = np.floor(np.minimum(A, B)) - 1
            hi = np.floor(np.maximum(A, B)) + 1
            st = {}
            for x in range(int(lo[0]), int(hi[0]) + 1):
                for y in range(int(lo[1]), int(hi[1]) + 1):
                    for z in range(int(lo[2]), int(hi[2]) + 1):
                        st[(x, y, z)] = _lb_state(A, B, np.array([x, y, z], float))
            states.append(st)
        if states[0] != states[1] or states[0] != states[2]:
            return True
    return False


def test_fit_gradient_matches_central_differences():
    wl, pts = _small_fabric()
    lo, hi = 1, 5
    L0 = _init_L(wl.grid, pts, wl.offsets, wl.radius, lo, hi, 4)
    pc = pts.astype(np.float64)
    loss, lv, dL, dp = oracle.fit_eval(wl.grid, pts, pc, wl.offsets, wl.radius, lo, hi, L0)
    assert loss > 0 and np.isfinite(dp).all() and np.abs(dp).max() > 0
    h = 1e-3
    rng = np.random.default_rng(42)
    fd, an, kinks = [], [], 0
    tried = 0
    while len(fd) < 40 and tried < 400:
        tried += 1
        i = int(rng.integers(0, len(pts)))
        a = int(rng.integers(0, 3))
        delta = np.zeros(3)
        delta[a] = h
        if _crosses(pc, i, wl.offsets, wl.grid, delta):
            kinks += 1
            continue
        def cd(step):
            P1, P2 = pc.copy(), pc.copy()
            P1[i, a] += step
            P2[i, a] -= step
            _, l1, _, _ = oracle.fit_eval(wl.grid, pts, P1, wl.offsets, wl.radius, lo, hi, L0, grad=False)
            _, l2, _, _ = oracle.fit_eval(wl.grid, pts, P2, wl.offsets, wl.radius, lo, hi, L0, grad=False)
            return (l1 - l2).sum() / (2 * step)      # per-voxel differences: no cancellation
        # central differences at h and h/2, Richardson-extrapolated (the h^2 term cancels)
        fd.append((4.0 * cd(h / 2) - cd(h)) / 3.0)
        an.append(dp[i, a])
    fd, an = np.array(fd), np.array(an)
    assert len(fd) >= 30, (len(fd), kinks)
    assert np.linalg.norm(fd - an) <= 1e-5 * np.linalg.norm(an), (np.abs(fd - an).max(), np.linalg.norm(an))
    # lobe parameters: smooth wherever no lobe has L^T w = 0
    live = np.flatnonzero(np.abs(dL).sum(1) > 0)
    for r, c in [(int(r), c) for r in rng.choice(live, 4, replace=False) for c in range(12)]:
        L1, L2 = L0.copy(), L0.copy()
        L1[r, c] += 1e-5
        L2[r, c] -= 1e-5
        _, a1, _, _ = oracle.fit_eval(wl.grid, pts, pc, wl.offsets, wl.radius, lo, hi, L1, grad=False)
        _, a2, _, _ = oracle.fit_eval(wl.grid, pts, pc, wl.offsets, wl.radius, lo, hi, L2, grad=False)
        g = (a1 - a2).sum() / 2e-5
        assert abs(g - dL[r, c]) <= 1e-6 * max(1.0, abs(dL[r, c])), (r, c, g, dL[r, c])


def test_fit_zero_loss_at_exact_single_child_lobe():
    """One straight fiber inside one level-1 parent's single child: L1 L1^T = S/w, L2 = 0 gives
    f = tau in every direction, so the loss and the lobe gradient vanish."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    pts = np.array([[2.25, 2.5, 2.375], [2.75, 2.625, 2.5]], dtype=np.float32)   # inside voxel (2, 2, 2)
    off = np.array([0, 2])
    v = oracle.voxelize_fibers(grid, pts, off, 0.0)
    lod = oracle.build_lod(v, 2)
    n1 = oracle.fit_levels(grid, pts, off, 0.0, 1)
    assert n1[1] == 1
    S = lod[1].S[0] / lod[1].w[0]
    M = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])
    ev, evec = np.linalg.eigh(M)
    # a lower-triangular factor of the PSD (rank-2) matrix through its LDL^T / QR of a root
    R = evec @ np.diag(np.sqrt(np.maximum(ev, 0)))
    q, r = np.linalg.qr(R.T)
    Lf = r.T                                            # M = R R^T = r^T r, r^T lower triangular
    row = [Lf[0, 0], Lf[1, 0], Lf[1, 1], Lf[2, 0], Lf[2, 1], Lf[2, 2]] + [0.0] * 6
    loss, lv, dL, dp = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, np.array([row]))
    assert loss < 1e-24 and np.abs(dL).max() < 1e-12


def test_fit_directions_cover_the_sphere_evenly():
    W = oracle.fit_dirs()
    assert W.shape == (128, 3) and np.allclose(np.linalg.norm(W, axis=1), 1.0)
    assert np.allclose(W.T @ W / 128, np.eye(3) / 3, atol=2e-3)


def test_fit_target_over_several_children_by_hand():
    """Three children of one level-1 voxel, worked by hand: two x-directed fiber pieces of length
    3/4 (voxels (2,2,2) and (3,2,2), normalised SGGX diag(0, 1, 1)) and one y-directed piece of
    length 1/2 (voxel (2,3,2), diag(1, 0, 1)).  The target is the density-weighted mean of the
    children's projected areas, tau(w) = (3/4 sqrt(1 - wx^2) + 3/4 sqrt(1 - wx^2)
    + 1/2 sqrt(1 - wy^2)) / 2, and with both lobes zero the loss is the mean of tau^2 over the
    direction set.  An unweighted mean over the children, a division by the child count, or the
    square root of the summed moments all give other values."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    pts = np.array([[2.25, 2.5, 2.5], [3.75, 2.5, 2.5],      # x-directed, crosses x = 3
                    [2.5, 3.25, 2.5], [2.5, 3.75, 2.5]],     # y-directed, inside voxel (2, 3, 2)
                   dtype=np.float32)
    off = np.array([0, 2, 4])
    v = oracle.voxelize_fibers(grid, pts, off, 0.0)
    assert [tuple(c) for c in oracle.demorton(v.keys, 3)] == [(2, 2, 2), (3, 2, 2), (2, 3, 2)]
    assert np.allclose(v.w, [0.75, 0.75, 0.5], rtol=0, atol=1e-15)
    n = oracle.fit_levels(grid, pts, off, 0.0, 1)
    assert list(n) == [3, 1]
    W = oracle.fit_dirs()
    tau = (0.75 * np.sqrt(1 - W[:, 0] ** 2) * 2 + 0.5 * np.sqrt(1 - W[:, 1] ** 2)) / 2.0
    want = np.mean(tau ** 2)
    loss, lv, dL, _ = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, np.zeros((1, 12)))
    assert abs(loss - want) <= 1e-12 * want and abs(lv[0] - want) <= 1e-12 * want
    # the plausible misreadings, for the record: each differs from the target by far more
    unweighted = np.mean(((np.sqrt(1 - W[:, 0] ** 2) * 2 + np.sqrt(1 - W[:, 1] ** 2)) / 3.0) ** 2)
    summed = np.mean((np.sqrt(1.5 * (1 - W[:, 0] ** 2) + 0.5 * (1 - W[:, 1] ** 2)) / 2.0) ** 2)
    per_child = np.mean(((0.75 * np.sqrt(1 - W[:, 0] ** 2) * 2 + 0.5 * np.sqrt(1 - W[:, 1] ** 2)) / 3.0) ** 2)
    for other in (unweighted, summed, per_child):
        assert abs(other - want) > 1e-3 * want
    # with a single lobe L1 = diag(a, a, a) the fit is a |w| = a everywhere: loss = mean((a - tau)^2)
    a = 0.4
    row = np.array([[a, 0, a, 0, 0, a] + [0.0] * 6])
    loss2, _, dL2, _ = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, row)
    assert abs(loss2 - np.mean((a - tau) ** 2)) <= 1e-12 * loss2
    # d loss / d L00 = mean(2 (a - tau) * d|L^T w| / d L00) with |L^T w| = a |w|: y0 = a wx, so
    # d/dL00 of |y| = y0 wx / |y| = wx^2
    g00 = np.mean(2 * (a - tau) * W[:, 0] ** 2)
    assert abs(dL2[0, 0] - g00) <= 1e-12 * max(1.0, abs(g00))


def test_fit_given_direction_set_by_hand():
    """The direction set is an input: with 128 random unit directions (float32 values) the loss
    of the three-children case above is the mean of tau^2 over those directions, and the
    default set equals the float32-rounded Fibonacci set up to that rounding."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    pts = np.array([[2.25, 2.5, 2.5], [3.75, 2.5, 2.5], [2.5, 3.25, 2.5], [2.5, 3.75, 2.5]], dtype=np.float32)
    off = np.array([0, 2, 4])
    rng = np.random.default_rng(5)
    D = rng.normal(size=(128, 3))
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    Dd = D.astype(np.float64)
    n2 = (Dd ** 2).sum(1)                      # float32 directions are unit length only to ~1e-8
    tau = (0.75 * np.sqrt(n2 - Dd[:, 0] ** 2) * 2 + 0.5 * np.sqrt(n2 - Dd[:, 1] ** 2)) / 2.0
    loss, _, _, _ = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, np.zeros((1, 12)), dirs=D)
    want = np.mean(tau ** 2)
    assert abs(loss - want) <= 1e-12 * want
    F = synth.fibonacci_dirs(128)
    assert np.abs(F.astype(np.float64) - oracle.fit_dirs()).max() < 1e-7
    l_def = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, np.zeros((1, 12)))[0]
    l_f32 = oracle.fit_eval(grid, pts, pts.astype(np.float64), off, 0.0, 1, 1, np.zeros((1, 12)), dirs=F)[0]
    assert l_def != l_f32 and abs(l_def - l_f32) <= 1e-6 * l_def


def test_fit_gradient_of_axis_parallel_segments():
    """Segments with a coordinate held fixed (d_x = 0 or d_z = 0) whose capsule also touches the
    neighbouring column with no centreline inside it (weight 0): such touches carry no gradient.
    Central differences of the loss in every coordinate of every point, none near a clip kink."""
    grid = synth.Grid((0.0, 0.0, 0.0), 8.0, 3)
    pts = np.array([[1.3, 1.2, 3.4], [2.75, 1.9, 3.6],       # generic
                    [2.75, 4.3, 4.1],                        # d_x = 0 at x = 2.75: touches column x = 3
                    [2.75, 6.6, 3.45],                       # d_x = 0 again
                    [4.2, 5.1, 3.45], [5.6, 3.3, 3.45],      # d_z = 0 at z = 3.45: touches layer z = 4
                    [1.6, 6.2, 5.3], [2.3, 4.4, 6.2], [3.7, 2.2, 5.9]], dtype=np.float32)
    pts = _lattice_points(grid, pts)
    off = np.array([0, 6, 9])
    lo, hi = 1, 2
    L0 = _init_L(grid, pts, off, 0.5, lo, hi, 7)
    pc = pts.astype(np.float64)
    _, _, _, dp = oracle.fit_eval(grid, pts, pc, off, 0.5, lo, hi, L0)
    fd = np.zeros_like(dp)
    checked = 0
    for i in range(len(pts)):
        for a in range(3):
            delta = np.zeros(3)
            delta[a] = 1e-3
            if _crosses(pc, i, off, grid, delta):
                fd[i, a] = dp[i, a]
                continue
            def cd(step):
                P1, P2 = pc.copy(), pc.copy()
                P1[i, a] += step
                P2[i, a] -= step
                l1 = oracle.fit_eval(grid, pts, P1, off, 0.5, lo, hi, L0, grad=False)[1]
                l2 = oracle.fit_eval(grid, pts, P2, off, 0.5, lo, hi, L0, grad=False)[1]
                return (l1 - l2).sum() / (2 * step)
            fd[i, a] = (4.0 * cd(5e-4) - cd(1e-3)) / 3.0
            checked += 1
    assert checked >= 20
    assert np.abs(dp).max() > 0
    assert np.abs(fd - dp).max() <= 1e-6 * np.abs(dp).max(), np.abs(fd - dp).max(axis=1)
