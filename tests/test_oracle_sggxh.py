"""Pins of the SGGX-H oracle (Sec. 4.4: lobes compared through histograms of their samples under a
Wasserstein distance, the closest pair merged by pooling samples until the lobe cap).

* the random numbers: SplitMix64's published output sequence for seed 1234567;
* the sampled normals: area-weighted normals of the ellipsoid x^T S x = 1, checked through the
  projected-area identity E|v . n| = c sqrt(v^T S v) (the same c for every direction v), the
  sphere's uniform marginals for an isotropic lobe and the great circle of a fiber lobe;
* the distance and the merges: hand-worked histograms, and an exact-rational brute force of the
  greedy merging on random small histograms;
* the level: lobes at or under the cap kept, zero weights dropped, sums conserved, and lobes of
  two clearly different families separated the same way the moment metric separates them.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_splitmix64_published_sequence():
    # the reference SplitMix64 (Steele, Lea, Flood 2014) seeded with 1234567 outputs these first
    assert [oracle.splitmix_at(1234567, i) for i in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]


def _reg(S6):
    S = np.array([[S6[0], S6[3], S6[4]], [S6[3], S6[1], S6[5]], [S6[4], S6[5], S6[2]]], float)
    return S + 1e-3 * np.trace(S) * np.eye(3)


@pytest.mark.parametrize("S6", [[2.0, 1.0, 0.5, 0.3, 0.1, -0.2], [1.0, 1.0, 0.0, 0.0, 0.0, 0.0],
                                [0.05, 0.02, 1.0, 0.01, 0.0, 0.03], [1.0, 0.2, 0.2, 0.0, 0.0, 0.0]])
def test_normals_follow_the_projected_area(S6):
    """For area-uniform points of the ellipsoid x^T S x = 1, the mean of |v . n| over normals is
    proportional to the ellipsoid's projected area along v, sqrt(v^T S v)."""
    n = oracle.sggxh_samples(S6, 1.0, 17, 120000)
    assert len(n) == 120000 and np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
    S = _reg(S6)
    rng = np.random.default_rng(1)
    V = rng.normal(size=(12, 3))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    ratio = np.abs(n @ V.T).mean(0) / np.sqrt(np.einsum("ij,jk,ik->i", V, S, V))
    assert ratio.std() / ratio.mean() < 0.01, ratio


def test_isotropic_and_fiber_histograms():
    h = oracle.sggxh_hist([1, 1, 1, 0, 0, 0], 1.0, 3, 5000)
    assert h.sum() == 5000
    for m in (h.sum((1, 2)), h.sum((0, 2)), h.sum((0, 1))):    # Archimedes: each axis uniform
        assert np.all(np.abs(m - 1000) < 4 * np.sqrt(1000 * 0.8)), m
    h = oracle.sggxh_hist([1, 1, 0, 0, 0, 0], 1.0, 3, 5000)     # fiber along z: normals on z = 0
    assert h.sum((0, 1))[2] >= 4900
    mx = h.sum((1, 2))                                          # cos of a uniform angle: arcsine
    assert mx[0] > mx[2] and mx[4] > mx[2]
    # the weight does not matter, only S / w
    assert np.array_equal(oracle.sggxh_hist([2, 2, 0, 0, 0, 0], 2.0, 3, 500),
                          oracle.sggxh_hist([1, 1, 0, 0, 0, 0], 1.0, 3, 500))


def _onebin(x, y, z, n):
    h = np.zeros((5, 5, 5), np.int32)
    h[x, y, z] = n
    return h


def test_distance_and_merges_by_hand():
    """A and C in bin (0, 2, 2), B in (4, 2, 2): W(A, C) = 0 merges first; W(A, B) moves all mass
    four bins of 0.4 along x: 1.6; with the pooled A+C against B also 1.6."""
    N = 10
    counts = [_onebin(0, 2, 2, N), _onebin(4, 2, 2, N), _onebin(0, 2, 2, N)]
    S = np.eye(3)[[0, 1, 2]].repeat(2, axis=1)[:, :6]
    w = np.array([1.0, 2.0, 3.0])
    nl, ow, oS, of = oracle.sggxh_reduce(w, S, counts, 2)
    assert nl == 2 and list(of) == [0, 1, 0] and np.allclose(ow, [4.0, 2.0])
    assert np.allclose(oS[0], S[0] + S[2]) and np.allclose(oS[1], S[1])
    nl, ow, oS, of = oracle.sggxh_reduce(w, S, counts, 1)
    assert nl == 1 and list(of) == [0, 0, 0] and np.allclose(ow, [6.0]) and np.allclose(oS[0], S.sum(0))
    # ties: three identical histograms merge (0, 1) first
    nl, ow, _, of = oracle.sggxh_reduce(np.array([1.0, 1.5, 2.0]), S, [_onebin(1, 1, 1, N)] * 3, 2)
    assert list(of) == [0, 0, 1] and ow.tolist() == [2.5, 2.0]


def _W(a, b):
    """Exact Wasserstein-1 of the axis marginals, bin width 2/5, for pooled count histograms."""
    ha, ma = a
    hb, mb = b
    tot = Fraction(0)
    for ax in range(3):
        ca = np.cumsum(ha.sum(axis=tuple(i for i in range(3) if i != ax)))[:4]
        cb = np.cumsum(hb.sum(axis=tuple(i for i in range(3) if i != ax)))[:4]
        for x, y in zip(ca, cb):
            tot += abs(Fraction(int(x), ma) - Fraction(int(y), mb))
    return tot * Fraction(2, 5)


@pytest.mark.parametrize("seed", range(6))
def test_merges_match_exact_rational_brute_force(seed):
    rng = np.random.default_rng(seed)
    n, K = int(rng.integers(5, 10)), int(rng.integers(1, 4))
    counts = []
    for _ in range(n):
        h = np.zeros(125, np.int64)
        np.add.at(h, rng.integers(0, 125 if seed % 2 else 20, size=12), 1)   # 12 samples each
        counts.append(h.reshape(5, 5, 5))
    w = rng.uniform(0.5, 2.0, n)
    S = rng.uniform(0, 1, (n, 6))
    nl, ow, oS, of = oracle.sggxh_reduce(w, S, counts, K)
    groups = [[i] for i in range(n)]
    hist = [(c.copy(), 12) for c in counts]
    while len(groups) > K:
        best = None
        for i in range(len(groups)):
            for j in range(i + 1, len(groups)):
                d = _W(hist[i], hist[j])
                if best is None or d < best[0]:
                    best = (d, i, j)
        _, i, j = best
        groups[i] += groups[j]
        hist[i] = (hist[i][0] + hist[j][0], hist[i][1] + hist[j][1])
        del groups[j], hist[j]
    want = sorted(groups, key=lambda g: -sum(w[g]))
    assert nl == len(want)
    for o, g in enumerate(want):
        assert sorted(np.flatnonzero(of == o).tolist()) == sorted(g)
        assert np.isclose(ow[o], w[g].sum()) and np.allclose(oS[o], S[g].sum(0))


def test_same_lobe_close_and_different_lobes_far():
    N = 5000
    a = oracle.sggxh_hist([1, 1, 0, 0, 0, 0], 1.0, 11, N)
    b = oracle.sggxh_hist([1, 1, 0, 0, 0, 0], 1.0, 12, N)      # same lobe, other stream
    c = oracle.sggxh_hist([0, 1, 1, 0, 0, 0], 1.0, 13, N)      # fiber along x
    assert _W((a, N), (b, N)) < Fraction(1, 20)
    assert _W((a, N), (c, N)) > 10 * _W((a, N), (b, N))


def test_level_keeps_caps_drops_zero_weights_and_conserves():
    """Three parents: 3 lobes (cap 4, kept and sorted), 6 lobes including a zero weight
    (reduced to 4), and only zero weights (none)."""
    rng = np.random.default_rng(5)
    Kc = 2
    nl = np.array([2, 1, 2, 2, 2, 1], np.int32)
    w = rng.uniform(0.5, 2.0, (6, Kc))
    w[3, 1] = 0.0
    w[5, 0] = 0.0
    nl[5] = 1
    S = rng.uniform(0.0, 1.0, (6, Kc, 6))
    S[:, :, 3:] *= 0.1
    S[3, 1] = 0.0                  # a lobe of zero weight has no moment either
    child = oracle.Lobes(nl, w, S, np.zeros(6), np.zeros(6))
    cs = np.array([0, 2, 5, 6])
    out = oracle.sggxh_level(child, cs, np.array([7, 8, 9], np.uint64), 1, 4, 400)
    assert list(out.nl) == [3, 4, 0]
    assert np.all(np.diff(out.w[0, :3]) <= 0) and np.all(np.diff(out.w[1]) <= 0)
    for p in range(2):
        ws = sum(w[c, k] for c in range(cs[p], cs[p + 1]) for k in range(nl[c]))
        Ss = sum(S[c, k] for c in range(cs[p], cs[p + 1]) for k in range(nl[c]))
        assert np.isclose(out.w[p].sum(), ws) and np.allclose(out.S[p].sum(0), Ss)


def test_two_families_split_like_the_moment_metric():
    """Eight fiber lobes, four near x and four near z: with K = 2 the histogram distance and the
    moment metric (Ward, no Lloyd) both split them by family."""
    rng = np.random.default_rng(2)
    S, w = [], []
    for t in [np.array([1, 0, 0])] * 4 + [np.array([0, 0, 1])] * 4:
        d = t + rng.normal(0, 0.05, 3)
        d /= np.linalg.norm(d)
        M = np.eye(3) - np.outer(d, d)
        S.append([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])
        w.append(rng.uniform(0.5, 1.5))
    S = np.array(S) * np.array(w)[:, None]
    w = np.array(w)
    order = rng.permutation(8)
    S, w = S[order], w[order]
    child = oracle.Lobes(np.ones(8, np.int32), w.reshape(8, 1), S.reshape(8, 1, 6), np.zeros(8), np.zeros(8))
    cs = np.array([0, 8])
    h = oracle.sggxh_level(child, cs, np.array([3], np.uint64), 1, 2, 2000)
    m = oracle.cluster_level(oracle.Lobes(child.nl, child.w, child.S, np.full(8, np.inf), np.full(8, np.inf),
                                          np.full(8, np.inf), np.full(8, np.inf)), cs, 2, 0)
    fam = np.array([0] * 4 + [1] * 4)[order]
    for out in (h, m):
        assert out.nl[0] == 2
        sums = sorted(out.w[0, :2].tolist())
        assert np.allclose(sums, sorted([w[fam == 0].sum(), w[fam == 1].sum()]))
