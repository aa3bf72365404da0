"""Pins of the eigen-fit and 6-byte SGGX code oracle (Sec. 4.1 fitting, Sec. 4.3 compact SGGX).

Every expected value here is a closed form worked out by hand or an invariant of the
mathematics (eigen-equation, orthonormality, quantisation bound), never the oracle's output.
"""
import math

import numpy as np
import pytest

from oracle import compact as oc

EPS = 1e-3


def _six(M):
    M = np.asarray(M, dtype=np.float64)
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])[:, None]


def _rot(ax, ang):
    c, s = math.cos(ang), math.sin(ang)
    if ax == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def test_diagonal_order_and_axes():
    w = np.array([2.0])
    lam, vec, Sfit = oc.eigen_fit(w, 2.0 * _six(np.diag([1.5, 0.5, 1.0])), EPS)
    assert np.allclose(lam[:, 0], [1.5, 1.0, 0.5], atol=1e-14)
    # eigenvector i is the axis of the i-th largest entry: x, z, y
    assert np.allclose(vec[:, :, 0], [[1, 0, 0], [0, 0, 1], [0, 1, 0]], atol=1e-14)
    assert np.allclose(Sfit[:, 0], [1.5, 0.5, 1.0, 0, 0, 0], atol=1e-14)


def test_known_rotation_recovers_frame():
    Q = _rot("x", math.radians(40.0)) @ _rot("z", math.radians(30.0))
    L = np.array([0.9, 0.4, 0.1])
    M = Q @ np.diag(L) @ Q.T
    w = np.array([3.0])
    lam, vec, Sfit = oc.eigen_fit(w, 3.0 * _six(M), EPS)
    assert np.allclose(lam[:, 0], L, atol=1e-13)
    for i in range(3):
        q = Q[:, i].copy()
        # sign rule: the component of largest magnitude is positive
        if q[np.argmax(np.abs(q))] < 0:
            q = -q
        assert np.allclose(vec[i, :, 0], q, atol=1e-12), i
    assert np.allclose(Sfit[:, 0], _six(M)[:, 0], atol=1e-13)


def test_single_fiber_floor():
    t = np.array([1.0, 2.0, 2.0]) / 3.0
    M = np.eye(3) - np.outer(t, t)          # SGGX of one fiber along t: eigenvalues 1, 1, 0
    lam, vec, Sfit = oc.eigen_fit(np.array([1.0]), _six(M), EPS)
    assert np.allclose(lam[:, 0], [1.0, 1.0, EPS], atol=1e-14)
    assert np.allclose(vec[2, :, 0], t, atol=1e-14)
    expect = np.eye(3) - (1.0 - EPS) * np.outer(t, t)
    assert np.allclose(Sfit[:, 0], _six(expect)[:, 0], atol=1e-14)


def test_single_plane_floor():
    n = np.array([0.0, 0.6, -0.8])
    M = np.outer(n, n)                       # SGGX of one flake with normal n: eigenvalues 1, 0, 0
    lam, vec, Sfit = oc.eigen_fit(np.array([0.25]), 0.25 * _six(M), EPS)
    assert np.allclose(lam[:, 0], [1.0, EPS, EPS], atol=1e-14)
    assert np.allclose(vec[0, :, 0], [0.0, -0.6, 0.8], atol=1e-14)   # largest component made positive
    expect = EPS * np.eye(3) + (1.0 - EPS) * np.outer(n, n)
    assert np.allclose(Sfit[:, 0], _six(expect)[:, 0], atol=1e-14)


def test_isotropic_and_empty_codes():
    w = np.array([1.0, 0.0, 5.0])
    S = np.concatenate([_six(np.eye(3)), np.zeros((6, 1)), np.zeros((6, 1))], axis=1)
    lam, vec, Sfit, code = oc.compact(w, S, EPS)
    assert (code == np.array([255, 255, 255, 128, 128, 128], dtype=np.uint8)).all()
    assert np.array_equal(lam, np.ones((3, 3)))
    dec = oc.decode(code)
    assert np.array_equal(dec, np.tile(np.array([1, 1, 1, 0, 0, 0], np.float32)[:, None], (1, 3)))


def test_hand_worked_bytes():
    # diag(1, 0.64, 0.04): sigma = 1, 0.8, 0.2 -> 255, 204, 51; no correlation -> 128
    # [[1, .6, 0], [.6, 1, 0], [0, 0, .36]]: sigma = 1, 1, 0.6 -> 255, 255, 153; r_xy = 0.6 -> 128 + 76
    S = np.concatenate([_six(np.diag([1.0, 0.64, 0.04])),
                        _six([[1.0, 0.6, 0.0], [0.6, 1.0, 0.0], [0.0, 0.0, 0.36]])], axis=1)
    code = oc.compact(np.array([1.0, 1.0]), S, EPS)[3]
    assert code.tolist() == [[255, 204, 51, 128, 128, 128], [255, 255, 153, 204, 128, 128]]
    # the eigenvalue floor acts before the code: one fiber along x gives sigma_x = sqrt(EPS)
    code = oc.compact(np.array([1.0]), _six(np.diag([0.0, 1.0, 1.0])), EPS)[3]
    assert code.tolist() == [[round(255 * math.sqrt(EPS)), 255, 255, 128, 128, 128]]


def _random_spd(n, seed):
    g = np.random.default_rng(seed)
    A = g.normal(size=(n, 3, 3))
    M = A @ np.transpose(A, (0, 2, 1)) + 0.05 * np.eye(3)
    w = g.uniform(0.1, 4.0, size=n)
    S = np.stack([M[:, 0, 0], M[:, 1, 1], M[:, 2, 2], M[:, 0, 1], M[:, 0, 2], M[:, 1, 2]]) * w
    return w, S, M


def test_eigen_equation_and_orthonormality():
    w, S, M = _random_spd(500, 3)
    lam, vec, Sfit = oc.eigen_fit(w, S, 1e-9)
    for v in range(0, 500, 7):
        V = vec[:, :, v]
        assert np.allclose(V @ V.T, np.eye(3), atol=1e-12)
        for i in range(3):
            assert np.allclose(M[v] @ V[i], lam[i, v] * V[i], atol=1e-10 * lam[0, v])
        assert lam[0, v] >= lam[1, v] >= lam[2, v]
    assert np.allclose(Sfit, S / w, atol=1e-12 * np.abs(S / w).max())


def test_scale_invariance_of_code():
    w, S, _ = _random_spd(300, 5)
    c1 = oc.compact(w, S, EPS)[3]
    c2 = oc.compact(w, 7.0 * S, EPS)[3]
    c3 = oc.compact(2.0 * w, 2.0 * S, EPS)[3]
    v = oc.encode_values(oc.eigen_fit(w, S, EPS)[2])
    frac = np.abs(v - np.rint(v))
    sure = (np.abs(frac - 0.5) > 1e-6).all(axis=0)   # voxels with no code value near a rounding tie
    assert sure.mean() > 0.95
    assert np.array_equal(c1[sure], c2[sure]) and np.array_equal(c1[sure], c3[sure])


def test_round_trip_within_quantisation_bound():
    w, S, _ = _random_spd(1000, 11)
    Sfit = oc.eigen_fit(w, S, EPS)[2]
    dec = oc.decode(oc.encode(Sfit)).astype(np.float64)
    d = Sfit[:3] / Sfit[:3].max(axis=0)
    sig, sig_dec = np.sqrt(d), np.sqrt(dec[:3])
    assert np.abs(sig - sig_dec).max() <= 0.5 / 255 + 1e-6
    for c, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
        r = Sfit[3 + c] / np.sqrt(Sfit[a] * Sfit[b])
        r_dec = dec[3 + c] / np.sqrt(dec[a] * dec[b])
        assert np.abs(r - r_dec).max() <= 0.5 / 127 + 1e-5


@pytest.mark.parametrize("eps", [1e-3, 1e-2])
def test_floor_bounds_condition_number(eps):
    w, S, _ = _random_spd(400, 17)
    S[:, :100] = 0.0
    S[1, :100] = w[:100]          # 100 single-plane voxels (normal along y): rank one
    lam = oc.eigen_fit(w, S, eps)[0]
    assert (lam[2] >= eps * lam[0] * (1 - 1e-12)).all()
    assert np.allclose(lam[:, :100], np.array([[1.0], [eps], [eps]]), atol=1e-14)
