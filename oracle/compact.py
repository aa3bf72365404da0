"""FP64 CPU oracle for the leaf eigen-fit and the 6-byte SGGX code -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
use this module; the product path never does, and this file shares nothing with it.

What it follows:

* ``eigen_fit`` -- Sec. 4.1 ("Fitting to SGGX distribution"): the orientation matrix of a voxel
  is decomposed into eigenvectors w_1, w_2, w_3 and eigenvalues, the eigenvalues being the
  projected areas sigma(w_i) along those directions, and the SGGX matrix is rebuilt as
  (w_1 w_2 w_3) diag(sigma) (w_1 w_2 w_3)^T (the equation labelled SGGX-from-fit).  The same
  subsection asks that nearly single-orientation voxels, whose matrix is almost singular, be
  made well defined; here that is a floor on the eigenvalues, ``lam_i >= eps * lam_1``.
* ``encode`` / ``decode`` -- Sec. 4.3 ("Storing data", the compact-SGGX equation): three
  square roots of the diagonal and three correlation coefficients, one byte each.

Readings (where the paper leaves it open):

* The matrix decomposed is the voxel's normalised SGGX ``M = S / w`` of the uncentred,
  weighted moment sums the voxelizer stores; ``w <= 0`` (a voxel only touched) or ``M = 0``
  gives the isotropic SGGX (identity, eigenvalues 1, eigenvectors the axes).
* Eigenvalues in descending order; each eigenvector has unit length and its component of
  largest magnitude positive (the first such component on ties).
* The byte code is scale free: the rebuilt matrix is divided by its largest diagonal entry,
  so the largest sigma is 1.  sigma in [0, 1] is stored as ``rint(255 sigma)``, a
  correlation r in [-1, 1] as ``128 + rint(127 r)`` (r = 0 is exactly 128), byte order
  sigma_x, sigma_y, sigma_z, r_xy, r_xz, r_yz.  Decoding inverts the two maps
  (``sigma = b / 255``, ``r = (b - 128) / 127``) and rebuilds ``S_aa = sigma_a^2``,
  ``S_ab = r_ab sigma_a sigma_b`` in FP64, rounded once to float.

Pins (``tests/test_oracle_compact.py``): diagonal matrices, matrices with a known rotation,
the single-fiber and single-plane closed forms, the isotropic code, scale invariance,
round-trip error within the quantisation bound, and byte values worked out by hand.
"""
from __future__ import annotations

import numpy as np

# component order of the stored six entries: xx, yy, zz, xy, xz, yz
_PAIRS = ((0, 1), (0, 2), (1, 2))


def _full(S6: np.ndarray) -> np.ndarray:
    """[6, n] upper entries -> [n, 3, 3] symmetric matrices (FP64)."""
    S6 = np.asarray(S6, dtype=np.float64)
    n = S6.shape[1]
    A = np.zeros((n, 3, 3))
    for a in range(3):
        A[:, a, a] = S6[a]
    for c, (a, b) in enumerate(_PAIRS):
        A[:, a, b] = S6[3 + c]
        A[:, b, a] = S6[3 + c]
    return A


def eigen_fit(w, S6, eps: float):
    """Leaf eigen-fit of Sec. 4.1 for n voxels.

    w: [n] weights; S6: [6, n] moment sums (xx, yy, zz, xy, xz, yz).
    Returns (lam [3, n] descending floored eigenvalues, vec [3, 3, n] with vec[i, c] the
    component c of eigenvector i, Sfit [6, n] the rebuilt matrix), all FP64.
    """
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    A = _full(S6)
    lam = np.ones((3, n))
    vec = np.zeros((3, 3, n))
    for i in range(3):
        vec[i, i, :] = 1.0
    ok = w > 0
    if ok.any():
        M = A[ok] / w[ok, None, None]
        val, V = np.linalg.eigh(M)              # ascending; V[:, :, j] is the j-th eigenvector
        val = val[:, ::-1]
        V = V[:, :, ::-1]
        good = val[:, 0] > 0
        for j in range(3):
            v = V[:, :, j]
            big = np.argmax(np.abs(v), axis=1)
            sgn = np.where(v[np.arange(v.shape[0]), big] < 0, -1.0, 1.0)
            V[:, :, j] = v * sgn[:, None]
        lamf = np.maximum(val, eps * val[:, :1])
        idx = np.nonzero(ok)[0][good]
        lam[:, idx] = lamf[good].T
        vec[:, :, idx] = np.transpose(V[good], (2, 1, 0))
    Sfit = np.empty((6, n))
    for a in range(3):
        Sfit[a] = np.einsum("in,in->n", vec[:, a, :] * lam, vec[:, a, :])
    for c, (a, b) in enumerate(_PAIRS):
        Sfit[3 + c] = np.einsum("in,in->n", vec[:, a, :] * lam, vec[:, b, :])
    return lam, vec, Sfit


def encode_values(Sfit):
    """The six pre-rounding code values (255 sigma, 127 r) of the compact-SGGX equation, FP64."""
    Sfit = np.asarray(Sfit, dtype=np.float64)
    d = Sfit[:3]
    scale = d.max(axis=0)
    sig = np.sqrt(d / scale)
    vals = np.empty_like(Sfit)
    vals[:3] = 255.0 * sig
    for c, (a, b) in enumerate(_PAIRS):
        vals[3 + c] = 127.0 * (Sfit[3 + c] / np.sqrt(d[a] * d[b]))
    return vals


def encode(Sfit) -> np.ndarray:
    """[6, n] rebuilt matrices -> [n, 6] bytes (sigma_x, sigma_y, sigma_z, r_xy, r_xz, r_yz)."""
    v = encode_values(Sfit)
    code = np.empty(v.shape, dtype=np.int64)
    code[:3] = np.rint(v[:3])
    code[3:] = 128 + np.rint(v[3:])
    return np.ascontiguousarray(code.T.astype(np.uint8))


def decode(code) -> np.ndarray:
    """[n, 6] bytes -> [6, n] float32 SGGX matrices (largest sigma about 1)."""
    b = np.asarray(code, dtype=np.float64).T
    sig = b[:3] / 255.0
    r = (b[3:] - 128.0) / 127.0
    out = np.empty((6, b.shape[1]))
    out[:3] = sig * sig
    for c, (a, q) in enumerate(_PAIRS):
        out[3 + c] = r[c] * sig[a] * sig[q]
    return out.astype(np.float32)


def compact(w, S6, eps: float):
    """The whole leaf step: eigen-fit, then the byte code.  Returns (lam, vec, Sfit, code)."""
    lam, vec, Sfit = eigen_fit(w, S6, eps)
    return lam, vec, Sfit, encode(Sfit)
