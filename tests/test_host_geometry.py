"""The kernels' exact geometry, compiled for the host, against the exact-rational brute force.

The device header (closed-box triangle test, clipped area in the triangle's barycentric plane,
capsule test, clipped segment length) is built with the host compiler and called on small
lattices with adversarial inputs: vertices on voxel planes, quarter- and half-voxel lattices,
triangles flat on an axis, axis-parallel segments.  The brute force (``oracle/brute.py``) uses
other methods in rational arithmetic (polygon clipping, Minkowski decomposition).  Touches must
agree exactly, areas and lengths to 1e-10 of the primitive's own measure, and exact zeros must
be zeros (a piece that closes to a point or a segment).  Voxels are drawn from each primitive's
candidate range, the only ones the kernels ever test.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SB = 4                       # 16 lattice units per voxel
S = 1 << SB
R = 8                        # voxels per axis


@pytest.fixture(scope="module")
def geom(tmp_path_factory):
    cxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if cxx is None or not os.path.isdir(inc):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("geom") / "libhostgeom.so"
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{inc}",
                    f"-I{ROOT}/paper_2604_13191_amd/csrc", f"-I{ROOT}/include",
                    os.path.join(ROOT, "tests", "host_geom.cpp"), "-o", str(out)], check=True)
    L = ctypes.CDLL(str(out))
    P = ctypes.c_void_p
    L.hg_tri_touch.argtypes = [P, P, ctypes.c_int]
    L.hg_tri_area_frac.argtypes = [P, P, ctypes.c_int]
    L.hg_tri_area_frac.restype = ctypes.c_double
    L.hg_cap_touch.argtypes = [P, P, ctypes.c_int, ctypes.c_int64]
    L.hg_seg_frac.argtypes = [P, P, ctypes.c_int]
    L.hg_seg_frac.restype = ctypes.c_double
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cand(mn, mx, rho=0):
    """The kernels' candidate range of one axis (closed box: a voxel whose face the primitive
    reaches is a candidate), clamped to the grid."""
    lo = -((-(mn - rho)) // S) - 1
    hi = (mx + rho) // S
    return max(lo, 0), min(hi, R - 1)


def _triangles(rng, n):
    out = []
    for i in range(n):
        mode = i % 5
        if mode == 0:
            q = rng.integers(S, (R - 1) * S, size=(3, 3))                    # generic
        elif mode == 1:
            q = rng.integers(2, 4 * (R - 1), size=(3, 3)) * (S // 4)        # quarter-voxel lattice
        elif mode == 2:
            q = rng.integers(1, 2 * (R - 1), size=(3, 3)) * (S // 2)        # half-voxel lattice
        elif mode == 3:
            q = rng.integers(S, (R - 1) * S, size=(3, 3))
            a = int(rng.integers(0, 3))
            q[:, a] = int(rng.integers(1, R - 1)) * S                       # flat on a voxel plane
        else:
            q = rng.integers(S, 3 * S, size=(3, 3)) + int(rng.integers(0, 3)) * S   # small
        out.append(q.astype(np.int64))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_triangle_touch_and_area(geom, seed):
    rng = np.random.default_rng(seed)
    checked = zeros = 0
    for q in _triangles(rng, 160):
        q9 = np.ascontiguousarray(q.reshape(9).astype(np.int32))
        e0, e1 = q[1] - q[0], q[2] - q[0]
        whole = 0.5 * float(np.linalg.norm(np.cross(e0.astype(float), e1.astype(float)))) / S ** 2
        ranges = [_cand(int(q[:, a].min()), int(q[:, a].max())) for a in range(3)]
        for _ in range(3):
            v = np.array([int(rng.integers(lo, hi + 1)) for lo, hi in ranges], np.int64)
            lo3 = [int(x) * S for x in v]
            t = bool(geom.hg_tri_touch(_ptr(q9), _ptr(v), SB))
            assert t == brute.tri_touch(q, lo3, S), (q.tolist(), v.tolist())
            if not t or whole == 0.0:
                continue
            got = geom.hg_tri_area_frac(_ptr(q9), _ptr(v), SB) * whole
            ref = brute.tri_area(q, lo3, S)
            if ref == 0.0:
                zeros += 1
                assert got == 0.0, (q.tolist(), v.tolist(), got)
            else:
                assert abs(got - ref) <= 1e-10 * whole, (q.tolist(), v.tolist(), got, ref)
            checked += 1
    assert checked > 200 and zeros > 0


@pytest.mark.parametrize("seed", [0, 1])
def test_segment_touch_and_length(geom, seed):
    rng = np.random.default_rng(100 + seed)
    checked = zeros = 0
    for i in range(160):
        mode = i % 4
        a = rng.integers(S, (R - 1) * S, size=3)
        if mode == 1:
            a = rng.integers(2, 4 * (R - 1), size=3) * (S // 4)
        b = a + rng.integers(-2 * S, 2 * S, size=3)
        if mode == 2:
            b[int(rng.integers(0, 3))] = a[int(rng.integers(0, 3))]       # one axis parallel-ish
        if mode == 3:
            k = int(rng.integers(0, 3))
            b = a.copy()
            b[k] = a[k] + int(rng.integers(-2 * S, 2 * S))                  # axis-parallel
        b = np.clip(b, 0, R * S - 1)
        rho = int(rng.integers(1, S))
        r16 = np.zeros(16, np.int32)
        r16[0:3], r16[3:6] = a, b
        ranges = [_cand(int(min(a[k], b[k])), int(max(a[k], b[k])), rho) for k in range(3)]
        length = float(np.linalg.norm((b - a).astype(float))) / S
        for _ in range(3):
            v = np.array([int(rng.integers(lo, hi + 1)) for lo, hi in ranges], np.int64)
            lo3 = [int(x) * S for x in v]
            t = bool(geom.hg_cap_touch(_ptr(r16), _ptr(v), SB, rho))
            assert t == brute.cap_touch(a, b, lo3, S, rho), (a.tolist(), b.tolist(), v.tolist(), rho)
            if length == 0.0:
                continue
            got = geom.hg_seg_frac(_ptr(r16), _ptr(v), SB) * length
            ref = brute.seg_length(a, b, lo3, S)
            if ref == 0.0:
                zeros += 1
                assert got == 0.0, (a.tolist(), b.tolist(), v.tolist(), got)
            else:
                # the kernel returns the clipped fraction in FP32
                assert abs(got - ref) <= 1e-6 * length, (a.tolist(), b.tolist(), v.tolist(), got, ref)
            checked += 1
    assert checked > 200 and zeros > 0
