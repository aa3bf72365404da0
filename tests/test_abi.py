"""CPU checks of the C ABI library: it loads, exports every function include/vx.h declares,
and its host-only calls behave (no kernel is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vx.h")
LIB = os.path.join(ROOT, "paper_2604_13191_amd", "libvx.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2604_13191_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_host_only_calls(lib):
    f = lib.vx_voxelize_workspace_size
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    assert f(0, 100, 1000, 500, 800, 6) > 0
    assert f(1, 100, 1000, 500, 800, 12) > f(1, 100, 1000, 500, 800, 6)      # 64-bit keys need more room
    assert f(1, 100, 1000, 500, 80000, 6) > f(1, 100, 1000, 500, 800, 6)     # leaf staging
    assert f(0, 1 << 32, 1, 1, 1, 6) == 0                                     # primitive ids are 32-bit
    assert f(3, 100, 1000, 500, 800, 6) == 0 and f(0, -1, 0, 0, 1, 6) == 0 and f(0, 1, 1, 1, 1, 21) == 0
    assert f(0, 1, 1, 1, 0, 6) == 0
    g = lib.vx_lod_workspace_size
    g.restype = ctypes.c_size_t
    g.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    assert g(1000, 7, 1) > 0 and g(0, 7, 1) == 0 and g(10, 7, 9) == 0
    s = lib.vx_status_str
    s.restype = ctypes.c_char_p
    assert s(0) == b"ok" and s(2) == b"capacity exceeded"


def test_argument_errors_before_any_launch(lib):
    class CGrid(ctypes.Structure):
        _fields_ = [("bmin", ctypes.c_double * 3), ("extent", ctypes.c_double), ("log2_res", ctypes.c_int32)]
    f = lib.vx_voxelize_triangles
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(CGrid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p]
    bad = CGrid((ctypes.c_double * 3)(0, 0, 0), 0.0, 4)
    assert f(ctypes.byref(bad), None, 0, 0, 0, None, 0, None, None, None, None) == 1
    good = CGrid((ctypes.c_double * 3)(0, 0, 0), 1.0, 4)
    assert f(ctypes.byref(good), None, 0, 0, 0, None, 0, None, None, None, None) == 1     # no outputs


def test_batch_and_graph_calls_host_side(lib):
    ws = lib.vx_batch_workspace_size
    ws.restype = ctypes.c_size_t
    ws.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    assert ws(1000, 1000, 5000, 4000, 4000) > ws(1, 1000, 5000, 4000, 4000) > 0
    assert ws(0, 1, 1, 1, 1) == 0 and ws(70000, 1, 1, 1, 1) == 0 and ws(2, 1 << 32, 1, 1, 1) == 0
    assert ws(2, 1, 1, 1, 0) == 0
    b = lib.vx_batch_build
    b.restype = ctypes.c_int
    assert b(None, None, 1, None, 0, None, 0, 1, 1, 0, 0, 0, None, None, None, None, None, None, 0, None, None) == 1
    gb = lib.vx_graph_begin
    gb.restype = ctypes.c_int
    gb.argtypes = [ctypes.c_void_p]
    assert gb(None) == 1                       # the null stream cannot be captured
    gl = lib.vx_graph_launch
    gl.restype = ctypes.c_int
    gl.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert gl(None, None) == 1
    lib.vx_graph_destroy.argtypes = [ctypes.c_void_p]
    lib.vx_graph_destroy(None)


class CTuning(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_int32), ("unit_budget", ctypes.c_int32), ("grids", ctypes.c_int32 * 5)]


def test_tuning_values_are_checked_before_any_launch(lib):
    class CGrid(ctypes.Structure):
        _fields_ = [("bmin", ctypes.c_double * 3), ("extent", ctypes.c_double), ("log2_res", ctypes.c_int32)]
    f = lib.vx_voxelize_triangles
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(CGrid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(CTuning),
                  ctypes.c_void_p]
    good = CGrid((ctypes.c_double * 3)(0, 0, 0), 1.0, 4)
    grids = (ctypes.c_int32 * 5)(0, 0, 0, 0, 0)
    for bad in (CTuning(5, 0, grids), CTuning(1, 0, grids), CTuning(0, 1000, grids), CTuning(0, 4096, grids),
                CTuning(0, 0, (ctypes.c_int32 * 5)(63, 0, 0, 0, 0)), CTuning(0, 0, (ctypes.c_int32 * 5)(0, 0, 0, 0, 16385))):
        assert f(ctypes.byref(good), None, 0, 0, 0, None, 0, None, None, ctypes.byref(bad), None) == 1
    assert not hasattr(lib, "vx_set_launch_grids")           # no tuning state in the library


def test_sggx_compact_argument_errors(lib):
    class CVox(ctypes.Structure):
        _fields_ = [("keys", ctypes.c_void_p), ("count", ctypes.c_void_p), ("w", ctypes.c_void_p),
                    ("S", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("cap", ctypes.c_int64)]
    f = lib.vx_sggx_compact
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(CVox), ctypes.c_void_p, ctypes.c_float] + [ctypes.c_void_p] * 4
    fake = 4096                                   # never dereferenced: every call below fails its checks
    v = CVox(None, None, fake, fake, None, 8)
    assert f(ctypes.byref(v), fake, 0.0, None, None, fake, None) == 1          # eps must be > 0
    assert f(ctypes.byref(v), fake, 1.5, None, None, fake, None) == 1          # eps <= 1
    assert f(ctypes.byref(v), fake, float("nan"), None, None, fake, None) == 1
    assert f(ctypes.byref(v), fake, 1e-3, None, None, None, None) == 1         # code is required
    assert f(ctypes.byref(v), fake, 1e-3, None, None, fake + 1, None) == 1     # code 2-byte aligned
    assert f(ctypes.byref(v), None, 1e-3, None, None, fake, None) == 1         # count required
    v0 = CVox(None, None, fake, fake, None, 0)
    assert f(ctypes.byref(v0), fake, 1e-3, None, None, fake, None) == 1        # cap >= 1
    d = lib.vx_sggx_decode
    d.restype = ctypes.c_int
    d.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    assert d(None, fake, 8, fake, None) == 1 and d(fake, fake, 0, fake, None) == 1
    assert d(fake + 1, fake, 8, fake, None) == 1
