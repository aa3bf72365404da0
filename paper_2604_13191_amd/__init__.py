"""Sparse SGGX voxelization and LoD pyramids on MI355X (gfx950).

Thin Python binding over ``libvx.so`` (C ABI in ``include/vx.h``): argument marshalling,
device buffers from PyTorch, and the caller's HIP stream.  Every step of the path runs in the
library's HIP kernels; there is no fallback.  If the library is missing or no GPU is visible,
``load()`` raises.

Operations (arXiv 2604.13191):
  voxelize(primitives, grid bounds, resolution) -> sparse Morton-keyed leaf voxels holding
      {count, w, S} -- Sec. 3.1-3.4 and Sec. 4.1;
  build_lod(voxels, levels, lobes_per_voxel) -> pyramid -- Sec. 4.3-4.4.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvx.so")

VX_NSTAT = 4
STAT_CAND, STAT_PAIRS, STAT_VOXELS, STAT_FLAGS = range(4)
FLAG_CAND_CAPACITY, FLAG_PAIR_CAPACITY, FLAG_VOXEL_CAPACITY, FLAG_INPUT, FLAG_OFFSETS = 1, 2, 4, 8, 16
STATUS = {0: "ok", 1: "invalid argument", 2: "capacity exceeded", 3: "HIP runtime error",
          4: "non-finite or out-of-range input, or invalid fiber offsets", 5: "bad workspace"}


class VxError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class CGrid(ctypes.Structure):
    _fields_ = [("bmin", ctypes.c_double * 3), ("extent", ctypes.c_double), ("log2_res", ctypes.c_int32)]


class CVoxels(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("count", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("S", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("cap", ctypes.c_int64)]


class CLobes(ctypes.Structure):
    _fields_ = [("nl", ctypes.c_void_p), ("w", ctypes.c_void_p), ("S", ctypes.c_void_p), ("cap", ctypes.c_int64)]


_lib = None


def load():
    """Load libvx.so (built by __graft_entry__.build() / paper_2604_13191_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2604_13191_amd needs a visible AMD GPU (gfx950); none found")
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2604_13191_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.vx_voxelize_workspace_size.restype = sz
    L.vx_voxelize_workspace_size.argtypes = [i32, i64, i64, i64, i32]
    L.vx_voxelize_triangles.restype = ctypes.c_int
    L.vx_voxelize_triangles.argtypes = [ctypes.POINTER(CGrid), vp, i64, i64, i64, vp, sz,
                                        ctypes.POINTER(CVoxels), vp, vp]
    L.vx_voxelize_fibers.restype = ctypes.c_int
    L.vx_voxelize_fibers.argtypes = [ctypes.POINTER(CGrid), vp, i64, vp, i64, ctypes.c_float, i64, i64, vp, sz,
                                     ctypes.POINTER(CVoxels), vp, vp]
    L.vx_lod_workspace_size.restype = sz
    L.vx_lod_workspace_size.argtypes = [i64, i32, i32]
    L.vx_build_lod.restype = ctypes.c_int
    L.vx_build_lod.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CVoxels), vp, i32, i32, i32,
                               ctypes.POINTER(CVoxels), ctypes.POINTER(CLobes), vp, vp, sz, vp]
    L.vx_check_stats.restype = ctypes.c_int
    L.vx_check_stats.argtypes = [vp, vp]
    L.vx_status_str.restype = ctypes.c_char_p
    L.vx_status_str.argtypes = [ctypes.c_int]
    L.vx_timing_enable.argtypes = [i32]
    L.vx_timing_reset.argtypes = []
    L.vx_timing_collect.restype = i32
    L.vx_timing_collect.argtypes = [vp, vp, vp, i32]
    _lib = L
    return L


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _cgrid(grid) -> CGrid:
    return CGrid((ctypes.c_double * 3)(*[float(x) for x in grid.bmin]), float(grid.extent), int(grid.log2_res))


def key_dtype(log2_res):
    import torch
    return torch.int64 if log2_res > 10 else torch.int32


def _ws(nbytes, device):
    import torch
    # 256-byte alignment: the caching allocator hands out 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class Voxels:
    """One level of voxels on the device (capacity-sized tensors; ``n`` valid entries)."""
    keys: object          # int32 (uint32 bit pattern) or int64 [cap]
    count: object         # int32 (uint32 bit pattern) [cap]
    w: object             # float32 [cap]
    S: object             # float32 [6, cap] (xx, yy, zz, xy, xz, yz)
    mask: object          # uint8 [cap] or None at the leaf
    n: int = -1           # host copy of the count once known

    @property
    def cap(self):
        return int(self.w.shape[0])

    def cstruct(self) -> CVoxels:
        return CVoxels(self.keys.data_ptr(), self.count.data_ptr(), self.w.data_ptr(), self.S.data_ptr(),
                       self.mask.data_ptr() if self.mask is not None else None, self.cap)

    def numpy(self, n=None):
        """Host copies of the first n entries: keys as unsigned, S as [n, 6]."""
        n = self.n if n is None else n
        k = self.keys[:n].cpu().numpy()
        k = k.view(np.uint32) if k.dtype == np.int32 else k.view(np.uint64)
        out = {"keys": k, "count": self.count[:n].cpu().numpy().view(np.uint32),
               "w": self.w[:n].cpu().numpy(), "S": self.S[:, :n].cpu().numpy().T.copy()}
        if self.mask is not None:
            out["mask"] = self.mask[:n].cpu().numpy()
        return out


def alloc_voxels(cap, log2_res, device, with_mask):
    import torch
    cap = max(int(cap), 1)
    return Voxels(torch.empty(cap, dtype=key_dtype(log2_res), device=device),
                  torch.empty(cap, dtype=torch.int32, device=device),
                  torch.empty(cap, dtype=torch.float32, device=device),
                  torch.empty((6, cap), dtype=torch.float32, device=device),
                  torch.empty(cap, dtype=torch.uint8, device=device) if with_mask else None)


class VoxelizePlan:
    """Buffers and capacities for voxelizing one set of primitives, reusable across runs.

    The capacities come from the library's own counts: a first call with zero capacities
    reports the candidate total, a second one the pair total (both via device stats, read
    back once here).  ``run()`` then enqueues the whole voxelize pass with no host sync.
    """

    def __init__(self, kind, grid, data, offsets=None, radius=0.0, max_cand=None, max_pairs=None, out_cap=None):
        import torch
        self.L = load()
        self.kind = kind
        self.grid = grid
        self.cgrid = _cgrid(grid)
        self.data = data.contiguous()
        if self.data.dtype != torch.float32 or not self.data.is_cuda:
            raise TypeError("primitives must be a float32 CUDA tensor")
        self.device = self.data.device
        if kind == 0:
            self.n_prims = int(self.data.numel() // 9)
            self.offsets = None
            self.n_fib = 0
        else:
            self.n_prims = int(self.data.numel() // 3)
            self.offsets = offsets.to(device=self.device, dtype=torch.int64).contiguous()
            self.n_fib = int(self.offsets.numel() - 1)
        self.radius = float(radius)
        self.stats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.device)
        if max_cand is None or max_pairs is None:
            mc, mp = self._count()
            max_cand = mc if max_cand is None else max_cand
            max_pairs = mp if max_pairs is None else max_pairs
        self.max_cand = int(max_cand)
        self.max_pairs = int(max_pairs)
        nb = self.L.vx_voxelize_workspace_size(kind, self.n_prims, self.max_cand, self.max_pairs,
                                               int(grid.log2_res))
        if nb == 0:
            raise VxError(1, "vx_voxelize_workspace_size")
        self.ws = _ws(nb, self.device)
        self.out = alloc_voxels(out_cap if out_cap is not None else self.max_pairs, grid.log2_res, self.device,
                                False)
        self._cout = self.out.cstruct()

    def _call(self, max_cand, max_pairs, ws, ws_bytes, cout, stream):
        if self.kind == 0:
            st = self.L.vx_voxelize_triangles(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims, max_cand,
                                              max_pairs, ws, ws_bytes, ctypes.byref(cout), _ptr(self.stats), stream)
        else:
            st = self.L.vx_voxelize_fibers(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                           _ptr(self.offsets), self.n_fib, self.radius, max_cand, max_pairs, ws,
                                           ws_bytes, ctypes.byref(cout), _ptr(self.stats), stream)
        if st != 0:
            raise VxError(st, "voxelize")

    def _count(self):
        """Candidate and pair totals from two counting calls (zero capacities)."""
        s = _stream()
        tmp_out = alloc_voxels(1, self.grid.log2_res, self.device, False)
        cout = tmp_out.cstruct()
        for step in range(2):
            mc = 0 if step == 0 else n_cand
            nb = self.L.vx_voxelize_workspace_size(self.kind, self.n_prims, mc, 0, int(self.grid.log2_res))
            ws = _ws(nb, self.device)
            self._call(mc, 0, _ptr(ws), nb, cout, s)
            st = self.L.vx_check_stats(_ptr(self.stats), s)
            h = self.stats.cpu().numpy()
            if h[STAT_FLAGS] & (FLAG_INPUT | FLAG_OFFSETS):
                raise VxError(4, "voxelize")
            if step == 0:
                n_cand = int(h[STAT_CAND])
            else:
                n_pairs = int(h[STAT_PAIRS])
            del ws
        return n_cand, n_pairs

    def run(self, stream=None):
        self._call(self.max_cand, self.max_pairs, _ptr(self.ws), self.ws.numel(), self._cout, _stream(stream))
        return self

    def check(self, stream=None):
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        h = self.stats.cpu().numpy()
        if st != 0:
            raise VxError(st, f"voxelize (stats {h.tolist()})")
        self.out.n = int(h[STAT_VOXELS])
        self.n_pairs = int(h[STAT_PAIRS])
        self.n_cand = int(h[STAT_CAND])
        return self.out


@dataclass
class Lobes:
    """Up to K SGGX lobes per voxel of one level (K > 1)."""
    nl: object            # uint8 [cap]
    w: object             # float32 [K, cap], descending weight
    S: object             # float32 [6, K, cap]
    n: int = -1

    def cstruct(self) -> CLobes:
        return CLobes(self.nl.data_ptr(), self.w.data_ptr(), self.S.data_ptr(), int(self.w.shape[1]))

    def numpy(self, n=None):
        n = self.n if n is None else n
        return {"nl": self.nl[:n].cpu().numpy(), "w": self.w[:, :n].cpu().numpy().T.copy(),
                "S": self.S[:, :, :n].cpu().numpy().transpose(2, 1, 0).copy()}


class LodPlan:
    """Per-level output buffers for build_lod; level caps default to the leaf's count."""

    def __init__(self, grid, leaf: Voxels, n_leaf_dev, levels, K=1, iters=2, caps=None):
        import torch
        self.L = load()
        self.grid, self.cgrid = grid, _cgrid(grid)
        self.leaf, self.levels, self.K, self.iters = leaf, int(levels), int(K), int(iters)
        dev = leaf.w.device
        self.n_leaf_dev = n_leaf_dev
        base = leaf.n if leaf.n > 0 else leaf.cap
        caps = caps or [base] * (self.levels - 1)
        self.out = [alloc_voxels(c, grid.log2_res, dev, True) for c in caps]
        self._cout = (CVoxels * max(1, len(self.out)))(*[v.cstruct() for v in self.out])
        self.lobes = []
        self._clobes = None
        if self.K > 1:
            self.lobes = [Lobes(torch.empty(v.cap, dtype=torch.uint8, device=dev),
                                torch.empty((self.K, v.cap), dtype=torch.float32, device=dev),
                                torch.empty((6, self.K, v.cap), dtype=torch.float32, device=dev)) for v in self.out]
            self._clobes = (CLobes * max(1, len(self.lobes)))(*[lb.cstruct() for lb in self.lobes])
        self._cleaf = leaf.cstruct()
        self.n_levels = torch.zeros(self.levels + 1, dtype=torch.int64, device=dev)
        nb = self.L.vx_lod_workspace_size(leaf.cap, self.levels, self.K)
        if nb == 0:
            raise VxError(1, "vx_lod_workspace_size")
        self.ws = _ws(nb, dev)

    def run(self, stream=None):
        st = self.L.vx_build_lod(ctypes.byref(self.cgrid), ctypes.byref(self._cleaf), _ptr(self.n_leaf_dev),
                                 self.levels, self.K, self.iters, self._cout, self._clobes, _ptr(self.n_levels),
                                 _ptr(self.ws), self.ws.numel(), _stream(stream))
        if st != 0:
            raise VxError(st, "build_lod")
        return self

    def check(self):
        import torch
        torch.cuda.synchronize()
        h = self.n_levels.cpu().numpy()
        if h[self.levels] & FLAG_VOXEL_CAPACITY:
            raise VxError(2, "build_lod")
        for L in range(1, self.levels):
            self.out[L - 1].n = int(h[L])
            if self.lobes:
                self.lobes[L - 1].n = int(h[L])
        return [self.leaf] + self.out


def voxelize_triangles(tris, grid, **kw):
    """Triangle soup float32 [n, 3, 3] on the GPU -> leaf Voxels (plan kept on .plan)."""
    p = VoxelizePlan(0, grid, tris, **kw).run()
    v = p.check()
    v.plan = p
    return v


def voxelize_fibers(pts, offsets, radius, grid, **kw):
    """Polylines: float32 [m, 3] points + int64 CSR offsets [F + 1] -> leaf Voxels."""
    p = VoxelizePlan(1, grid, pts, offsets=offsets, radius=radius, **kw).run()
    v = p.check()
    v.plan = p
    return v


def build_lod(grid, leaf: Voxels, levels, K=1, iters=2, n_leaf_dev=None, caps=None, return_lobes=False):
    """Leaf voxels -> list [leaf, level 1, ..., level levels-1] (Sec. 4.3); with K > 1 and
    return_lobes, also the per-level lobes [level 1, ...] (Sec. 4.4)."""
    import torch
    if n_leaf_dev is None:
        n_leaf_dev = torch.tensor([leaf.n], dtype=torch.int64, device=leaf.w.device)
    p = LodPlan(grid, leaf, n_leaf_dev, levels, K, iters, caps).run()
    out = p.check()
    if return_lobes:
        return out, p.lobes
    return out


def timing_enable(on=True):
    load().vx_timing_enable(1 if on else 0)


def timing_reset():
    load().vx_timing_reset()


def timing_collect():
    """{kernel name: (total ms, launches)} accumulated since the last reset (synchronises)."""
    L = load()
    n = 64
    names = (ctypes.c_char * 48 * n)()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    k = L.vx_timing_collect(names, ms, cnt, n)
    return {bytes(names[i]).split(b"\0")[0].decode(): (ms[i], cnt[i]) for i in range(min(k, n))}
