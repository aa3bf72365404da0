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

VX_NSTAT = 6
STAT_CAND, STAT_PAIRS, STAT_VOXELS, STAT_FLAGS, STAT_RECORDS, STAT_UNITS = range(6)
FLAG_CAND_CAPACITY, FLAG_PAIR_CAPACITY, FLAG_VOXEL_CAPACITY, FLAG_INPUT, FLAG_OFFSETS = 1, 2, 4, 8, 16
FLAG_RECORD_CAPACITY, FLAG_UNIT_CAPACITY = 32, 64
FLAG_FIT_ROWS, FLAG_FIT_KEYS, FLAG_OCC_LEAF = 128, 256, 512
NOALLOC_MAX_LEAF = 8388608          # leaf capacity limit of vx_build_lod_noalloc
STATUS = {0: "ok", 1: "invalid argument", 2: "capacity exceeded", 3: "HIP runtime error",
          4: "non-finite or out-of-range input, or invalid fiber offsets", 5: "bad workspace",
          6: "fit parameters bound to other voxels than the level holds"}


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


class CPatch(ctypes.Structure):
    _fields_ = [("grid", CGrid), ("pt_begin", ctypes.c_int64), ("pt_end", ctypes.c_int64),
                ("radius", ctypes.c_float), ("reserved", ctypes.c_int32)]


class CTuning(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_int32), ("unit_budget", ctypes.c_int32), ("grids", ctypes.c_int32 * 5)]


TUNE_KERNELS = ("unit", "unit_plan", "unit_compact", "lod_reduce", "lod_cluster")


@dataclass(frozen=True)
class Tuning:
    """Work decomposition of one call (include/vx.h, vx_tuning); 0 = the library's default.
    tile_bits: leaf tiles of 2^tile_bits voxels per axis (2..4); unit_budget: candidates per work
    unit (1024, 1536, 2048, 3072); grids: blocks of the kernels in TUNE_KERNELS order."""
    tile_bits: int = 0
    unit_budget: int = 0
    grids: tuple = (0, 0, 0, 0, 0)

    def cstruct(self) -> "CTuning":
        g = tuple(int(x) for x in self.grids)
        if len(g) != 5:
            raise ValueError("tuning: five grid sizes")
        return CTuning(int(self.tile_bits), int(self.unit_budget), (ctypes.c_int32 * 5)(*g))

    def as_dict(self):
        return {"tile_bits": int(self.tile_bits), "unit_budget": int(self.unit_budget),
                "grids": [int(x) for x in self.grids]}

    @staticmethod
    def from_dict(d):
        if d is None:
            return None
        return Tuning(int(d.get("tile_bits", 0)), int(d.get("unit_budget", 0)), tuple(d.get("grids", (0,) * 5)))


def _ctuning(t):
    return ctypes.byref(t.cstruct()) if t is not None else None


class CSampling(ctypes.Structure):
    _fields_ = [("chords_per_segment", ctypes.c_int32), ("samples_per_chord", ctypes.c_int32),
                ("max_triangle_samples", ctypes.c_int32)]


class COccupancy(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_void_p), ("hits", ctypes.c_void_p), ("cap", ctypes.c_int64)]


class CFibers(ctypes.Structure):
    _fields_ = [("pts", ctypes.c_void_p), ("n_pts", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("n_fibers", ctypes.c_int64), ("radius", ctypes.c_float)]


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
    L.vx_voxelize_workspace_size.argtypes = [i32, i64, i64, i64, i64, i32]
    L.vx_voxelize_triangles.restype = ctypes.c_int
    L.vx_voxelize_triangles.argtypes = [ctypes.POINTER(CGrid), vp, i64, i64, i64, vp, sz,
                                        ctypes.POINTER(CVoxels), vp, ctypes.POINTER(CTuning), vp]
    L.vx_voxelize_fibers.restype = ctypes.c_int
    L.vx_voxelize_fibers.argtypes = [ctypes.POINTER(CGrid), vp, i64, vp, i64, ctypes.c_float, i64, i64, vp, sz,
                                     ctypes.POINTER(CVoxels), vp, ctypes.POINTER(CTuning), vp]
    L.vx_sample_workspace_size.restype = sz
    L.vx_sample_workspace_size.argtypes = [i32, i64, i64, i64, i32, ctypes.POINTER(CSampling)]
    L.vx_sample_triangles.restype = ctypes.c_int
    L.vx_sample_triangles.argtypes = [ctypes.POINTER(CGrid), vp, i64, ctypes.POINTER(CSampling), i64, vp, sz,
                                      ctypes.POINTER(CVoxels), vp, vp]
    L.vx_sample_fibers.restype = ctypes.c_int
    L.vx_sample_fibers.argtypes = [ctypes.POINTER(CGrid), vp, i64, vp, i64, ctypes.POINTER(CSampling), i64, vp, sz,
                                   ctypes.POINTER(CVoxels), vp, vp]
    L.vx_build_sggxh.restype = ctypes.c_int
    L.vx_build_sggxh.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CVoxels), ctypes.POINTER(CVoxels), vp, i32,
                                 i32, i32, ctypes.POINTER(CLobes), vp, vp]
    L.vx_occupancy_workspace_size.restype = sz
    L.vx_occupancy_workspace_size.argtypes = [i32, i64, i64, i64, i32]
    L.vx_occupancy_triangles.restype = ctypes.c_int
    L.vx_occupancy_triangles.argtypes = [ctypes.POINTER(CGrid), vp, i64, ctypes.POINTER(CVoxels),
                                         ctypes.POINTER(CVoxels), vp, i32, i64, i64, ctypes.POINTER(COccupancy), vp,
                                         sz, vp, vp]
    L.vx_occupancy_fibers.restype = ctypes.c_int
    L.vx_occupancy_fibers.argtypes = [ctypes.POINTER(CGrid), vp, i64, vp, i64, ctypes.c_float,
                                      ctypes.POINTER(CVoxels), ctypes.POINTER(CVoxels), vp, i32, i64, i64,
                                      ctypes.POINTER(COccupancy), vp, sz, vp, vp]
    L.vx_lod_workspace_size.restype = sz
    L.vx_lod_workspace_size.argtypes = [i64, i32, i32]
    L.vx_build_lod.restype = ctypes.c_int
    L.vx_build_lod.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CVoxels), vp, i32, i32, i32,
                               ctypes.POINTER(CVoxels), ctypes.POINTER(CLobes), vp, vp, sz, ctypes.POINTER(CTuning), vp]
    L.vx_build_lod_noalloc.restype = ctypes.c_int
    L.vx_build_lod_noalloc.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CVoxels), vp, i32, i32, i32,
                                       ctypes.POINTER(CVoxels), ctypes.POINTER(CLobes), vp,
                                       ctypes.POINTER(CTuning), vp]
    L.vx_check_stats.restype = ctypes.c_int
    L.vx_check_stats.argtypes = [vp, vp]
    L.vx_status_str.restype = ctypes.c_char_p
    L.vx_status_str.argtypes = [ctypes.c_int]
    L.vx_fit_workspace_size.restype = sz
    L.vx_fit_workspace_size.argtypes = [i64, i64, i64, vp, i32, i32]
    L.vx_fit_forward.restype = ctypes.c_int
    L.vx_fit_forward.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CVoxels), vp, i32, i32, vp, vp, vp, vp, i32,
                                 vp, vp, vp, vp, sz, vp]
    L.vx_fit_backward.restype = ctypes.c_int
    L.vx_fit_backward.argtypes = [ctypes.POINTER(CGrid), ctypes.POINTER(CFibers), i64, i64, ctypes.POINTER(CVoxels),
                                  vp, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.vx_batch_workspace_size.restype = sz
    L.vx_batch_workspace_size.argtypes = [i32, i64, i64, i64, i64]
    L.vx_batch_build.restype = ctypes.c_int
    L.vx_batch_build.argtypes = [ctypes.POINTER(CPatch), vp, i32, vp, i64, vp, i64, i32, i32, i32, i64, i64,
                                 ctypes.POINTER(CVoxels), ctypes.POINTER(CLobes), vp, vp, vp, vp, sz,
                                 ctypes.POINTER(CTuning), vp]
    L.vx_graph_begin.restype = ctypes.c_int
    L.vx_graph_begin.argtypes = [vp]
    L.vx_graph_end.restype = ctypes.c_int
    L.vx_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
    L.vx_graph_launch.restype = ctypes.c_int
    L.vx_graph_launch.argtypes = [vp, vp]
    L.vx_graph_destroy.restype = None
    L.vx_graph_destroy.argtypes = [vp]
    L.vx_timing_filter.argtypes = [ctypes.c_char_p]
    L.vx_timing_filter.restype = None
    L.vx_timing_enable.argtypes = [i32]
    L.vx_timing_reset.argtypes = []
    L.vx_timing_collect.restype = i32
    L.vx_timing_collect.argtypes = [vp, vp, vp, i32]
    L.vx_sggx_compact.restype = i32
    L.vx_sggx_compact.argtypes = [ctypes.POINTER(CVoxels), vp, ctypes.c_float, vp, vp, vp, vp]
    L.vx_sggx_decode.restype = i32
    L.vx_sggx_decode.argtypes = [vp, vp, i64, vp, vp]
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

    The capacities come from the library's own counts: counting calls report the
    primitive-tile records, then the work units, then the leaf voxels (device stats, read back
    once each).  ``run()`` then enqueues the whole voxelize pass with no host sync.
    """

    def __init__(self, kind, grid, data, offsets=None, radius=0.0, max_records=None, max_units=None, out_cap=None,
                 tuning=None):
        import torch
        self.L = load()
        self.kind = kind
        self.tuning = tuning
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
        if max_records is None or max_units is None or out_cap is None:
            r, u, v = self._count(max_records, max_units)
            max_records = r if max_records is None else max_records
            max_units = u if max_units is None else max_units
            out_cap = v if out_cap is None else out_cap
        self.max_records = int(max_records)
        self.max_units = int(max_units)
        self.out = alloc_voxels(max(int(out_cap), 1), grid.log2_res, self.device, False)
        self.ws = self._ws_for(self.max_records, self.max_units, self.out.cap)
        self._cout = self.out.cstruct()

    def _ws_for(self, max_records, max_units, max_voxels):
        nb = self.L.vx_voxelize_workspace_size(self.kind, self.n_prims, max_records, max_units, max(max_voxels, 1),
                                               int(self.grid.log2_res))
        if nb == 0:
            raise VxError(1, "vx_voxelize_workspace_size")
        return _ws(nb, self.device)

    def _call(self, max_records, max_units, ws, ws_bytes, cout, stream):
        if self.kind == 0:
            st = self.L.vx_voxelize_triangles(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims, max_records,
                                              max_units, ws, ws_bytes, ctypes.byref(cout), _ptr(self.stats),
                                              _ctuning(self.tuning), stream)
        else:
            st = self.L.vx_voxelize_fibers(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                           _ptr(self.offsets), self.n_fib, self.radius, max_records, max_units, ws,
                                           ws_bytes, ctypes.byref(cout), _ptr(self.stats), _ctuning(self.tuning),
                                           stream)
        if st != 0:
            raise VxError(st, "voxelize")

    def _count(self, max_records=None, max_units=None):
        """Record, unit and leaf-voxel totals from counting calls (capacities still unknown are 0)."""
        s = _stream()
        tmp_out = alloc_voxels(1, self.grid.log2_res, self.device, False)
        cout = tmp_out.cstruct()
        r = max_records
        u = max_units
        for step in range(3):
            if step == 0 and r is not None:
                continue
            if step == 1 and u is not None:
                continue
            rr = 0 if r is None else r
            uu = 0 if u is None else u
            ws = self._ws_for(rr, uu, 1)
            self._call(rr, uu, _ptr(ws), ws.numel(), cout, s)
            self.L.vx_check_stats(_ptr(self.stats), s)
            h = self.stats.cpu().numpy()
            if h[STAT_FLAGS] & (FLAG_INPUT | FLAG_OFFSETS):
                raise VxError(4, "voxelize")
            if step == 0:
                r = int(h[STAT_RECORDS])
            elif step == 1:
                u = int(h[STAT_UNITS])
            else:
                v = int(h[STAT_VOXELS])
            del ws
        return r, u, v

    def run(self, stream=None):
        self._call(self.max_records, self.max_units, _ptr(self.ws), self.ws.numel(), self._cout, _stream(stream))
        return self

    def check(self, stream=None):
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        h = self.stats.cpu().numpy()
        if st != 0:
            raise VxError(st, f"voxelize (stats {h.tolist()})")
        self.out.n = int(h[STAT_VOXELS])
        self.n_pairs = int(h[STAT_PAIRS])
        self.n_cand = int(h[STAT_CAND])
        self.n_records = int(h[STAT_RECORDS])
        self.n_units = int(h[STAT_UNITS])
        return self.out


class SamplePlan:
    """The sampling voxelizer (Sec. 3.2-3.3) for one set of primitives, reusable across runs.

    kind 0: triangles float32 [n, 3, 3], ``N`` samples for the largest triangle (the others in
    proportion to their area); kind 1: fibers float32 [m, 3] + int64 offsets, ``chords`` chords
    per Catmull-Rom span and ``per_chord`` samples per chord.  The sample and voxel capacities
    come from two counting calls (device stats read back once each); ``run()`` then enqueues the
    whole pass with no host sync.
    """

    def __init__(self, kind, grid, data, offsets=None, N=16, chords=4, per_chord=4, max_samples=None, out_cap=None):
        import torch
        self.L = load()
        self.kind = kind
        self.grid = grid
        self.cgrid = _cgrid(grid)
        self.sampling = CSampling(int(chords), int(per_chord), int(N))
        self.data = data.contiguous()
        if self.data.dtype != torch.float32 or not self.data.is_cuda:
            raise TypeError("primitives must be a float32 CUDA tensor")
        self.device = self.data.device
        if kind == 0:
            self.n_prims = int(self.data.numel() // 9)
            self.offsets, self.n_fib = None, 0
        else:
            self.n_prims = int(self.data.numel() // 3)
            self.offsets = offsets.to(device=self.device, dtype=torch.int64).contiguous()
            self.n_fib = int(self.offsets.numel() - 1)
        self.stats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.device)
        if max_samples is None or out_cap is None:
            s = _stream()
            tmp = alloc_voxels(1, grid.log2_res, self.device, False)
            ms = 0 if max_samples is None else int(max_samples)
            for step in range(2):
                if step == 0 and max_samples is not None:
                    continue
                ws = self._ws_for(ms, 1)
                self._call(ms, ws, tmp.cstruct(), s)
                self.L.vx_check_stats(_ptr(self.stats), s)
                h = self.stats.cpu().numpy()
                if h[STAT_FLAGS] & (FLAG_INPUT | FLAG_OFFSETS):
                    raise VxError(4, "sample")
                if step == 0:
                    ms = int(h[STAT_CAND])
                else:
                    v = int(h[STAT_VOXELS])
                del ws
            max_samples = ms if max_samples is None else max_samples
            out_cap = v if out_cap is None else out_cap
        self.max_samples = int(max_samples)
        self.out = alloc_voxels(max(int(out_cap), 1), grid.log2_res, self.device, False)
        self.ws = self._ws_for(self.max_samples, self.out.cap)
        self._cout = self.out.cstruct()

    def _ws_for(self, max_samples, max_voxels):
        nb = self.L.vx_sample_workspace_size(self.kind, self.n_prims, max_samples, max(max_voxels, 1),
                                             int(self.grid.log2_res), ctypes.byref(self.sampling))
        if nb == 0:
            raise VxError(1, "vx_sample_workspace_size")
        return _ws(nb, self.device)

    def _call(self, max_samples, ws, cout, stream):
        if self.kind == 0:
            st = self.L.vx_sample_triangles(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                            ctypes.byref(self.sampling), max_samples, _ptr(ws), ws.numel(),
                                            ctypes.byref(cout), _ptr(self.stats), stream)
        else:
            st = self.L.vx_sample_fibers(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                         _ptr(self.offsets), self.n_fib, ctypes.byref(self.sampling), max_samples,
                                         _ptr(ws), ws.numel(), ctypes.byref(cout), _ptr(self.stats), stream)
        if st != 0:
            raise VxError(st, "sample")

    def run(self, stream=None):
        self._call(self.max_samples, self.ws, self._cout, _stream(stream))
        return self

    def check(self, stream=None):
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        h = self.stats.cpu().numpy()
        if st != 0:
            raise VxError(st, f"sample (stats {h.tolist()})")
        self.out.n = int(h[STAT_VOXELS])
        self.n_samples = int(h[STAT_CAND])
        self.n_inside = int(h[STAT_PAIRS])
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

    def __init__(self, grid, leaf: Voxels, n_leaf_dev, levels, K=1, iters=2, caps=None, noalloc=False, tuning=None):
        """noalloc: run vx_build_lod_noalloc (the library's own scratch, no workspace tensor;
        leaf caps up to NOALLOC_MAX_LEAF; calls on one GPU must not overlap)."""
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
        self.noalloc = bool(noalloc)
        self.tuning = tuning
        self.ws = None
        if not self.noalloc:
            nb = self.L.vx_lod_workspace_size(leaf.cap, self.levels, self.K)
            if nb == 0:
                raise VxError(1, "vx_lod_workspace_size")
            self.ws = _ws(nb, dev)

    def run(self, stream=None):
        if self.noalloc:
            st = self.L.vx_build_lod_noalloc(ctypes.byref(self.cgrid), ctypes.byref(self._cleaf),
                                             _ptr(self.n_leaf_dev), self.levels, self.K, self.iters, self._cout,
                                             self._clobes, _ptr(self.n_levels), _ctuning(self.tuning),
                                             _stream(stream))
        else:
            st = self.L.vx_build_lod(ctypes.byref(self.cgrid), ctypes.byref(self._cleaf), _ptr(self.n_leaf_dev),
                                     self.levels, self.K, self.iters, self._cout, self._clobes, _ptr(self.n_levels),
                                     _ptr(self.ws), self.ws.numel(), _ctuning(self.tuning), _stream(stream))
        if st != 0:
            raise VxError(st, "build_lod_noalloc" if self.noalloc else "build_lod")
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


SGGXH_SAMPLES = 5000


class SggxhPlan:
    """The paper's SGGX-H lobes (Sec. 4.4) over the pyramid `lod` (a LodPlan, run and checked):
    up to K lobes per voxel of levels 1 .. levels-1, merged by the histogram distance.  ``run()``
    enqueues all levels with no host sync; ``check()`` returns the Lobes of levels 1 ..."""

    def __init__(self, lod, K=4, samples=SGGXH_SAMPLES):
        import torch
        self.L = load()
        self.lod, self.K, self.samples = lod, int(K), int(samples)
        dev = lod.leaf.w.device
        self.lobes = [Lobes(torch.zeros(v.cap, dtype=torch.uint8, device=dev),
                            torch.zeros((self.K, v.cap), dtype=torch.float32, device=dev),
                            torch.zeros((6, self.K, v.cap), dtype=torch.float32, device=dev)) for v in lod.out]
        self._clobes = (CLobes * max(1, len(self.lobes)))(*[lb.cstruct() for lb in self.lobes])
        self._cleaf = lod.leaf.cstruct()
        self._cout = (CVoxels * max(1, len(lod.out)))(*[v.cstruct() for v in lod.out])
        self.stats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=dev)

    def run(self, stream=None):
        st = self.L.vx_build_sggxh(ctypes.byref(self.lod.cgrid), ctypes.byref(self._cleaf), self._cout,
                                   _ptr(self.lod.n_levels), self.lod.levels, self.K, self.samples, self._clobes,
                                   _ptr(self.stats), _stream(stream))
        if st != 0:
            raise VxError(st, "build_sggxh")
        return self

    def check(self, stream=None):
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        if st != 0:
            raise VxError(st, "build_sggxh")
        n = self.lod.n_levels.cpu().numpy()
        for L, lb in enumerate(self.lobes, start=1):
            lb.n = int(n[L])
        return self.lobes


@dataclass
class Occupancy:
    """Sub-cell occupancy of one level: mask int64 [8, cap] (uint64 bit patterns; word w of voxel
    i at mask[w, i]), hits int16 [4, cap] (hit sub-cells, XY, XZ, YZ cells)."""
    mask: object
    hits: object
    n: int = -1

    @property
    def cap(self):
        return int(self.mask.shape[1])

    def cstruct(self) -> COccupancy:
        return COccupancy(self.mask.data_ptr(), self.hits.data_ptr(), self.cap)

    def numpy(self, n=None):
        n = self.n if n is None else n
        m = self.mask[:, :n].cpu().numpy().view(np.uint64).T.copy()
        h = self.hits[:, :n].cpu().numpy().astype(np.int64)
        return {"mask": m, "hits": h[0], "xy": h[1], "xz": h[2], "yz": h[3]}


class OccupancyPlan:
    """Sub-voxel occupancy (Sec. 3.5, Sec. 4.2) of the pyramid `lod` (a LodPlan, run and
    checked) built from these primitives.  Candidate and pair capacities come from two counting
    calls; ``run()`` then enqueues the pass with no host sync."""

    def __init__(self, kind, grid, data, lod, offsets=None, radius=0.0, max_cand=None, max_pairs=None):
        import torch
        self.L = load()
        self.kind, self.grid, self.cgrid = kind, grid, _cgrid(grid)
        self.data = data.contiguous()
        self.device = self.data.device
        if kind == 0:
            self.n_prims, self.offsets, self.n_fib = int(self.data.numel() // 9), None, 0
        else:
            self.n_prims = int(self.data.numel() // 3)
            self.offsets = offsets.to(device=self.device, dtype=torch.int64).contiguous()
            self.n_fib = int(self.offsets.numel() - 1)
        self.radius = float(radius)
        self.lod = lod
        self.levels = lod.levels
        self.stats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.device)
        caps = [lod.leaf.cap] + [v.cap for v in lod.out]
        self.occ = [Occupancy(torch.empty((8, c), dtype=torch.int64, device=self.device),
                              torch.empty((4, c), dtype=torch.int16, device=self.device)) for c in caps]
        self._cocc = (COccupancy * len(self.occ))(*[o.cstruct() for o in self.occ])
        self._cleaf = lod.leaf.cstruct()
        self._cout = (CVoxels * max(1, len(lod.out)))(*[v.cstruct() for v in lod.out])
        if max_cand is None or max_pairs is None:
            mc, mp = 0 if max_cand is None else int(max_cand), 0
            for step in range(2):
                if step == 0 and max_cand is not None:
                    continue
                ws = self._ws_for(mc, mp)
                self._call(mc, mp, ws, _stream())
                self.L.vx_check_stats(_ptr(self.stats), _stream())
                h = self.stats.cpu().numpy()
                if h[STAT_FLAGS] & (FLAG_INPUT | FLAG_OFFSETS):
                    raise VxError(4, "occupancy")
                if step == 0:
                    mc = int(h[STAT_CAND])
                else:
                    mp = int(h[STAT_PAIRS])
                del ws
            max_cand = mc if max_cand is None else max_cand
            max_pairs = mp if max_pairs is None else max_pairs
        self.max_cand, self.max_pairs = int(max_cand), int(max_pairs)
        self.ws = self._ws_for(self.max_cand, self.max_pairs)

    def _ws_for(self, max_cand, max_pairs):
        nb = self.L.vx_occupancy_workspace_size(self.kind, self.n_prims, max_cand, max_pairs, int(self.grid.log2_res))
        if nb == 0:
            raise VxError(1, "vx_occupancy_workspace_size")
        return _ws(nb, self.device)

    def _call(self, max_cand, max_pairs, ws, stream):
        if self.kind == 0:
            st = self.L.vx_occupancy_triangles(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                               ctypes.byref(self._cleaf), self._cout, _ptr(self.lod.n_levels),
                                               self.levels, max_cand, max_pairs, self._cocc, _ptr(ws), ws.numel(),
                                               _ptr(self.stats), stream)
        else:
            st = self.L.vx_occupancy_fibers(ctypes.byref(self.cgrid), _ptr(self.data), self.n_prims,
                                            _ptr(self.offsets), self.n_fib, self.radius, ctypes.byref(self._cleaf),
                                            self._cout, _ptr(self.lod.n_levels), self.levels, max_cand, max_pairs,
                                            self._cocc, _ptr(ws), ws.numel(), _ptr(self.stats), stream)
        if st != 0:
            raise VxError(st, "occupancy")

    def run(self, stream=None):
        self._call(self.max_cand, self.max_pairs, self.ws, _stream(stream))
        return self

    def check(self, stream=None):
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        h = self.stats.cpu().numpy()
        if st != 0:
            raise VxError(st, f"occupancy (stats {h.tolist()})")
        n = self.lod.n_levels.cpu().numpy()
        for L, o in enumerate(self.occ):
            o.n = int(n[L])
        self.n_pairs = int(h[STAT_PAIRS])
        return self.occ


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


def build_lod(grid, leaf: Voxels, levels, K=1, iters=2, n_leaf_dev=None, caps=None, return_lobes=False, tuning=None):
    """Leaf voxels -> list [leaf, level 1, ..., level levels-1] (Sec. 4.3); with K > 1 and
    return_lobes, also the per-level lobes [level 1, ...] (Sec. 4.4)."""
    import torch
    if n_leaf_dev is None:
        n_leaf_dev = torch.tensor([leaf.n], dtype=torch.int64, device=leaf.w.device)
    p = LodPlan(grid, leaf, n_leaf_dev, levels, K, iters, caps, tuning=tuning).run()
    out = p.check()
    if return_lobes:
        return out, p.lobes
    return out


def _count_dev(n, cap, device):
    import torch
    if n is None:
        n = cap
    if isinstance(n, int):
        return torch.tensor([n], dtype=torch.int64, device=device)
    return n


def sggx_compact(w, S, n=None, eps=1e-3, vectors=True, stream=None):
    """Leaf eigen-fit and 6-byte SGGX code of the first n voxels (Sec. 4.1, Sec. 4.3).

    w: float32 [cap]; S: float32 [6, cap]; n: int or device int64 [1] (default cap).
    Returns (lam float32 [3, cap], vec float32 [9, cap] or None, code uint8 [cap, 6]).
    """
    import torch
    cap = int(w.shape[0])
    if S.shape != (6, cap) or w.dtype != torch.float32 or S.dtype != torch.float32:
        raise VxError(1, "sggx_compact: w [cap] and S [6, cap] float32")
    w, S = w.contiguous(), S.contiguous()
    n_dev = _count_dev(n, cap, w.device)
    lam = torch.empty((3, cap), dtype=torch.float32, device=w.device)
    vec = torch.empty((9, cap), dtype=torch.float32, device=w.device) if vectors else None
    code = torch.empty((cap, 6), dtype=torch.uint8, device=w.device)
    cv = CVoxels(None, None, w.data_ptr(), S.data_ptr(), None, cap)
    st = load().vx_sggx_compact(ctypes.byref(cv), _ptr(n_dev), float(eps), _ptr(lam), _ptr(vec), _ptr(code),
                                _stream(stream))
    if st != 0:
        raise VxError(st, "sggx_compact")
    return lam, vec, code


def sggx_decode(code, n=None, stream=None):
    """uint8 [cap, 6] codes -> float32 [6, cap] SGGX matrices (largest sigma about 1)."""
    import torch
    cap = int(code.shape[0])
    if code.shape != (cap, 6) or code.dtype != torch.uint8:
        raise VxError(1, "sggx_decode: code uint8 [cap, 6]")
    code = code.contiguous()
    n_dev = _count_dev(n, cap, code.device)
    S = torch.empty((6, cap), dtype=torch.float32, device=code.device)
    st = load().vx_sggx_decode(_ptr(code), _ptr(n_dev), cap, _ptr(S), _stream(stream))
    if st != 0:
        raise VxError(st, "sggx_decode")
    return S


def timing_enable(on=True):
    load().vx_timing_enable(1 if on else 0)


def timing_filter(name=None):
    """Time only launches named `name` (None: all)."""
    load().vx_timing_filter(name.encode() if name else None)


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


# ------------------------------------------------------------------------------------------------
# Differentiable two-lobe fit (vx_fit_forward / vx_fit_backward)
# ------------------------------------------------------------------------------------------------

def fit_dirs(ndir=128, device="cuda"):
    """Fibonacci directions on the sphere: z = 1 - (2k+1)/n, phi = k pi (3 - sqrt 5)."""
    import torch
    k = torch.arange(ndir, dtype=torch.float64)
    z = 1.0 - (2.0 * k + 1.0) / ndir
    phi = k * (np.pi * (3.0 - np.sqrt(5.0)))
    r = torch.sqrt(1.0 - z * z)
    return torch.stack([r * torch.cos(phi), r * torch.sin(phi), z], 1).to(torch.float32).to(device).contiguous()


class FitPlan:
    """Voxelize + K = 1 pyramid + two-lobe fit at levels lo..hi for one fiber set.

    Buffers are sized from a calibration run with 25 % slack.  The lobe parameters are bound to
    the calibration's voxels: row r of level L belongs to the voxel at index r of that level.  If
    control points move so that a fitted level gains, loses or changes voxels, the library flags
    it (the kernels never leave the parameter rows) and ``check()`` raises VxError
    (VX_ERR_CAPACITY for a changed count, VX_ERR_BINDING for changed keys); a run that outgrows the
    buffers also raises VX_ERR_CAPACITY."""

    def __init__(self, grid, pts, offsets, radius, lo=1, hi=6, ndir=128, slack=1.25, dirs=None):
        """dirs: the direction set [ndir, 3] (float32 values), or None for ``fit_dirs(ndir)``."""
        import torch
        self.L = load()
        self.grid, self.cgrid, self.lo, self.hi = grid, _cgrid(grid), int(lo), int(hi)
        self.pts = pts.detach().contiguous().clone()
        self.offsets = offsets.to(device=self.pts.device, dtype=torch.int64).contiguous()
        self.radius = float(radius)
        cal = VoxelizePlan(1, grid, self.pts, offsets=self.offsets, radius=radius)
        cal.run()
        cal.check()
        mc = int(cal.n_cand * slack) + 64
        mp = int(cal.n_pairs * slack) + 64
        self.vox = VoxelizePlan(1, grid, self.pts, offsets=self.offsets, radius=radius,
                                max_records=int(cal.max_records * slack) + 64,
                                max_units=int(cal.max_units * slack) + 64, out_cap=int(cal.out.n * slack) + 64)
        del cal
        self.vox.run()
        leaf = self.vox.check()
        lodc = LodPlan(grid, leaf, self.vox.stats[2:3], self.hi + 1).run()
        counts = [v.n for v in lodc.check()]
        del lodc
        self.lod = LodPlan(grid, leaf, self.vox.stats[2:3], self.hi + 1,
                           caps=[int(max(c, 1) * slack) + 64 for c in counts[1:]])
        self.counts = counts                                    # voxels per level at calibration
        self.lod.run()
        self.lod.check()
        self.levels = [leaf] + self.lod.out
        self._clevels = (CVoxels * (self.hi + 1))(*[v.cstruct() for v in self.levels])
        self._caps = (ctypes.c_int64 * (self.hi + 1))(*[v.cap for v in self.levels])
        # the parameters' binding: row counts and the keys of the fitted levels at calibration
        nfit = self.hi - self.lo + 1
        self._rows = (ctypes.c_int64 * nfit)(*[counts[L] for L in range(self.lo, self.hi + 1)])
        self.bound_keys = [self.levels[L].keys[:max(counts[L], 1)].clone() for L in range(self.lo, self.hi + 1)]
        self._bound = (ctypes.c_void_p * nfit)(*[k.data_ptr() for k in self.bound_keys])
        if dirs is None:
            self.dirs = fit_dirs(ndir, self.pts.device)
        else:
            self.dirs = torch.as_tensor(dirs, dtype=torch.float32).to(self.pts.device).reshape(-1, 3).contiguous()
            ndir = self.dirs.shape[0]
            if not 1 <= ndir <= 256:
                raise VxError(1, "fit: 1 to 256 directions")
        self.ndir = int(ndir)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.pts.device)
        self.fstats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.pts.device)
        self.bstats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.pts.device)
        nb = self.L.vx_fit_workspace_size(int(self.pts.shape[0]), mc, mp, self._caps, self.hi, int(grid.log2_res))
        if nb == 0:
            raise VxError(1, "vx_fit_workspace_size")
        self.ws = _ws(nb, self.pts.device)
        self.max_cand, self.max_pairs = mc, mp
        self.dpts = torch.zeros_like(self.pts)
        self.run_id = 0                                         # forwards evaluated on this plan

    def param_shapes(self):
        return [(self.counts[L], 12) for L in range(self.lo, self.hi + 1)]

    def _ptrs(self, tensors):
        return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])

    def _params(self, params):
        import torch
        params = [p.contiguous() for p in params]
        if len(params) != self.hi - self.lo + 1:
            raise VxError(1, "fit: one parameter tensor per fitted level")
        for L, p in zip(range(self.lo, self.hi + 1), params):
            if tuple(p.shape) != (self.counts[L], 12) or p.dtype != torch.float32 or p.device != self.pts.device:
                raise VxError(1, f"fit: level {L} parameters must be float32 [{self.counts[L]}, 12]")
        return params

    def forward(self, pts, params, stream=None, check=True):
        """Voxelize the (possibly moved) points, build the pyramid, evaluate the fit loss.  With
        check, synchronise and raise if the fitted levels no longer match the parameters."""
        params = self._params(params)
        self.pts.copy_(pts.detach())
        self.vox.run(stream)
        self.lod.run(stream)
        st = self.L.vx_fit_forward(ctypes.byref(self.cgrid), self._clevels, _ptr(self.lod.n_levels), self.lo, self.hi,
                                   self._ptrs(params), self._rows, self._bound, _ptr(self.dirs), self.ndir,
                                   _ptr(self.loss), _ptr(self.fstats), self._caps, _ptr(self.ws), self.ws.numel(),
                                   _stream(stream))
        if st != 0:
            raise VxError(st, "vx_fit_forward")
        self.run_id += 1
        if check:
            self.check_forward(stream)
        return self.loss

    def check_forward(self, stream=None):
        """Synchronise and raise if the last forward outgrew a buffer or lost the binding."""
        self.vox.check(stream)
        self.lod.check()
        st = self.L.vx_check_stats(_ptr(self.fstats), _stream(stream))
        if st != 0:
            raise VxError(st, "vx_fit_forward")

    def backward(self, dloss, params, stream=None):
        import torch
        params = self._params(params)
        dparams = [torch.empty_like(p) for p in params]
        fib = CFibers(self.pts.data_ptr(), int(self.pts.shape[0]), self.offsets.data_ptr(),
                      int(self.offsets.numel() - 1), self.radius)
        st = self.L.vx_fit_backward(ctypes.byref(self.cgrid), ctypes.byref(fib), self.max_cand, self.max_pairs,
                                    self._clevels, _ptr(self.lod.n_levels), self.lo, self.hi, self._ptrs(params),
                                    self._rows, self._bound, _ptr(self.dirs), self.ndir, _ptr(dloss),
                                    self._ptrs(dparams), _ptr(self.dpts), _ptr(self.bstats), self._caps,
                                    _ptr(self.ws), self.ws.numel(), _stream(stream))
        if st != 0:
            raise VxError(st, "vx_fit_backward")
        return self.dpts.clone(), dparams

    def check(self, stream=None):
        """Synchronise and raise if a buffer was outgrown or the parameters lost their voxels."""
        self.check_forward(stream)
        st = self.L.vx_check_stats(_ptr(self.bstats), _stream(stream))
        if st != 0:
            raise VxError(st, "vx_fit_backward")


def _make_lobe_fit():
    import torch

    class LobeFit(torch.autograd.Function):
        """loss = LobeFit.apply(plan, pts, *params): the two-lobe fit loss with hand-written
        backward kernels for the lobes (params, one [n_L, 12] tensor per level) and the control
        points.  The plan holds one forward state (its points and pyramid); a backward after
        another forward on the same plan raises instead of differentiating the wrong state."""

        @staticmethod
        def forward(ctx, plan, pts, *params):
            loss = plan.forward(pts, params)
            ctx.plan = plan
            ctx.run_id = plan.run_id
            ctx.save_for_backward(*params)
            return loss[0].clone()

        @staticmethod
        def backward(ctx, gloss):
            if ctx.plan.run_id != ctx.run_id:
                raise RuntimeError("lobe_fit: the plan ran another forward after this loss; backward would "
                                   "differentiate that later state (use one FitPlan per live loss)")
            params = ctx.saved_tensors
            g = gloss.reshape(1).to(torch.float32).contiguous()
            dpts, dparams = ctx.plan.backward(g, params)
            ctx.plan.check()
            return (None, dpts, *dparams)

    return LobeFit


_LobeFit = None


def lobe_fit(plan, pts, params):
    """Differentiable fit loss (a torch scalar on the GPU)."""
    global _LobeFit
    if _LobeFit is None:
        _LobeFit = _make_lobe_fit()
    return _LobeFit.apply(plan, pts, *params)


def fit_init(plan, seed=4, noise=0.01):
    """Initial lobes per fitted voxel: 0.5 chol(S/w + 0.05 I) + N(0, noise^2) for both lobes
    (zeros where w = 0), computed on the GPU from the plan's current pyramid."""
    import torch
    g = torch.Generator(device=plan.pts.device)
    g.manual_seed(seed)
    out = []
    for L in range(plan.lo, plan.hi + 1):
        v = plan.levels[L]
        n = plan.counts[L]
        w = v.w[:n].double()
        S = v.S[:, :n].double()
        Sb = torch.where(w > 0, S / w.clamp_min(1e-30), torch.zeros_like(S))
        M = torch.zeros((n, 3, 3), dtype=torch.float64, device=w.device)
        idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        for c, (i, j) in enumerate(idx):
            M[:, i, j] = Sb[c]
            M[:, j, i] = Sb[c]
        M = M + 0.05 * torch.eye(3, dtype=torch.float64, device=w.device)
        C = 0.5 * torch.linalg.cholesky(M)
        row = torch.stack([C[:, 0, 0], C[:, 1, 0], C[:, 1, 1], C[:, 2, 0], C[:, 2, 1], C[:, 2, 2]], 1)
        row = torch.where((w > 0)[:, None], row, torch.zeros_like(row))
        P = torch.cat([row, row], 1)
        P = P + noise * torch.randn(P.shape, generator=g, device=w.device, dtype=torch.float64)
        out.append(P.to(torch.float32).contiguous())
    return out


# ------------------------------------------------------------------------------------------------
# Launch geometry and graphs
# ------------------------------------------------------------------------------------------------

class Graph:
    """A captured sequence of library calls on one (non-null) stream, replayed as one launch."""

    def __init__(self, handle, stream):
        self.handle, self.stream = handle, stream

    def replay(self, stream=None):
        st = load().vx_graph_launch(self.handle, _stream(stream if stream is not None else self.stream))
        if st != 0:
            raise VxError(st, "vx_graph_launch")

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vx_graph_destroy(self.handle)
            self.handle = None


def capture(fn, stream):
    """Capture everything ``fn(stream)`` enqueues on ``stream`` into a Graph.  Kernel timing must
    be off; the buffers used by ``fn`` must stay alive as long as the graph."""
    L = load()
    cs = _stream(stream)
    st = L.vx_graph_begin(cs)
    if st != 0:
        raise VxError(st, "vx_graph_begin")
    try:
        fn(stream)
    finally:
        h = ctypes.c_void_p()
        st2 = L.vx_graph_end(cs, ctypes.byref(h))
    if st2 != 0:
        raise VxError(st2, "vx_graph_end")
    return Graph(h, stream)


# ------------------------------------------------------------------------------------------------
# Batched patches (vx_batch_build)
# ------------------------------------------------------------------------------------------------

PATCH_SHIFT = 33


@dataclass
class Patch:
    """One fiber patch of a batch: its own grid, points [n, 3] (float32, GPU), local CSR
    offsets [F + 1] and radius."""
    grid: object
    pts: object
    offsets: object
    radius: float


class BatchPlan:
    """Many fiber patches voxelized and LoD-built by one batched call (one pass of every kernel
    over all patches' primitives), optionally captured into a graph.

    ``levels`` defaults to the deepest patch's full pyramid; a shallower patch keeps its root
    voxel on the levels above it.  Capacities come from counting calls of the same entry point
    (candidates, pairs, leaf voxels, then per-level counts), synchronising once per call."""

    def __init__(self, patches, K=4, iters=2, levels=None, device=None, tuning=None):
        import torch
        self.L = load()
        self.tuning = tuning
        self.patches = list(patches)
        self.n_patches = len(self.patches)
        if self.n_patches < 1:
            raise ValueError("a batch needs at least one patch")
        dev = device if device is not None else self.patches[0].pts.device
        self.device = torch.device(dev)
        pts, offs, cp = [], [], (CPatch * self.n_patches)()
        base_pt, base_fib = 0, 0
        for i, P in enumerate(self.patches):
            p = P.pts.to(device=self.device, dtype=torch.float32).reshape(-1, 3)
            o = torch.as_tensor(P.offsets).to(device=self.device, dtype=torch.int64).reshape(-1)
            n = int(p.shape[0])
            pts.append(p)
            offs.append(o[1:] + base_pt if i else o + base_pt)
            cp[i].grid = _cgrid(P.grid)
            cp[i].pt_begin, cp[i].pt_end = base_pt, base_pt + n
            cp[i].radius = float(P.radius)
            base_pt += n
            base_fib += int(o.numel() - 1)
        self.pts = torch.cat(pts).contiguous()
        self.offsets = torch.cat(offs).contiguous()
        self.n_pts, self.n_fib = int(self.pts.shape[0]), int(self.offsets.numel() - 1)
        self._cp = cp
        self.patches_dev = torch.frombuffer(bytearray(bytes(cp)), dtype=torch.uint8).to(self.device)
        self.levels = int(levels) if levels is not None else max(P.grid.log2_res for P in self.patches) + 1
        self.K, self.iters = int(K), int(iters)
        self.stats = torch.zeros(VX_NSTAT, dtype=torch.int64, device=self.device)
        self.n_levels = torch.zeros(self.levels + 1, dtype=torch.int64, device=self.device)
        self.patch_table = torch.zeros((self.levels, self.n_patches + 1), dtype=torch.int64, device=self.device)
        self._plan_capacities()

    # -- one call of the entry point ------------------------------------------------------------
    def _call(self, levels, K, max_records, max_units, cout, clobes, ws, stream):
        st = self.L.vx_batch_build(self._cp, _ptr(self.patches_dev), self.n_patches, _ptr(self.pts), self.n_pts,
                                   _ptr(self.offsets), self.n_fib, levels, K, self.iters, max_records, max_units, cout,
                                   clobes, _ptr(self.n_levels), _ptr(self.patch_table), _ptr(self.stats), _ptr(ws),
                                   ws.numel(), _ctuning(self.tuning), stream)
        if st != 0:
            raise VxError(st, "vx_batch_build")

    def _ws_for(self, max_records, max_units, leaf_cap):
        nb = self.L.vx_batch_workspace_size(self.n_patches, self.n_pts, max_records, max_units, leaf_cap)
        if nb == 0:
            raise VxError(1, "vx_batch_workspace_size")
        return _ws(nb, self.device)

    def _stats(self, s):
        self.L.vx_check_stats(_ptr(self.stats), s)
        h = self.stats.cpu().numpy()
        if h[STAT_FLAGS] & (FLAG_INPUT | FLAG_OFFSETS):
            raise VxError(4, "vx_batch_build")
        return h

    def _plan_capacities(self):
        import torch
        s = _stream()
        one = alloc_voxels(1, 11, self.device, False)
        c1 = (CVoxels * 1)(one.cstruct())
        ws = self._ws_for(0, 0, 1)
        self._call(1, 1, 0, 0, c1, None, ws, s)
        n_rec = int(self._stats(s)[STAT_RECORDS])
        ws = self._ws_for(n_rec, 0, 1)
        self._call(1, 1, n_rec, 0, c1, None, ws, s)
        n_units = int(self._stats(s)[STAT_UNITS])
        del ws
        ws = self._ws_for(n_rec, n_units, 1)
        self._call(1, 1, n_rec, n_units, c1, None, ws, s)
        n_leaf = max(1, int(self._stats(s)[STAT_VOXELS]))
        del ws
        # per-level counts: K = 1, two level buffers of the leaf's size used in turn
        leaf = alloc_voxels(n_leaf, 11, self.device, False)
        ping = [alloc_voxels(n_leaf, 11, self.device, True) for _ in range(min(2, self.levels - 1))]
        cl = [leaf] + [ping[(L - 1) % 2] for L in range(1, self.levels)]
        cout = (CVoxels * self.levels)(*[v.cstruct() for v in cl])
        ws = self._ws_for(n_rec, n_units, n_leaf)
        self._call(self.levels, 1, n_rec, n_units, cout, None, ws, s)
        self._stats(s)
        torch.cuda.synchronize()
        counts = [int(x) for x in self.n_levels[:self.levels].cpu()]
        del leaf, ping, cl, cout, ws
        self.max_records, self.max_units, self.counts = n_rec, n_units, counts
        self.out = [alloc_voxels(max(c, 1), 11, self.device, L > 0) for L, c in enumerate(counts)]
        self._cout = (CVoxels * self.levels)(*[v.cstruct() for v in self.out])
        self.lobes, self._clobes = [], None
        if self.K > 1 and self.levels > 1:
            self.lobes = [Lobes(torch.empty(v.cap, dtype=torch.uint8, device=self.device),
                                torch.empty((self.K, v.cap), dtype=torch.float32, device=self.device),
                                torch.empty((6, self.K, v.cap), dtype=torch.float32, device=self.device))
                          for v in self.out[1:]]
            self._clobes = (CLobes * len(self.lobes))(*[lb.cstruct() for lb in self.lobes])
        self.ws = self._ws_for(n_rec, n_units, self.out[0].cap)

    # -- hot path -------------------------------------------------------------------------------
    def run(self, stream=None):
        self._call(self.levels, self.K, self.max_records, self.max_units, self._cout, self._clobes, self.ws,
                   _stream(stream))
        return self

    def capture(self, stream):
        """Graph of one whole batched build on ``stream`` (a torch.cuda.Stream, not the default)."""
        return capture(lambda st: self.run(st), stream)

    def check(self, stream=None):
        """Synchronise, raise on a capacity or input flag, and fetch counts and patch tables."""
        import torch
        st = self.L.vx_check_stats(_ptr(self.stats), _stream(stream))
        h = self.stats.cpu().numpy()
        if st != 0:
            raise VxError(st, f"vx_batch_build (stats {h.tolist()})")
        torch.cuda.synchronize()
        nl = self.n_levels.cpu().numpy()
        if nl[self.levels] & FLAG_VOXEL_CAPACITY:
            raise VxError(2, "vx_batch_build")
        for L in range(self.levels):
            self.out[L].n = int(nl[L])
            if L > 0 and self.lobes:
                self.lobes[L - 1].n = int(nl[L])
        self.n_pairs, self.n_cand = int(h[STAT_PAIRS]), int(h[STAT_CAND])
        self.table = self.patch_table.cpu().numpy()
        return self

    def patch_level(self, p, L):
        """Host copy of patch p's voxels at level L (keys without the patch bits; with K > 1 and
        L > 0 also 'nl', 'lw', 'lS' lobes)."""
        a, b = int(self.table[L, p]), int(self.table[L, p + 1])
        v = self.out[L]
        k = v.keys[a:b].cpu().numpy().view(np.uint64) & np.uint64((1 << PATCH_SHIFT) - 1)
        out = {"keys": k, "count": v.count[a:b].cpu().numpy().view(np.uint32), "w": v.w[a:b].cpu().numpy(),
               "S": v.S[:, a:b].cpu().numpy().T.copy()}
        if v.mask is not None:
            out["mask"] = v.mask[a:b].cpu().numpy()
        if L > 0 and self.lobes:
            lb = self.lobes[L - 1]
            out["nl"] = lb.nl[a:b].cpu().numpy()
            out["lw"] = lb.w[:, a:b].cpu().numpy().T.copy()
            out["lS"] = lb.S[:, :, a:b].cpu().numpy().transpose(2, 1, 0).copy()
        return out
