"""Python binding of libgsmfma, an MI355X (gfx950) tile-based Gaussian
splatting rasteriser.

Argument marshalling only: every step of the rendering path runs in the HIP
kernels of ``libgsmfma.so``.  PyTorch provides device memory and the current
stream.  There is no CPU fallback: when the library is missing or no GPU is
present the calls raise.

Entry points mirror the C ABI in ``include/gs.h``:

* :func:`preprocess` / :func:`preprocess_2d` -- projection (TC-GS Sec. 3.1)
* :func:`bin_sort` -- per-tile depth-ordered splat lists (Sec. 3.1)
* :func:`rasterize_fwd` -- Algorithm 1 with the exponent computed per
  ``precision`` (plain FP32, EarlyCull, Frag2Mat on FP16/BF16 matrix cores
  with G2L local coordinates, Sec. 4)
* :func:`rasterize_beta` -- diagnostic dump of the exponent matrix B
* :func:`render` -- the three stages chained
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_size_t, c_uint32, c_void_p

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgsmfma.so")

TILE = 16

GS_MAX_BIN_VIEWS = 64  # views one gs_bin_sort_multiview call serves

PRECISIONS = {
    "fp32": 0,
    "fp32_earlycull": 1,
    "fp16_global": 2,
    "fp16_g2l": 3,
    "fp16_g2l_split": 4,
    "bf16_g2l_split": 5,
    # ablation only (one-view forward): the FP16 split without EarlyCull
    "fp16_g2l_split_nocull": 6,
}

STATUS = {0: "GS_OK", 1: "GS_ERR_INVALID_ARG", 2: "GS_ERR_UNSUPPORTED", 3: "GS_ERR_HIP",
          4: "GS_ERR_CAPACITY", 5: "GS_ERR_NOT_IMPLEMENTED"}


class GSError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)}")
        self.status = status


class gs_camera(ctypes.Structure):
    _fields_ = [("viewmat", c_float * 16), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32), ("near_z", c_float),
                ("frustum_guard", c_float), ("lowpass", c_float), ("campos", c_float * 3)]


class gs_view(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("tile_ranges", c_void_p),
                ("sorted_ids", c_void_p), ("means2d", c_void_p), ("conics", c_void_p),
                ("log_opacities", c_void_p), ("rgb", c_void_p), ("background", c_float * 3),
                ("out_rgb", c_void_p), ("out_T", c_void_p), ("out_ncontrib", c_void_p)]


class gs_batch_tune(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("blocks_per_cu", c_int32), ("xcd_queues", c_int32)]

    def as_tuple(self):
        return (self.batch, self.blocks_per_cu, self.xcd_queues)


class gs_raster_tune(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("chunk_rows", c_int32)]

    def as_tuple(self):
        return (self.batch, self.chunk_rows)


def make_raster_tune(batch=128, chunk_rows=2) -> gs_raster_tune:
    """Launch shape of the one-view rasteriser (gs_rasterize_fwd_tuned)."""
    t = gs_raster_tune()
    t.batch, t.chunk_rows = int(batch), int(chunk_rows)
    return t


def make_tune(batch=256, blocks_per_cu=5, xcd_queues=1) -> gs_batch_tune:
    return gs_batch_tune(int(batch), int(blocks_per_cu), int(xcd_queues))


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgsmfma.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2505_24796_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp = c_void_p
        L.gs_status_string.restype = ctypes.c_char_p
        L.gs_status_string.argtypes = [ctypes.c_int]
        L.gs_version.restype = ctypes.c_int
        L.gs_preprocess.restype = ctypes.c_int
        L.gs_preprocess.argtypes = [c_int32, vp, vp, vp, vp, vp, c_int32, POINTER(gs_camera),
                                    vp, vp, vp, vp, vp, vp, vp, vp]
        L.gs_preprocess_2d.restype = ctypes.c_int
        L.gs_preprocess_2d.argtypes = [c_int32, vp, vp, vp, c_int32, c_int32, vp, vp, vp, vp, vp]
        L.gs_bin_sort_workspace_bytes.restype = c_size_t
        L.gs_bin_sort_workspace_bytes.argtypes = [c_int32, c_uint32, c_int32, c_int32]
        L.gs_bin_sort.restype = ctypes.c_int
        L.gs_bin_sort.argtypes = [c_int32, vp, vp, vp, c_int32, c_int32, c_uint32, vp, c_size_t,
                                  vp, vp, vp, vp]
        L.gs_bin_sort_noalloc.restype = ctypes.c_int
        L.gs_bin_sort_noalloc.argtypes = [c_int32, vp, vp, vp, c_int32, c_int32, c_uint32, vp, vp,
                                          vp, vp]
        L.gs_rasterize_fwd.restype = ctypes.c_int
        L.gs_rasterize_fwd.argtypes = [c_int32, c_int32, vp, vp, vp, vp, vp, vp,
                                       POINTER(c_float), c_int32, vp, vp, vp, vp, vp]
        L.gs_rasterize_fwd_tuned.restype = ctypes.c_int
        L.gs_rasterize_fwd_tuned.argtypes = [c_int32, c_int32, vp, vp, vp, vp, vp, vp,
                                             POINTER(c_float), c_int32, POINTER(gs_raster_tune),
                                             vp, vp, vp, vp, vp]
        L.gs_rasterize_bwd.restype = ctypes.c_int
        L.gs_rasterize_bwd.argtypes = [c_int32, c_int32, vp, vp, vp, vp, vp, vp, POINTER(c_float),
                                       c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.gs_rasterize_beta.restype = ctypes.c_int
        L.gs_rasterize_beta.argtypes = [c_int32, c_int32, c_int32, vp, vp, vp, vp, vp, c_int32,
                                        c_int32, vp, vp]
        L.gs_bin_sort_precise_workspace_bytes.restype = c_size_t
        L.gs_bin_sort_precise_workspace_bytes.argtypes = [c_int32, c_uint32, c_int32, c_int32]
        L.gs_bin_sort_precise.restype = ctypes.c_int
        L.gs_bin_sort_precise.argtypes = [c_int32, vp, vp, vp, vp, vp, c_int32, c_int32, c_uint32,
                                          vp, c_size_t, vp, vp, vp, vp]
        L.gs_bin_sort_multiview_workspace_bytes.restype = c_size_t
        L.gs_bin_sort_multiview_workspace_bytes.argtypes = [c_int32, c_int32, c_uint32,
                                                            POINTER(c_int32), POINTER(c_int32),
                                                            c_int32]
        L.gs_bin_sort_multiview.restype = ctypes.c_int
        L.gs_bin_sort_multiview.argtypes = [c_int32, c_int32, POINTER(c_int32), POINTER(c_int32),
                                            vp, vp, vp, vp, vp, c_int32, c_uint32, vp, c_size_t,
                                            vp, vp, vp, vp, vp]
        L.gs_preprocess_multiview.restype = ctypes.c_int
        L.gs_preprocess_multiview.argtypes = [c_int32, vp, vp, vp, vp, vp, c_int32, c_int32,
                                              POINTER(gs_camera), vp, vp, vp, vp, vp, vp, vp, vp]
        L.gs_batch_plan_bytes.restype = c_size_t
        L.gs_batch_plan_bytes.argtypes = [c_int32]
        L.gs_batch_workspace_bytes.restype = c_size_t
        L.gs_batch_workspace_bytes.argtypes = [c_int32]
        L.gs_batch_plan_write.restype = ctypes.c_int
        L.gs_batch_plan_write.argtypes = [c_int32, POINTER(gs_view), vp, c_size_t]
        L.gs_rasterize_fwd_batched.restype = ctypes.c_int
        L.gs_rasterize_fwd_batched.argtypes = [c_int32, vp, c_int32, POINTER(gs_batch_tune), vp,
                                               c_size_t, vp, vp]
        L.gs_peak_probe.restype = ctypes.c_int
        L.gs_peak_probe.argtypes = [c_int32, c_int32, c_int32, vp, vp]
        L.gs_clock_stamp.restype = ctypes.c_int
        L.gs_clock_stamp.argtypes = [vp, vp]
        L.gs_wall_clock_khz.restype = ctypes.c_int
        L.gs_wall_clock_khz.argtypes = [POINTER(c_int32)]
        _lib = L
    return _lib


def _check(fn: str, status: int):
    if status != 0:
        raise GSError(fn, status)


def _ptr(t):
    return c_void_p(0) if t is None else c_void_p(t.data_ptr())


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def grid(width: int, height: int):
    return (width + TILE - 1) // TILE, (height + TILE - 1) // TILE


def make_camera(viewmat, fx, fy, cx, cy, width, height, near_z=0.2, frustum_guard=1.3,
                lowpass=0.3, campos=(0.0, 0.0, 0.0)) -> gs_camera:
    c = gs_camera()
    vm = [float(v) for v in (viewmat.reshape(-1).tolist() if hasattr(viewmat, "reshape") else viewmat)]
    c.viewmat[:] = vm
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.width, c.height = int(width), int(height)
    c.near_z, c.frustum_guard, c.lowpass = float(near_z), float(frustum_guard), float(lowpass)
    c.campos[:] = [float(v) for v in campos]
    return c


def preprocess(means3d, scales, quats, opacities, sh, cam: gs_camera, sh_degree: int = 3) -> dict:
    """gs_preprocess: means2d, conics, log_opacities (ln o), depths, radii,
    rgb, tiles_touched."""
    P = means3d.shape[0]
    f32 = torch.float32
    for n, t in (("means3d", means3d), ("scales", scales), ("quats", quats),
                 ("opacities", opacities), ("sh", sh)):
        _dev(t, f32, n)
    dev = means3d.device
    out = dict(means2d=torch.empty(P, 2, dtype=f32, device=dev),
               conics=torch.empty(P, 3, dtype=f32, device=dev),
               log_opacities=torch.empty(P, dtype=f32, device=dev),
               depths=torch.empty(P, dtype=f32, device=dev),
               radii=torch.empty(P, dtype=torch.int32, device=dev),
               rgb=torch.empty(P, 3, dtype=f32, device=dev),
               tiles_touched=torch.empty(P, dtype=torch.int32, device=dev))
    st = lib().gs_preprocess(P, _ptr(means3d), _ptr(scales), _ptr(quats), _ptr(opacities),
                             _ptr(sh), sh_degree, ctypes.byref(cam), _ptr(out["means2d"]),
                             _ptr(out["conics"]), _ptr(out["log_opacities"]),
                             _ptr(out["depths"]), _ptr(out["radii"]), _ptr(out["rgb"]),
                             _ptr(out["tiles_touched"]), _stream())
    _check("gs_preprocess", st)
    return out


def preprocess_2d(means2d, cov2d, opacities, width: int, height: int) -> dict:
    """gs_preprocess_2d: conics, log_opacities (ln o), radii, tiles_touched."""
    P = means2d.shape[0]
    _dev(means2d, torch.float32, "means2d")
    _dev(cov2d, torch.float32, "cov2d")
    _dev(opacities, torch.float32, "opacities")
    dev = means2d.device
    out = dict(conics=torch.empty(P, 3, dtype=torch.float32, device=dev),
               log_opacities=torch.empty(P, dtype=torch.float32, device=dev),
               radii=torch.empty(P, dtype=torch.int32, device=dev),
               tiles_touched=torch.empty(P, dtype=torch.int32, device=dev))
    st = lib().gs_preprocess_2d(P, _ptr(means2d), _ptr(cov2d), _ptr(opacities), width, height,
                                _ptr(out["conics"]), _ptr(out["log_opacities"]),
                                _ptr(out["radii"]), _ptr(out["tiles_touched"]), _stream())
    _check("gs_preprocess_2d", st)
    return out


class BinSorter:
    """Owns a workspace and output buffers for gs_bin_sort at a fixed
    (P, capacity, width, height); reusable across frames (no allocation per
    call).  With ``precise`` it runs gs_bin_sort_precise (then the call
    also takes the conics and ln o)."""

    def __init__(self, P: int, capacity: int, width: int, height: int, device="cuda",
                 workspace: torch.Tensor | None = None, precise: bool = False):
        self.P, self.capacity, self.width, self.height = P, int(capacity), width, height
        self.precise = bool(precise)
        wsb = (lib().gs_bin_sort_precise_workspace_bytes if self.precise
               else lib().gs_bin_sort_workspace_bytes)
        nbytes = wsb(P, self.capacity, width, height)
        if nbytes == 0:
            raise ValueError("invalid bin_sort sizes")
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        elif workspace.numel() < nbytes or workspace.dtype != torch.uint8:
            raise ValueError(f"shared workspace needs {nbytes} uint8 bytes")
        # a shared workspace serves several sorters whose calls are ordered on
        # one stream
        self.workspace = workspace
        gx, gy = grid(width, height)
        self.sorted_ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.ranges = torch.empty(gx * gy, 2, dtype=torch.int32, device=device)
        self.num_splats = torch.zeros(1, dtype=torch.int32, device=device)

    def __call__(self, means2d, radii, depths, conics=None, log_opacities=None):
        _dev(means2d, torch.float32, "means2d")
        _dev(radii, torch.int32, "radii")
        _dev(depths, torch.float32, "depths")
        if self.precise:
            if conics is None or log_opacities is None:
                raise ValueError("precise binning needs conics and log_opacities")
            _dev(conics, torch.float32, "conics")
            _dev(log_opacities, torch.float32, "log_opacities")
            st = lib().gs_bin_sort_precise(self.P, _ptr(means2d), _ptr(radii), _ptr(depths),
                                           _ptr(conics), _ptr(log_opacities), self.width,
                                           self.height,
                                           self.capacity, _ptr(self.workspace),
                                           self.workspace.numel(), _ptr(self.sorted_ids),
                                           _ptr(self.ranges), _ptr(self.num_splats), _stream())
            _check("gs_bin_sort_precise", st)
        else:
            st = lib().gs_bin_sort(self.P, _ptr(means2d), _ptr(radii), _ptr(depths), self.width,
                                   self.height, self.capacity, _ptr(self.workspace),
                                   self.workspace.numel(), _ptr(self.sorted_ids),
                                   _ptr(self.ranges), _ptr(self.num_splats), _stream())
            _check("gs_bin_sort", st)
        return self.sorted_ids, self.ranges, self.num_splats

    def n_splats(self) -> int:
        """Host read of the device splat count (synchronises)."""
        return int(self.num_splats.item()) & 0xFFFFFFFF


class MultiViewBinSorter:
    """gs_bin_sort_multiview at a fixed (views, P, capacity): the lists of
    every view in one call.  ``ranges(v)`` / ``sorted_ids`` are what a
    one-view rasterisation of view v takes; ``view_splats`` holds the
    per-view counts (device)."""

    def __init__(self, P: int, capacity: int, sizes, device="cuda", precise: bool = False):
        self.P, self.capacity, self.precise = P, int(capacity), bool(precise)
        self.sizes = [(int(w), int(h)) for w, h in sizes]
        self.V = len(self.sizes)
        self._w = (c_int32 * self.V)(*[w for w, _ in self.sizes])
        self._h = (c_int32 * self.V)(*[h for _, h in self.sizes])
        nbytes = lib().gs_bin_sort_multiview_workspace_bytes(self.V, P, self.capacity, self._w,
                                                             self._h, int(self.precise))
        if nbytes == 0:
            raise ValueError("invalid multi-view bin_sort sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        nt = [grid(w, h)[0] * grid(w, h)[1] for w, h in self.sizes]
        self.tile_base = [0]
        for n in nt:
            self.tile_base.append(self.tile_base[-1] + n)
        self.all_ranges = torch.empty(self.tile_base[-1], 2, dtype=torch.int32, device=device)
        self.sorted_ids = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.num_splats = torch.zeros(1, dtype=torch.int32, device=device)
        self.view_splats = torch.zeros(self.V, dtype=torch.int32, device=device)

    def ranges(self, v: int) -> torch.Tensor:
        return self.all_ranges[self.tile_base[v]:self.tile_base[v + 1]]

    def __call__(self, means2d, radii, depths, conics=None, log_opacities=None):
        """means2d [V, P, 2], radii [V, P], depths [V, P] (and, precise,
        conics [V, P, 3] and log_opacities [P])."""
        _dev(means2d, torch.float32, "means2d")
        _dev(radii, torch.int32, "radii")
        _dev(depths, torch.float32, "depths")
        if self.precise:
            if conics is None or log_opacities is None:
                raise ValueError("precise binning needs conics and log_opacities")
            _dev(conics, torch.float32, "conics")
            _dev(log_opacities, torch.float32, "log_opacities")
        st = lib().gs_bin_sort_multiview(self.V, self.P, self._w, self._h, _ptr(means2d),
                                         _ptr(radii), _ptr(depths),
                                         _ptr(conics) if self.precise else None,
                                         _ptr(log_opacities) if self.precise else None,
                                         int(self.precise), self.capacity, _ptr(self.workspace),
                                         self.workspace.numel(), _ptr(self.sorted_ids),
                                         _ptr(self.all_ranges), _ptr(self.num_splats),
                                         _ptr(self.view_splats), _stream())
        _check("gs_bin_sort_multiview", st)
        return self.sorted_ids, self.all_ranges, self.num_splats

    def n_splats(self) -> int:
        return int(self.num_splats.item()) & 0xFFFFFFFF

    def view_counts(self) -> list:
        return [int(x) & 0xFFFFFFFF for x in self.view_splats.cpu().tolist()]


def preprocess_multiview(means3d, scales, quats, opacities, sh, cams, sh_degree: int = 3,
                         out: dict | None = None) -> dict:
    """gs_preprocess for several cameras in one pass; every output has a
    leading view axis (V, P, ...) except log_opacities (P,)."""
    P, V = means3d.shape[0], len(cams)
    f32 = torch.float32
    for n, t in (("means3d", means3d), ("scales", scales), ("quats", quats),
                 ("opacities", opacities), ("sh", sh)):
        _dev(t, f32, n)
    dev = means3d.device
    if out is None:
        out = dict(means2d=torch.empty(V, P, 2, dtype=f32, device=dev),
                   conics=torch.empty(V, P, 3, dtype=f32, device=dev),
                   log_opacities=torch.empty(P, dtype=f32, device=dev),
                   depths=torch.empty(V, P, dtype=f32, device=dev),
                   radii=torch.empty(V, P, dtype=torch.int32, device=dev),
                   rgb=torch.empty(V, P, 3, dtype=f32, device=dev),
                   tiles_touched=torch.empty(V, P, dtype=torch.int32, device=dev))
    arr = (gs_camera * V)(*cams)
    st = lib().gs_preprocess_multiview(P, _ptr(means3d), _ptr(scales), _ptr(quats),
                                       _ptr(opacities), _ptr(sh), sh_degree, V, arr,
                                       _ptr(out["means2d"]), _ptr(out["conics"]),
                                       _ptr(out["log_opacities"]), _ptr(out["depths"]),
                                       _ptr(out["radii"]), _ptr(out["rgb"]),
                                       _ptr(out["tiles_touched"]), _stream())
    _check("gs_preprocess_multiview", st)
    return out


def bin_sort(means2d, radii, depths, width: int, height: int, capacity: int | None = None,
             conics=None, log_opacities=None, precise: bool = False):
    """One-shot binning.  Without ``capacity`` the splat count is computed by
    a first call with capacity 0 (one host synchronisation)."""
    P = means2d.shape[0]
    if capacity is None:
        probe = BinSorter(P, 0, width, height, device=means2d.device, precise=precise)
        probe(means2d, radii, depths, conics, log_opacities)
        capacity = max(probe.n_splats(), 1)
    bs = BinSorter(P, capacity, width, height, device=means2d.device, precise=precise)
    bs(means2d, radii, depths, conics, log_opacities)
    return bs


NOALLOC_SCRATCH_BYTES = 128 << 20  # GS_NOALLOC_SCRATCH_BYTES of gs.h


def bin_sort_noalloc(means2d, radii, depths, width: int, height: int, sorted_ids, ranges,
                     num_splats):
    """gs_bin_sort_noalloc into caller-owned outputs (sorted_ids int32
    [capacity], ranges int32 [tiles][2], num_splats int32 [1]); the library
    works in its static device scratch array and allocates nothing.  Calls
    on one GPU must not overlap (they share that array)."""
    for n, t, dt in (("means2d", means2d, torch.float32), ("radii", radii, torch.int32),
                     ("depths", depths, torch.float32), ("sorted_ids", sorted_ids, torch.int32),
                     ("ranges", ranges, torch.int32), ("num_splats", num_splats, torch.int32)):
        _dev(t, dt, n)
    gx, gy = grid(width, height)
    if ranges.numel() != 2 * gx * gy or num_splats.numel() < 1:
        raise ValueError("ranges must hold 2 x tiles entries, num_splats one")
    st = lib().gs_bin_sort_noalloc(means2d.shape[0], _ptr(means2d), _ptr(radii), _ptr(depths),
                                   width, height, sorted_ids.numel(), _ptr(sorted_ids),
                                   _ptr(ranges), _ptr(num_splats), _stream())
    _check("gs_bin_sort_noalloc", st)
    return sorted_ids, ranges, num_splats


class Rasterizer:
    """Owns the output buffers of gs_rasterize_fwd for one image size.
    ``tune`` (a gs_raster_tune, e.g. from autotune.tune_raster) selects the
    launch shape; None is the library default."""

    def __init__(self, width: int, height: int, device="cuda", tune: "gs_raster_tune | None" = None):
        self.width, self.height = width, height
        self.tune = tune
        self.rgb = torch.empty(3, height, width, dtype=torch.float32, device=device)
        self.T = torch.empty(height, width, dtype=torch.float32, device=device)
        self.n_contrib = torch.empty(height, width, dtype=torch.int32, device=device)
        self.counters = torch.zeros(4, dtype=torch.int64, device=device)

    def __call__(self, ranges, sorted_ids, means2d, conics, log_opacities, rgb, precision="fp32",
                 background=(0.0, 0.0, 0.0), count: bool = False, tune=None,
                 ncontrib: bool = True):
        """ncontrib=False: n_contrib is not written (the kernels skip that
        bookkeeping; the backward needs it)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        for n, t, dt in (("ranges", ranges, torch.int32), ("sorted_ids", sorted_ids, torch.int32),
                         ("means2d", means2d, torch.float32), ("conics", conics, torch.float32),
                         ("log_opacities", log_opacities, torch.float32),
                         ("rgb", rgb, torch.float32)):
            _dev(t, dt, n)
        bg = (c_float * 3)(*[float(b) for b in background])
        if count:
            self.counters.zero_()
        tune = self.tune if tune is None else tune
        if tune is None:
            st = lib().gs_rasterize_fwd(self.width, self.height, _ptr(ranges), _ptr(sorted_ids),
                                        _ptr(means2d), _ptr(conics), _ptr(log_opacities), _ptr(rgb),
                                        bg, prec, _ptr(self.rgb), _ptr(self.T),
                                        _ptr(self.n_contrib) if ncontrib else c_void_p(0),
                                        _ptr(self.counters) if count else c_void_p(0), _stream())
            _check("gs_rasterize_fwd", st)
        else:
            st = lib().gs_rasterize_fwd_tuned(self.width, self.height, _ptr(ranges),
                                              _ptr(sorted_ids), _ptr(means2d), _ptr(conics),
                                              _ptr(log_opacities), _ptr(rgb), bg, prec,
                                              ctypes.byref(tune), _ptr(self.rgb), _ptr(self.T),
                                              _ptr(self.n_contrib) if ncontrib else c_void_p(0),
                                              _ptr(self.counters) if count else c_void_p(0),
                                              _stream())
            _check("gs_rasterize_fwd_tuned", st)
        return self.rgb, self.T, self.n_contrib


def rasterize_fwd(width, height, ranges, sorted_ids, means2d, conics, log_opacities, rgb,
                  precision="fp32", background=(0.0, 0.0, 0.0), count=False):
    r = Rasterizer(width, height, device=means2d.device)
    r(ranges, sorted_ids, means2d, conics, log_opacities, rgb, precision, background, count)
    return r


def rasterize_bwd(width, height, ranges, sorted_ids, means2d, conics, log_opacities, rgb, out_T,
                  out_ncontrib, dL_dimg, precision="fp32", background=(0.0, 0.0, 0.0)):
    """Gradients through rasterize_fwd (same precision as the forward): returns
    dict(means2d, conics, opacities (d/do), rgb) of freshly
    zeroed-then-accumulated tensors."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for n, t, dt in (("out_T", out_T, torch.float32), ("out_ncontrib", out_ncontrib, torch.int32),
                     ("dL_dimg", dL_dimg, torch.float32)):
        _dev(t, dt, n)
    g = dict(means2d=torch.zeros_like(means2d), conics=torch.zeros_like(conics),
             opacities=torch.zeros_like(log_opacities), rgb=torch.zeros_like(rgb))
    bg = (c_float * 3)(*[float(b) for b in background])
    st = lib().gs_rasterize_bwd(width, height, _ptr(ranges), _ptr(sorted_ids), _ptr(means2d),
                                _ptr(conics), _ptr(log_opacities), _ptr(rgb), bg, prec, _ptr(out_T),
                                _ptr(out_ncontrib), _ptr(dL_dimg), _ptr(g["means2d"]),
                                _ptr(g["conics"]), _ptr(g["opacities"]), _ptr(g["rgb"]), _stream())
    _check("gs_rasterize_bwd", st)
    return g


class RasterizeFn(torch.autograd.Function):
    """Differentiable tile rasteriser: (means2d, conics, opacities, rgb) ->
    image (3, H, W), for fixed per-tile lists.  Both directions run in
    libgsmfma (gs_rasterize_fwd / gs_rasterize_bwd) with the same precision.
    The rasteriser reads ln o (`log_opacities`, as preprocess writes it from
    the same `opacities`); the gradient returned for `opacities` is d/do."""

    @staticmethod
    def forward(ctx, means2d, conics, opacities, rgb, log_opacities, ranges, sorted_ids, width,
                height, precision="fp16_g2l_split", background=(0.0, 0.0, 0.0)):
        r = Rasterizer(width, height, device=means2d.device)
        means2d, conics = means2d.contiguous(), conics.contiguous()
        log_opacities, rgb = log_opacities.contiguous(), rgb.contiguous()
        r(ranges, sorted_ids, means2d, conics, log_opacities, rgb, precision, background)
        ctx.save_for_backward(means2d, conics, log_opacities, rgb, ranges, sorted_ids, r.T,
                              r.n_contrib)
        ctx.cfg = (width, height, precision, tuple(background))
        return r.rgb

    @staticmethod
    def backward(ctx, dL_dimg):
        means2d, conics, log_opacities, rgb, ranges, sorted_ids, T, nc = ctx.saved_tensors
        width, height, precision, background = ctx.cfg
        g = rasterize_bwd(width, height, ranges, sorted_ids, means2d, conics, log_opacities, rgb, T,
                          nc, dL_dimg.contiguous(), precision, background)
        return (g["means2d"], g["conics"], g["opacities"], g["rgb"], None, None, None, None, None,
                None, None)


def rasterize_beta(width, height, tile, ranges, sorted_ids, means2d, conics, log_opacities,
                   precision="fp16_g2l_split", count=32):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    out = torch.empty(count, 256, dtype=torch.float32, device=means2d.device)
    st = lib().gs_rasterize_beta(width, height, int(tile), _ptr(ranges), _ptr(sorted_ids),
                                 _ptr(means2d), _ptr(conics), _ptr(log_opacities), prec, int(count),
                                 _ptr(out), _stream())
    _check("gs_rasterize_beta", st)
    return out


def render(means3d, scales, quats, sh, opacities, cam: gs_camera, precision="fp16_g2l_split",
           capacity=None, background=(0.0, 0.0, 0.0)):
    """Preprocess -> bin/sort -> rasterise, all on the current stream."""
    pre = preprocess(means3d, scales, quats, opacities, sh, cam)
    bs = bin_sort(pre["means2d"], pre["radii"], pre["depths"], cam.width, cam.height, capacity)
    r = Rasterizer(cam.width, cam.height, device=means3d.device)
    r(bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], pre["log_opacities"], pre["rgb"],
      precision, background)
    return r, bs, pre


PEAK_PROBES = {"exp": (0, 8), "fma": (1, 16), "mfma_f16": (2, 4 * 32768)}


def peak_probe(kind: str, iters: int, blocks: int, reps: int = 3) -> float:
    """Measured peak rate of the device for one operation kind (gs_peak_probe):
    "exp" -> v_exp_f32 per second, "fma" -> FP32 FMA flop/s, "mfma_f16" ->
    flop/s of v_mfma_f32_32x32x16_f16.  Best of `reps` timed launches (after
    one warm-up) on the current stream."""
    k, per = PEAK_PROBES[kind]
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for r in range(reps + 1):
        ev0.record()
        _check("gs_peak_probe", lib().gs_peak_probe(k, iters, blocks, _ptr(out), _stream()))
        ev1.record()
        torch.cuda.synchronize()
        if r:
            best = min(best, ev0.elapsed_time(ev1) / 1e3)
    if kind == "mfma_f16":
        ops = blocks * 4 * iters * per  # four waves per workgroup
    else:
        ops = blocks * 256 * iters * per
    return ops / best


def wall_clock_khz() -> int:
    k = c_int32(0)
    _check("gs_wall_clock_khz", lib().gs_wall_clock_khz(ctypes.byref(k)))
    return int(k.value)


class MultiViewRenderer:
    """Renders one scene to several cameras per frame: one multi-view
    preprocess, the views' bin/sort (one gs_bin_sort per view,
    ``bin_streams`` views at a time on as many streams; or, with
    ``joint_bin``, gs_bin_sort_multiview over ``bin_groups`` groups of
    views, one stream each), and ONE persistent batched rasteriser launch
    over every (view, tile) pair.
    Buffers are sized once (splat capacity per view from a probe frame times
    ``slack``); a frame allocates nothing, so it can be captured in a
    hipGraph (:meth:`capture`).  Per-view latency inside a frame comes from
    device wall-clock stamps (frame start, last tile of each view)."""

    def __init__(self, scene: dict, cams, precision="fp16_g2l_split", slack=1.15,
                 background=(0.0, 0.0, 0.0), sh_degree=3, precise=False, bin_streams=4,
                 joint_bin=False, bin_groups=1):
        self.scene = {k: _dev(scene[k], torch.float32, k)
                      for k in ("means3d", "scales", "quats", "sh", "opacities")}
        self.cams = list(cams)
        self.V, self.P = len(self.cams), self.scene["means3d"].shape[0]
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.sh_degree = sh_degree
        self.precise = bool(precise)
        dev = self.scene["means3d"].device
        self.device = dev
        self.pre = preprocess_multiview(self.scene["means3d"], self.scene["scales"],
                                        self.scene["quats"], self.scene["opacities"],
                                        self.scene["sh"], self.cams, sh_degree)
        self.slack = slack
        self.joint = bool(joint_bin)
        self.K = max(1, min(int(bin_streams), self.V))
        self.sorters = None
        self._bin_streams = None
        sizes = [(c.width, c.height) for c in self.cams]
        if self.V > GS_MAX_BIN_VIEWS:
            self.joint = False
        # probe frame: splat count per view (capacity 0)
        if self.joint:
            probe = MultiViewBinSorter(self.P, 0, sizes, device=dev, precise=self.precise)
            probe(*self._bin_inputs_all())
            counts = probe.view_counts()
            del probe
        else:
            counts = []
            for v, c in enumerate(self.cams):
                probe = BinSorter(self.P, 0, c.width, c.height, device=dev, precise=self.precise)
                probe(*self._bin_inputs(v))
                counts.append(probe.n_splats())
        self.probe_counts = counts
        self.capacity = [int(n * slack) + 1024 for n in counts]
        if self.joint:
            # G groups of consecutive views, one joint call each (on G streams)
            G = max(1, min(int(bin_groups), self.V))
            cuts = [round(g * self.V / G) for g in range(G + 1)]
            self.groups = [(cuts[g], cuts[g + 1]) for g in range(G)]
            self.mvbins = [MultiViewBinSorter(self.P, sum(self.capacity[a:b]), sizes[a:b],
                                              device=dev, precise=self.precise)
                           for a, b in self.groups]
            self.mvbin = self.mvbins[0]
        else:
            self._per_view_sorters()
        self.images = [Rasterizer(c.width, c.height, device=dev) for c in self.cams]
        views = (gs_view * self.V)()
        for v, (c, r) in enumerate(zip(self.cams, self.images)):
            g = views[v]
            g.width, g.height = c.width, c.height
            rg, ids = self._lists(v)
            g.tile_ranges, g.sorted_ids = rg.data_ptr(), ids.data_ptr()
            g.means2d = self.pre["means2d"][v].data_ptr()
            g.conics = self.pre["conics"][v].data_ptr()
            g.log_opacities = self.pre["log_opacities"].data_ptr()
            g.rgb = self.pre["rgb"][v].data_ptr()
            g.background[:] = [float(b) for b in background]
            g.out_rgb, g.out_T = r.rgb.data_ptr(), r.T.data_ptr()
            g.out_ncontrib = r.n_contrib.data_ptr()
        self.views = views
        L = lib()
        self.plan = torch.empty(L.gs_batch_plan_bytes(self.V), dtype=torch.uint8, device=dev)
        _check("gs_batch_plan_write",
               L.gs_batch_plan_write(self.V, views, _ptr(self.plan), self.plan.numel()))
        self.batch_ws = torch.empty(L.gs_batch_workspace_bytes(self.V), dtype=torch.uint8,
                                    device=dev)
        self.clock = torch.zeros(self.V + 1, dtype=torch.int64, device=dev)  # [0] frame start
        self.tune = make_tune()

    # -- stages -----------------------------------------------------------
    def preprocess(self):
        preprocess_multiview(self.scene["means3d"], self.scene["scales"], self.scene["quats"],
                             self.scene["opacities"], self.scene["sh"], self.cams, self.sh_degree,
                             out=self.pre)

    def _bin_inputs(self, v):
        return (self.pre["means2d"][v], self.pre["radii"][v], self.pre["depths"][v],
                self.pre["conics"][v], self.pre["log_opacities"])

    def _bin_inputs_all(self):
        return (self.pre["means2d"], self.pre["radii"], self.pre["depths"], self.pre["conics"],
                self.pre["log_opacities"])

    def _per_view_sorters(self):
        """One BinSorter per view (views are sorted K at a time on K streams,
        view v on stream v % K, each stream with its own workspace): the
        pipelined frame and the per-view comparison use them."""
        if self.sorters is None:
            dev = self.device
            wsb = (lib().gs_bin_sort_precise_workspace_bytes if self.precise
                   else lib().gs_bin_sort_workspace_bytes)
            ws = max(wsb(self.P, cap, c.width, c.height) for cap, c in zip(self.capacity, self.cams))
            self.bin_workspaces = [torch.empty(ws, dtype=torch.uint8, device=dev)
                                   for _ in range(self.K)]
            self.sorters = [BinSorter(self.P, cap, c.width, c.height, device=dev,
                                      workspace=self.bin_workspaces[v % self.K],
                                      precise=self.precise)
                            for v, (cap, c) in enumerate(zip(self.capacity, self.cams))]
        return self.sorters

    def _group_of(self, v):
        for g, (a, b) in enumerate(self.groups):
            if a <= v < b:
                return g, v - a
        raise IndexError(v)

    def _lists(self, v):
        """(tile ranges, sorted ids) of view v for the frame's rasterisation."""
        if self.joint:
            g, w = self._group_of(v)
            return self.mvbins[g].ranges(w), self.mvbins[g].sorted_ids
        return self.sorters[v].ranges, self.sorters[v].sorted_ids

    def view_lists(self, v):
        """Host copies of view v's lists as one-view binning gives them:
        (ranges [ntiles, 2] counted from the view's first splat, empty tiles
        [0, 0]; sorted ids [n])."""
        rg, ids = self._lists(v)
        rg = rg.cpu().numpy().astype(np.int64)
        if self.joint:
            g, w = self._group_of(v)
            counts = self.mvbins[g].view_counts()
            base, n = sum(counts[:w]), counts[w]
        else:
            base, n = 0, self.sorters[v].n_splats()
        full = rg[:, 1] > rg[:, 0]
        out = np.zeros_like(rg)
        out[full] = rg[full] - base
        return out, ids[base:base + n].cpu().numpy()

    def bin_sort(self, concurrent: bool = True):
        """Every view's lists: one gs_bin_sort_multiview call (joint), or one
        gs_bin_sort per view."""
        if not self.joint:
            self.bin_sort_per_view(concurrent)
            return
        m2, rad, dep, con, opac = self._bin_inputs_all()
        if len(self.groups) == 1:
            self.mvbin(m2, rad, dep, con, opac)
            return
        cur = torch.cuda.current_stream()
        if self._bin_streams is None or len(self._bin_streams) < len(self.groups):
            self._bin_streams = [torch.cuda.Stream(device=self.device)
                                 for _ in range(max(len(self.groups), self.K))]
        for st in self._bin_streams[:len(self.groups)]:
            st.wait_stream(cur)
        for (a, b), mb, st in zip(self.groups, self.mvbins, self._bin_streams):
            with torch.cuda.stream(st):
                mb(m2[a:b], rad[a:b], dep[a:b], con[a:b], opac)
        for st in self._bin_streams[:len(self.groups)]:
            cur.wait_stream(st)

    def bin_sort_per_view(self, concurrent: bool = True):
        """One gs_bin_sort per view (K streams when ``concurrent``) into the
        per-view sorters' own buffers."""
        self._per_view_sorters()
        if self.K == 1 or not concurrent:
            for v, bs in enumerate(self.sorters):
                bs(*self._bin_inputs(v))
            return
        cur = torch.cuda.current_stream()
        if self._bin_streams is None:
            self._bin_streams = [torch.cuda.Stream(device=self.device) for _ in range(self.K)]
        for st in self._bin_streams:
            st.wait_stream(cur)
        for v, bs in enumerate(self.sorters):
            with torch.cuda.stream(self._bin_streams[v % self.K]):
                bs(*self._bin_inputs(v))
        for st in self._bin_streams:
            cur.wait_stream(st)

    def raster(self, tune: gs_batch_tune | None = None, stamp=True):
        t = self.tune if tune is None else tune
        st = lib().gs_rasterize_fwd_batched(self.V, _ptr(self.plan), self.precision,
                                            ctypes.byref(t), _ptr(self.batch_ws),
                                            self.batch_ws.numel(),
                                            c_void_p(self.clock.data_ptr() + 8) if stamp
                                            else c_void_p(0), _stream())
        _check("gs_rasterize_fwd_batched", st)

    def raster_per_view(self):
        """The same images with one gs_rasterize_fwd launch per view."""
        for v, r in enumerate(self.images):
            rg, ids = self._lists(v)
            r(rg, ids, self.pre["means2d"][v], self.pre["conics"][v],
              self.pre["log_opacities"], self.pre["rgb"][v], self.precision,
              tuple(self.views[v].background))

    def frame(self, tune: gs_batch_tune | None = None):
        """preprocess -> bin/sort of every view -> ONE batched raster launch."""
        _check("gs_clock_stamp", lib().gs_clock_stamp(_ptr(self.clock), _stream()))
        self.preprocess()
        self.bin_sort()
        self.raster(tune)

    def frame_pipelined(self):
        """The same images with the rasterisation of view v (one launch per
        view, on a second stream) overlapping the bin/sort of the views after
        it: bin/sort is bound by memory traffic, the rasteriser by the vector
        ALUs.  The second stream joins the current one at the end; each
        view's clock stamp follows its raster on the second stream."""
        cur = torch.cuda.current_stream()
        if getattr(self, "_side", None) is None:
            self._side = torch.cuda.Stream(device=self.device)
            self._events = [torch.cuda.Event() for _ in range(self.V)]
        L = lib()
        self._per_view_sorters()
        _check("gs_clock_stamp", L.gs_clock_stamp(_ptr(self.clock), _stream()))
        self.preprocess()
        side = self._side
        side.wait_stream(cur)
        for v, (bs, r) in enumerate(zip(self.sorters, self.images)):
            bs(*self._bin_inputs(v))
            self._events[v].record(cur)
            with torch.cuda.stream(side):
                side.wait_event(self._events[v])
                r(bs.ranges, bs.sorted_ids, self.pre["means2d"][v], self.pre["conics"][v],
                  self.pre["log_opacities"], self.pre["rgb"][v], self.precision,
                  tuple(self.views[v].background))
                _check("gs_clock_stamp",
                       L.gs_clock_stamp(c_void_p(self.clock.data_ptr() + 8 * (v + 1)), _stream()))
        cur.wait_stream(side)

    def capture(self, tune: gs_batch_tune | None = None, pipelined: bool = False) -> "torch.cuda.CUDAGraph":
        """A hipGraph of one whole frame (replay with ``g.replay()``):
        :meth:`frame`, or :meth:`frame_pipelined` (two streams, forked and
        joined inside the graph)."""
        run = self.frame_pipelined if pipelined else (lambda: self.frame(tune))
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            run()  # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run()
        return g

    # -- results ----------------------------------------------------------
    def n_splats(self):
        if self.joint:
            return [c for mb in self.mvbins for c in mb.view_counts()]
        return [bs.n_splats() for bs in self.sorters]

    def overflowed(self):
        if self.joint:
            return [mb.n_splats() > mb.capacity for (a, b), mb in zip(self.groups, self.mvbins)
                    for _ in range(b - a)]
        return [n > cap for n, cap in zip(self.n_splats(), self.capacity)]

    def latencies_ms(self):
        """Per-view time from the frame-start stamp to the view's last tile
        (host read; synchronises)."""
        c = self.clock.cpu().tolist()
        khz = wall_clock_khz()
        return [(c[1 + v] - c[0]) / khz for v in range(self.V)]
