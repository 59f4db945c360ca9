"""Autotuners for the launch shapes of the rasterisers.

* Batched multi-view rasteriser (gs_rasterize_fwd_batched): the splats
  staged per round (64 / 128 / 256), the persistent workgroups per compute
  unit (the kernel's occupancy) and the work queue layout (eight per-XCD
  queues of two-row tile bands with stealing, or one row-major queue).
* One-view rasteriser (gs_rasterize_fwd_tuned): the splats staged per round
  (64 / 128 / 256) and the tile rows per XCD chunk (1 or 2).

Every candidate is timed on the caller's own frame (its bin/sort lists
already built) with HIP events on the current stream, and its images are
compared bit for bit with the first candidate's: the per-tile arithmetic
does not depend on the launch shape, so any difference is a defect and
raises.

Results can be kept in a small JSON cache keyed by device and workload.
"""
from __future__ import annotations

import itertools
import json
import os
import statistics

import torch

from . import PRECISIONS, Rasterizer, make_raster_tune, make_tune

DEFAULT_SPACE = {"batch": (64, 128, 256), "blocks_per_cu": (2, 3, 4, 5), "xcd_queues": (0, 1)}
RASTER_SPACE = {"batch": (64, 128, 256), "chunk_rows": (1, 2)}


def time_ms(fn, reps: int = 5, warmup: int = 1, before=None) -> list:
    """Per-call times of fn() in ms (HIP events around each call on the
    current stream).  before(), if given, runs ahead of every call, outside
    the events."""
    for _ in range(warmup):
        if before is not None:
            before()
        fn()
    out = []
    st = torch.cuda.current_stream()
    for _ in range(reps):
        if before is not None:
            before()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def _snapshot(renderer):
    return [(r.rgb.clone(), r.T.clone(), r.n_contrib.clone()) for r in renderer.images]


def _same(a, b) -> bool:
    return all(torch.equal(x, y) for pa, pb in zip(a, b) for x, y in zip(pa, pb))


def tune_batched(renderer, space: dict | None = None, reps: int = 5, warmup: int = 1,
                 check: bool = True) -> dict:
    """Times every launch shape of ``space`` on the renderer's current frame
    and installs the fastest as ``renderer.tune``.  Returns
    {"best": {...}, "table": [{batch, blocks_per_cu, xcd_queues, ms_median, ms_min}]}."""
    space = dict(DEFAULT_SPACE, **(space or {}))
    renderer.preprocess()
    renderer.bin_sort()
    ref, rows = None, []
    for nb, bpc, xq in itertools.product(space["batch"], space["blocks_per_cu"],
                                         space["xcd_queues"]):
        t = make_tune(nb, bpc, xq)
        ts = time_ms(lambda: renderer.raster(t, stamp=False), reps, warmup)
        if check:
            snap = _snapshot(renderer)
            if ref is None:
                ref = snap
            elif not _same(ref, snap):
                raise RuntimeError(f"batched raster output differs for launch shape {t.as_tuple()}")
        rows.append({"batch": nb, "blocks_per_cu": bpc, "xcd_queues": xq,
                     "ms_median": statistics.median(ts), "ms_min": min(ts)})
    best = min(rows, key=lambda r: r["ms_median"])
    renderer.tune = make_tune(best["batch"], best["blocks_per_cu"], best["xcd_queues"])
    return {"best": best, "table": rows}


def tune_raster(rasterizer: Rasterizer, ranges, sorted_ids, means2d, conics, log_opacities, rgb,
                precision="fp16_g2l_split", space: dict | None = None, reps: int = 5,
                warmup: int = 1, check: bool = True, ncontrib: bool = True, before=None) -> dict:
    """Times every launch shape of ``space`` for one-view rasterisation of
    the given lists and installs the fastest as ``rasterizer.tune``.  The
    FP32 kernels stage a fixed 256 splats, so only the chunk height is tried
    for them.  Returns {"best": {batch, chunk_rows, ms_median, ms_min},
    "table": [...]}.  ncontrib as for Rasterizer: tune the launches that
    write n_contrib, or those that skip it.  before(), if given, runs ahead
    of every timed call (e.g. the frame's preprocess and bin/sort, which must
    leave the lists unchanged), so each shape is timed in the state a frame
    leaves the GPU in."""
    space = dict(RASTER_SPACE, **(space or {}))
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    batches = space["batch"] if prec >= PRECISIONS["fp16_global"] else (128,)
    ref, rows = None, []
    for nb, cr in itertools.product(batches, space["chunk_rows"]):
        t = make_raster_tune(nb, cr)
        ts = time_ms(lambda: rasterizer(ranges, sorted_ids, means2d, conics, log_opacities, rgb,
                                        precision, tune=t, ncontrib=ncontrib), reps, warmup,
                     before)
        if check:
            snap = (rasterizer.rgb.clone(), rasterizer.T.clone()) + (
                (rasterizer.n_contrib.clone(),) if ncontrib else ())
            if ref is None:
                ref = snap
            elif not all(torch.equal(x, y) for x, y in zip(ref, snap)):
                raise RuntimeError(f"one-view raster output differs for launch shape {t.as_tuple()}")
        rows.append({"batch": nb, "chunk_rows": cr, "ms_median": statistics.median(ts),
                     "ms_min": min(ts)})
    best = min(rows, key=lambda r: r["ms_median"])
    rasterizer.tune = make_raster_tune(best["batch"], best["chunk_rows"])
    return {"best": best, "table": rows}


def raster_key(rasterizer: Rasterizer, precision, n_splats: int) -> str:
    """Cache key of a one-view shape: device, precision, image size and the
    splat count to within a factor of 2."""
    name = torch.cuda.get_device_name(rasterizer.rgb.device)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return (f"{name}|raster|prec{prec}|{rasterizer.width}x{rasterizer.height}"
            f"|N2^{max(int(n_splats), 1).bit_length()}")


def workload_key(renderer) -> str:
    """Cache key: device name, precision, scene size and view resolutions."""
    name = torch.cuda.get_device_name(renderer.device)
    res = ",".join(f"{c.width}x{c.height}" for c in renderer.cams)
    return f"{name}|prec{renderer.precision}|P{renderer.P}|{res}"


class TuneCache:
    """JSON file of tuned launch shapes keyed by :func:`workload_key`."""

    def __init__(self, path: str):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, renderer):
        b = self.data.get(workload_key(renderer))
        return None if b is None else make_tune(b["batch"], b["blocks_per_cu"], b["xcd_queues"])

    def put(self, renderer, best: dict):
        self.data[workload_key(renderer)] = {k: best[k] for k in ("batch", "blocks_per_cu",
                                                                   "xcd_queues")}
        with open(self.path, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)

    def tune_raster(self, rasterizer: Rasterizer, n_splats: int, *args, precision="fp16_g2l_split",
                    **kw):
        """Cached one-view shape for this workload if present, else
        :func:`tune_raster` and store the result."""
        key = raster_key(rasterizer, precision, n_splats)
        b = self.data.get(key)
        if b is not None:
            rasterizer.tune = make_raster_tune(b["batch"], b["chunk_rows"])
            return {"best": dict(b), "cached": True}
        res = tune_raster(rasterizer, *args, precision=precision, **kw)
        self.data[key] = {k: res["best"][k] for k in ("batch", "chunk_rows")}
        with open(self.path, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        return res

    def tune(self, renderer, **kw):
        """Cached shape if present, else tune and store."""
        t = self.get(renderer)
        if t is not None:
            renderer.tune = t
            return {"best": dict(zip(("batch", "blocks_per_cu", "xcd_queues"), t.as_tuple())),
                    "cached": True}
        res = tune_batched(renderer, **kw)
        self.put(renderer, res["best"])
        return res
