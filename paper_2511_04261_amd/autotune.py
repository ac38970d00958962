"""Tile-shape autotuner.

Results never depend on the tile shape or the launch mode (exact integer sums,
an index-ordered scan, geometry-keyed noise), so the tuner is free to pick the
fastest.  For each geometry class (layout, H, W, C, b, s_b) it times
plan + forward on a synthetic batch of that class large enough to fill the GPU,
for a few tile widths and workgroup sizes and both launch modes, with HIP
events around steps enqueued back to back, and keeps the fastest.  Winners are cached in a JSON file keyed
by the device name and the class.  `tune_whole_batch` instead times whole
candidate configurations of one given batch.
"""
from __future__ import annotations

import json
import os
import statistics
import time
from dataclasses import replace
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import F32_CHW, U8_HWC, FrameParams, Plan

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dppix", "autotune.json")
TILE_BYTES = (1024, 2048, 4096, 8192)
#: 0: the library's per-class choice (128 for tiles with few row items, else 256)
THREADS = (0, 128, 192, 256, 512)
#: 0: one workgroup per tile; 1: resident grid pulling tiles from a ticket
LAUNCH_MODES = (0, 1)


def class_key(fp: FrameParams) -> str:
    sb = fp.b if fp.sb is None else fp.sb
    return "%s:%dx%dx%d:b%d:s%d" % ("u8" if fp.layout == U8_HWC else "f32", fp.height, fp.width, fp.channels,
                                    fp.b, sb)


def tile_candidates(fp: FrameParams) -> List[int]:
    unit = fp.b * fp.channels if fp.layout == U8_HWC else 4 * fp.b
    gc = -(-fp.width // fp.b)
    out = {0}
    for tb in TILE_BYTES:
        out.add(int(min(gc, max(1, tb // unit))))
    return sorted(out)


def with_tile_bytes(frames: Sequence[FrameParams], tile_bytes: int) -> List[FrameParams]:
    """The frames with tile rows of about `tile_bytes` (0: the library's choice)."""
    if tile_bytes == 0:
        return [replace(fp, tile_cells=0) for fp in frames]
    out = []
    for fp in frames:
        unit = fp.b * fp.channels if fp.layout == U8_HWC else 4 * fp.b
        gc = -(-fp.width // fp.b)
        out.append(replace(fp, tile_cells=int(min(gc, max(1, tile_bytes // unit)))))
    return out


def _device_name(device) -> str:
    import torch
    return torch.cuda.get_device_name(device).replace(" ", "_")


def _class_batch(fp: FrameParams, device, min_pixels: float):
    """Synthetic frames of one class: random bytes, ~15% rectangle masks."""
    import torch
    from . import synth
    n = max(1, int(np.ceil(min_pixels / (fp.height * fp.width))))
    g = torch.Generator(device=device)
    g.manual_seed(1234)
    rng = np.random.Generator(np.random.PCG64(4321))
    imgs, masks = [], []
    for _ in range(n):
        if fp.layout == U8_HWC:
            imgs.append(torch.randint(0, 256, (fp.height, fp.width, fp.channels), dtype=torch.uint8, device=device,
                                      generator=g))
        else:
            imgs.append(torch.rand((fp.channels, fp.height, fp.width), device=device, generator=g) * 255)
        masks.append(synth.paint_mask_torch(synth.draw_rects(rng, fp.height, fp.width), fp.height, fp.width, device))
    return n, imgs, masks


def time_config(frames: Sequence[FrameParams], imgs, masks, device, threads: int, persistent: int,
                reps: int = 5, fused: bool = True, warm_s: float = 0.015) -> float:
    """GPU ms of one plan + forward for one launch configuration: the median
    of three windows of `reps` steps enqueued back to back through the C ABI
    (no host work between steps inside a window)."""
    import ctypes
    import torch
    from . import _lib
    plan = Plan(frames, device=device, threads=threads, persistent=persistent)
    outs = [torch.empty_like(t) for t in imgs] if fused else None
    plan.plan(masks)
    plan.forward(imgs, out=outs)      # checks shapes once, builds the pointer tables
    lib, h, st = plan.lib, plan.handle, ctypes.byref(plan.store.c)
    ip = ctypes.c_void_p(plan.pointer_table(imgs).data_ptr())
    mt = plan.pointer_table(masks)
    mp = None if mt is None else ctypes.c_void_p(mt.data_ptr())
    op = None if outs is None else ctypes.c_void_p(plan.pointer_table(outs).data_ptr())
    stream = torch.cuda.current_stream()
    sh = ctypes.c_void_p(stream.cuda_stream)
    # untimed steps first: after host work the GPU's clocks need some 10 ms
    # of load to settle, and a configuration timed before that reads slow
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(reps):
            _lib.check(lib.dp_pix_plan(h, mp, st, sh))
            _lib.check(lib.dp_pix_forward(h, ip, st, None, None, op, sh))
        torch.cuda.synchronize()
    times = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            _lib.check(lib.dp_pix_plan(h, mp, st, sh))
            _lib.check(lib.dp_pix_forward(h, ip, st, None, None, op, sh))
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / reps)
    plan.close()
    return statistics.median(times)


class Autotuner:
    def __init__(self, device=None, cache_path: Optional[str] = DEFAULT_CACHE, min_pixels: float = 64e6,
                 reps: int = 5, threads: Sequence[int] = THREADS, launch_modes: Sequence[int] = LAUNCH_MODES):
        import torch
        self.device = torch.device(device if device is not None else "cuda:0")
        self.cache_path = cache_path
        self.min_pixels = min_pixels
        self.reps = reps
        self.threads = tuple(threads)
        self.launch_modes = tuple(launch_modes)
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self):
        if not self.cache_path:
            return
        os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
        tmp = self.cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def tune_class(self, fp: FrameParams) -> dict:
        key = "%s|%s|thr%s|modes%s" % (_device_name(self.device), class_key(fp),
                                       ",".join(map(str, self.threads)), ",".join(map(str, self.launch_modes)))
        if key in self.cache:
            return self.cache[key]
        n, imgs, masks = _class_batch(fp, self.device, self.min_pixels)
        results: List[Tuple[float, int, int, int]] = []
        for tc in tile_candidates(fp):
            frames = [replace(fp, tile_cells=tc, frame_index=i) for i in range(n)]
            for th in self.threads:
                for pers in self.launch_modes:
                    ms = time_config(frames, imgs, masks, self.device, th, pers, self.reps)
                    results.append((ms, tc, th, pers))
        results.sort()
        ms, tc, th, pers = results[0]
        best = dict(tile_cells=tc, threads=th, persistent=pers, ms=ms, frames=n,
                    mpix_per_s=n * fp.height * fp.width / (ms * 1e-3) / 1e6,
                    tried=[dict(ms=r[0], tile_cells=r[1], threads=r[2], persistent=r[3]) for r in results[:8]])
        self.cache[key] = best
        self._save()
        return best

    def tune_whole_batch(self, frames: Sequence[FrameParams], imgs, masks,
                         tile_bytes: Sequence[int] = (0, 1024, 1536, 3072, 4096),
                         margin: float = 0.01) -> Tuple[List[FrameParams], dict]:
        """Tile shapes for one batch as it will run: every frame's tile row is
        about `tile_bytes` long (0: the library's choice), for each candidate
        and workgroup size the whole batch is timed (plan + forward on its own
        images and masks), and the fastest wins.  Per-class tuning on
        separate small batches does not see how classes share the GPU in a
        mixed batch; this does, at the cost of one timing per candidate.
        The library's own choice (tile_bytes 0, threads 0) is kept unless a
        candidate beats it by more than `margin`, so that timing noise does
        not flip the shapes from run to run."""
        results = []
        for tb in tile_bytes:
            cand = with_tile_bytes(frames, tb)
            for th in self.threads:
                for pers in self.launch_modes:
                    ms = time_config(cand, imgs, masks, self.device, th, pers, self.reps)
                    results.append((ms, tb, th, pers, cand))
        results.sort(key=lambda r: r[0])
        default = [r for r in results if r[1] == 0 and r[2] == 0 and r[3] == 0]
        best = results[0]
        if default and best[0] > (1.0 - margin) * default[0][0]:
            best = default[0]
        ms, tb, th, pers, cand = best
        info = dict(ms=ms, tile_bytes=tb, threads=th, persistent=pers,
                    tried=[dict(ms=round(r[0], 4), tile_bytes=r[1], threads=r[2], persistent=r[3]) for r in results])
        return list(cand), info

    def tune_batch(self, frames: Sequence[FrameParams]) -> Tuple[List[FrameParams], dict]:
        """Per-class tile widths for every frame, and one launch shape for the
        batch: the (workgroup size, launch mode) pair voted by pixel count."""
        votes: Dict[Tuple[int, int], float] = {}
        out = []
        for fp in frames:
            best = self.tune_class(fp)
            out.append(replace(fp, tile_cells=best["tile_cells"]))
            k = (best["threads"], best["persistent"])
            votes[k] = votes.get(k, 0.0) + fp.height * fp.width
        threads, persistent = max(votes, key=votes.get)
        return out, dict(threads=threads, persistent=persistent)
