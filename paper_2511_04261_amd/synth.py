"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper measures on surveillance video (768x576 and 1920x1080 frames,
Sec. VII-A) and portrait photos with foreground masks (Sec. VII-B); those
datasets are not available, so these generators stand in for them: a smooth
ramp plus uniform integer noise U{-20..20} per channel for the frames, and
unions of axis-aligned rectangles for the foreground masks.

Every frame is defined by a small integer recipe drawn from a numpy PCG64
stream, and rendered with integer arithmetic only, so the host (numpy) and the
GPU (torch) produce the same bytes: large batches are rendered on the device,
and any frame can be re-rendered on the host for the oracle.

This module holds no part of the pixelization arithmetic; it only draws
numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

#: resolutions of the uneven batch: the two video sizes of the paper's runtime
#: study, UHD, and a 24 MP still
MIXED_RESOLUTIONS = ((576, 768), (1080, 1920), (2160, 3840), (4000, 6000))

_M32 = 0xFFFFFFFF
_MUL_A = 0x7FEB352D   # odd multipliers below 2^31: products stay below 2^63
_MUL_B = 0x4A09E667
_FIX = 1 << 16


def _mix(x, xp):
    """32-bit integer hash (xorshift-multiply), on int64 arrays of numpy or torch."""
    x = ((x ^ (x >> 16)) * _MUL_A) & _M32
    x = ((x ^ (x >> 15)) * _MUL_B) & _M32
    return x ^ (x >> 16)


@dataclass
class Ramp:
    """One channel: 128 + A * ((i - ic) cos t + (j - jc) sin t) / half, in
    16.16 fixed point, plus hash noise in [-20, 20]."""
    amp: int
    cos16: int
    sin16: int
    noise_key: int


def draw_ramp(rng: np.random.Generator) -> Ramp:
    amp = int(rng.integers(60, 101))
    theta = rng.uniform(0.0, 2.0 * math.pi)
    return Ramp(amp, int(round(math.cos(theta) * _FIX)), int(round(math.sin(theta) * _FIX)),
                int(rng.integers(0, 2**32)))


def _render_channel(r: Ramp, H: int, W: int, C: int, ch: int, xp, device=None):
    if xp is np:
        ii = np.arange(H, dtype=np.int64)[:, None]
        jj = np.arange(W, dtype=np.int64)[None, :]
    else:
        ii = xp.arange(H, dtype=xp.int64, device=device)[:, None]
        jj = xp.arange(W, dtype=xp.int64, device=device)[None, :]
    den = _FIX * max(H - 1, W - 1, 1)
    num = r.amp * (r.cos16 * (2 * ii - (H - 1)) + r.sin16 * (2 * jj - (W - 1)))
    if xp is np:
        ramp = 128 + np.floor_divide(num, den)
    else:
        ramp = 128 + xp.div(num, den, rounding_mode="floor")
    idx = (ii * W + jj) * C + ch
    h = _mix((idx + r.noise_key) & _M32, xp)
    h = _mix(h ^ r.noise_key, xp)
    noise = h % 41 - 20
    v = ramp + noise
    if xp is np:
        return np.clip(v, 0, 255).astype(np.uint8)
    return v.clamp(0, 255).to(xp.uint8)


def render_image(ramps: List[Ramp], H: int, W: int) -> np.ndarray:
    """uint8 (H, W, C) on the host."""
    C = len(ramps)
    out = np.empty((H, W, C), np.uint8)
    for ch, r in enumerate(ramps):
        out[:, :, ch] = _render_channel(r, H, W, C, ch, np)
    return out


def render_image_torch(ramps: List[Ramp], H: int, W: int, device):
    """uint8 (H, W, C) rendered on the device; byte-identical to render_image."""
    import torch
    C = len(ramps)
    out = torch.empty((H, W, C), dtype=torch.uint8, device=device)
    for ch, r in enumerate(ramps):
        out[:, :, ch] = _render_channel(r, H, W, C, ch, torch, device)
    return out


def gradient_image(rng: np.random.Generator, height: int, width: int, channels: int = 1) -> np.ndarray:
    """uint8 (H, W, C): per channel a ramp of amplitude A ~ U{60..100} along a
    random direction, centred on 128, plus noise U{-20..20}, clamped."""
    return render_image([draw_ramp(rng) for _ in range(channels)], height, width)


# --------------------------------------------------------------------------
# Foreground masks: unions of rectangles
# --------------------------------------------------------------------------
Rect = Tuple[int, int, int, int]   # y, x, h, w


def union_area(rects: List[Rect]) -> int:
    """Exact area of a union of axis-aligned rectangles (coordinate compression)."""
    if not rects:
        return 0
    ys = sorted({r[0] for r in rects} | {r[0] + r[2] for r in rects})
    xs = sorted({r[1] for r in rects} | {r[1] + r[3] for r in rects})
    area = 0
    for a in range(len(ys) - 1):
        for b in range(len(xs) - 1):
            y0, x0 = ys[a], xs[b]
            if any(r[0] <= y0 < r[0] + r[2] and r[1] <= x0 < r[1] + r[3] for r in rects):
                area += (ys[a + 1] - y0) * (xs[b + 1] - x0)
    return area


def draw_rects(rng: np.random.Generator, height: int, width: int, n_rects: int = 8, rect_frac: float = 0.02,
               cover: tuple = (0.13, 0.17), max_tries: int = 200) -> List[Rect]:
    """``n_rects`` rectangles of area ~rect_frac*H*W, aspect ratio U[0.5, 2],
    uniformly placed, redrawn until their union covers ``cover`` of the frame
    (the closest draw is kept if none does)."""
    best = None
    target = 0.5 * (cover[0] + cover[1])
    for _ in range(max_tries):
        rects = []
        for _r in range(n_rects):
            aspect = rng.uniform(0.5, 2.0)
            area = rect_frac * height * width
            h = max(1, min(height, int(round(math.sqrt(area / aspect)))))
            w = max(1, min(width, int(round(math.sqrt(area * aspect)))))
            y = int(rng.integers(0, height - h + 1))
            x = int(rng.integers(0, width - w + 1))
            rects.append((y, x, h, w))
        frac = union_area(rects) / float(height * width)
        if cover[0] <= frac <= cover[1]:
            return rects
        if best is None or abs(frac - target) < abs(best[0] - target):
            best = (frac, rects)
    return best[1]


def paint_mask(rects: List[Rect], height: int, width: int) -> np.ndarray:
    mk = np.zeros((height, width), np.uint8)
    for (y, x, h, w) in rects:
        mk[y:y + h, x:x + w] = 1
    return mk


def paint_mask_torch(rects: List[Rect], height: int, width: int, device):
    import torch
    mk = torch.zeros((height, width), dtype=torch.uint8, device=device)
    for (y, x, h, w) in rects:
        mk[y:y + h, x:x + w] = 1
    return mk


def rect_mask(rng: np.random.Generator, height: int, width: int, n_rects: int = 8, rect_frac: float = 0.02,
              cover: tuple = (0.13, 0.17), max_tries: int = 200) -> np.ndarray:
    """uint8 (H, W) foreground mask (1 = foreground) from draw_rects."""
    return paint_mask(draw_rects(rng, height, width, n_rects, rect_frac, cover, max_tries), height, width)


def uniform_f32(rng: np.random.Generator, shape) -> np.ndarray:
    """fp32 values uniform in [0, 255)."""
    return (rng.random(shape, dtype=np.float64) * 255.0).astype(np.float32)


# --------------------------------------------------------------------------
# Frames and batches
# --------------------------------------------------------------------------
@dataclass
class FrameSpec:
    """One frame: geometry, per-region parameters and the recipe of its data."""
    height: int
    width: int
    channels: int = 3
    b: int = 32             # grid size of simple (background) cells
    sb: int = 8             # subgrid size of complex (foreground) cells
    m: int = 16
    eps_simple: float = 1.0
    eps_complex: float = 0.3
    tau: int = 1            # complex when at least one foreground pixel
    seed: int = 0
    frame_index: int = 0
    ramps: List[Ramp] = field(default_factory=list, repr=False)
    rects: Optional[List[Rect]] = field(default=None, repr=False)
    _image: Optional[np.ndarray] = field(default=None, repr=False)
    _mask: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def image(self) -> np.ndarray:
        if self._image is None:
            self._image = render_image(self.ramps, self.height, self.width)
        return self._image

    @property
    def mask(self) -> Optional[np.ndarray]:
        if self.rects is None:
            return None
        if self._mask is None:
            self._mask = paint_mask(self.rects, self.height, self.width)
        return self._mask

    def image_torch(self, device):
        return render_image_torch(self.ramps, self.height, self.width, device)

    def mask_torch(self, device):
        return None if self.rects is None else paint_mask_torch(self.rects, self.height, self.width, device)

    def drop_host(self):
        self._image = None
        self._mask = None


def single_gray(seed: int = 1000, height: int = 256, width: int = 256) -> np.ndarray:
    """The single grayscale frame of the plain (uniform grid) case."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return gradient_image(rng, height, width, 1)


def region_batch(n_frames: int = 64, height: int = 1080, width: int = 1920, seed: int = 1001,
                 philox_seed: int = 1, b: int = 32, sb: int = 8, eps_simple: float = 1.0,
                 eps_complex: float = 0.3, m: int = 16) -> List[FrameSpec]:
    """Batch of RGB frames with 8-rectangle foreground masks (~15% cover)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frames = []
    for f in range(n_frames):
        ramps = [draw_ramp(rng) for _ in range(3)]
        rects = draw_rects(rng, height, width)
        frames.append(FrameSpec(height, width, 3, b, sb, m, eps_simple, eps_complex, 1, philox_seed, f,
                                ramps, rects))
    return frames


def uneven_batch(n_frames: int = 256, seed: int = 1002, philox_seed: int = 2,
                 resolutions=MIXED_RESOLUTIONS, m: int = 16) -> List[FrameSpec]:
    """Uneven batch: resolution uniform over ``resolutions``; per frame
    sb in {4, 8}, b in {16, 32}, eps_complex ~ U[0.1, 0.5], eps_simple ~ U[0.5, 2.0]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frames = []
    for f in range(n_frames):
        h, w = resolutions[int(rng.integers(0, len(resolutions)))]
        sb = int(rng.choice([4, 8]))
        b = int(rng.choice([16, 32]))
        ec = float(rng.uniform(0.1, 0.5))
        es = float(rng.uniform(0.5, 2.0))
        ramps = [draw_ramp(rng) for _ in range(3)]
        rects = draw_rects(rng, h, w)
        frames.append(FrameSpec(h, w, 3, b, sb, m, es, ec, 1, philox_seed, f, ramps, rects))
    return frames


def autograd_batch(n: int = 32, channels: int = 3, height: int = 512, width: int = 512, seed: int = 1003):
    """fp32 (n, C, H, W) images uniform in [0,255), (n, H, W) masks, and a
    fixed N(0,1) weight of the same shape as the images for a linear loss."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = uniform_f32(rng, (n, channels, height, width))
    masks = np.stack([rect_mask(rng, height, width) for _ in range(n)])
    w = rng.standard_normal((n, channels, height, width)).astype(np.float32)
    return x, masks, w


class MovingRects:
    """Foreground of one camera stream: rectangles moving at constant velocity
    and bouncing off the frame edges (~15% of the area in total)."""

    def __init__(self, rng: np.random.Generator, height: int, width: int, n_rects: int = 8,
                 rect_frac: float = 0.02):
        self.h, self.w = height, width
        self.rects = []
        for (y, x, rh, rw) in draw_rects(rng, height, width, n_rects, rect_frac):
            vy, vx = rng.uniform(-0.01, 0.01, size=2) * np.array([height, width])
            self.rects.append([float(y), float(x), rh, rw, float(vy), float(vx)])

    def step(self) -> List[Rect]:
        out = []
        for r in self.rects:
            y, x, rh, rw, vy, vx = r
            y, x = y + vy, x + vx
            if y < 0 or y > self.h - rh:
                vy = -vy
                y = min(max(y, 0.0), float(self.h - rh))
            if x < 0 or x > self.w - rw:
                vx = -vx
                x = min(max(x, 0.0), float(self.w - rw))
            r[:] = [y, x, rh, rw, vy, vx]
            out.append((int(y), int(x), rh, rw))
        return out


#: the 16 camera streams of the serving workload: (height, width, count)
STREAM_MIX = ((1080, 1920, 8), (576, 768, 6), (2160, 3840, 2))


def poisson_arrivals(rng: np.random.Generator, rate_hz: float, duration_s: float) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate on [0, duration)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.asarray(out)
        out.append(t)
