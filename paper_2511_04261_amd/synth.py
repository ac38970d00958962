"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper measures on surveillance video (768x576 and 1920x1080 frames,
Sec. VII-A) and portrait photos with foreground masks (Sec. VII-B); those
datasets are not available, so these generators stand in for them: smooth
gradients plus uniform pixel noise for the frames, and unions of axis-aligned
rectangles for the foreground masks.

This module holds no part of the pixelization arithmetic; it only draws
numbers.  Every generator takes a numpy PCG64 seed and is deterministic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

#: resolutions of the uneven batch: the two video sizes of the paper's
#: runtime study, UHD, and a 24 MP still
MIXED_RESOLUTIONS = ((576, 768), (1080, 1920), (2160, 3840), (4000, 6000))


def gradient_image(rng: np.random.Generator, height: int, width: int, channels: int = 1) -> np.ndarray:
    """uint8 (H, W, C): per channel a linear ramp of amplitude A ~ U[60,100] along a
    random direction theta ~ U[0, 2pi), centred on 128, plus integer noise
    U{-20..20}, clamped to [0, 255]."""
    out = np.empty((height, width, channels), np.uint8)
    ii = np.arange(height, dtype=np.float64)[:, None] - (height - 1) / 2.0
    jj = np.arange(width, dtype=np.float64)[None, :] - (width - 1) / 2.0
    half = max(height - 1, width - 1, 1) / 2.0
    for ch in range(channels):
        amp = rng.uniform(60.0, 100.0)
        theta = rng.uniform(0.0, 2.0 * math.pi)
        ramp = 128.0 + amp * (ii * math.cos(theta) + jj * math.sin(theta)) / half
        noise = rng.integers(-20, 21, size=(height, width))
        out[:, :, ch] = np.clip(np.round(ramp) + noise, 0, 255).astype(np.uint8)
    return out


def rect_mask(rng: np.random.Generator, height: int, width: int, n_rects: int = 8,
              rect_frac: float = 0.02, cover: tuple = (0.13, 0.17), max_tries: int = 200) -> np.ndarray:
    """uint8 (H, W) foreground mask (1 = foreground): the union of ``n_rects``
    axis-aligned rectangles, each of area ~rect_frac*H*W with aspect ratio
    U[0.5, 2], uniformly placed; redrawn until the union covers ``cover``."""
    best = None
    for _ in range(max_tries):
        mk = np.zeros((height, width), np.uint8)
        for _r in range(n_rects):
            aspect = rng.uniform(0.5, 2.0)
            area = rect_frac * height * width
            h = max(1, min(height, int(round(math.sqrt(area / aspect)))))
            w = max(1, min(width, int(round(math.sqrt(area * aspect)))))
            y = int(rng.integers(0, height - h + 1))
            x = int(rng.integers(0, width - w + 1))
            mk[y:y + h, x:x + w] = 1
        frac = mk.mean()
        if cover[0] <= frac <= cover[1]:
            return mk
        if best is None or abs(frac - sum(cover) / 2) < abs(best[0] - sum(cover) / 2):
            best = (frac, mk)
    return best[1]


def uniform_f32(rng: np.random.Generator, shape) -> np.ndarray:
    """fp32 values uniform in [0, 255)."""
    return (rng.random(shape, dtype=np.float64) * 255.0).astype(np.float32)


@dataclass
class FrameSpec:
    """One frame of a batch: geometry plus per-region parameters."""
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
    image: np.ndarray = field(default=None, repr=False)
    mask: np.ndarray = field(default=None, repr=False)


def single_gray(seed: int = 1000, height: int = 256, width: int = 256) -> np.ndarray:
    """The single 256x256 grayscale frame of the plain (uniform grid) case."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return gradient_image(rng, height, width, 1)


def region_batch(n_frames: int = 64, height: int = 1080, width: int = 1920, seed: int = 1001,
                 philox_seed: int = 1, b: int = 32, sb: int = 8, eps_simple: float = 1.0,
                 eps_complex: float = 0.3, m: int = 16, with_data: bool = True):
    """Batch of RGB frames with 8-rectangle foreground masks (~15% cover)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frames = []
    for f in range(n_frames):
        spec = FrameSpec(height, width, 3, b, sb, m, eps_simple, eps_complex, 1, philox_seed, f)
        if with_data:
            spec.image = gradient_image(rng, height, width, 3)
            spec.mask = rect_mask(rng, height, width)
        frames.append(spec)
    return frames


def uneven_batch(n_frames: int = 256, seed: int = 1002, philox_seed: int = 2, with_data: bool = True,
                 resolutions=MIXED_RESOLUTIONS, m: int = 16):
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
        spec = FrameSpec(h, w, 3, b, sb, m, es, ec, 1, philox_seed, f)
        if with_data:
            spec.image = gradient_image(rng, h, w, 3)
            spec.mask = rect_mask(rng, h, w)
        frames.append(spec)
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
        for _ in range(n_rects):
            aspect = rng.uniform(0.5, 2.0)
            area = rect_frac * height * width
            rh = max(1, min(height, int(round(math.sqrt(area / aspect)))))
            rw = max(1, min(width, int(round(math.sqrt(area * aspect)))))
            y = rng.uniform(0, height - rh)
            x = rng.uniform(0, width - rw)
            vy, vx = rng.uniform(-0.01, 0.01, size=2) * np.array([height, width])
            self.rects.append([y, x, rh, rw, vy, vx])

    def step(self) -> np.ndarray:
        mk = np.zeros((self.h, self.w), np.uint8)
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
            mk[int(y):int(y) + rh, int(x):int(x) + rw] = 1
        return mk


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
