"""Parameter sweeps of the paper's evaluation (Sec. VII-A and VII-B) on
synthetic frames, run end to end on the GPU: utility (MSE, SSIM from
dp_pix_metrics) and GPU time per frame.

  grid:    eps = 0.5, m = 16, b = 2 .. 20          (the paper's first sweep)
  m:       b = 16, eps = 0.5, m = 4 .. 256         (second sweep)
  eps:     b = 16, m = 16, eps = 0.1 .. 2.0        (third sweep)
  region:  region-adaptive, m = 32, eps = 0.5, b x n grid (Sec. VII-B shape)

Frames: grayscale 768x576 and 1920x1080 (the sizes of the paper's video
sets) and RGB 512x512 with a rectangle foreground for the region sweep.

    python -m paper_2511_04261_amd.sweeps --out sweeps.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def _frames(n, H, W, C, seed, masks=False):
    from . import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n):
        ramps = [synth.draw_ramp(rng) for _ in range(C)]
        rects = synth.draw_rects(rng, H, W, n_rects=2, rect_frac=0.12, cover=(0.2, 0.35)) if masks else None
        specs.append(synth.FrameSpec(H, W, C, ramps=ramps, rects=rects, frame_index=i))
    return specs


def run_point(specs, imgs, masks, dev, b, sb, m, eps, reps=5):
    """One parameter point: (mean MSE, mean SSIM, GPU ms per frame for plan + forward)."""
    import torch
    import paper_2511_04261_amd as dp
    frames = [dp.FrameParams(s.height, s.width, s.channels, dp.U8_HWC, b, sb, m, eps, eps, 1, dp.PAD_SYMMETRIC,
                             7, s.frame_index) for s in specs]
    plan = dp.Plan(frames, device=dev)
    outs = [torch.empty_like(t) for t in imgs]
    plan.plan(masks)
    plan.forward(imgs, out=outs)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.plan(masks)
        plan.forward(imgs, out=outs)
    z.record()
    z.synchronize()
    ms = a.elapsed_time(z) / reps / len(specs)
    met = plan.metrics(imgs, outs).cpu().numpy()
    plan.close()
    return float(met[:, 0].mean()), float(met[:, 1].mean()), ms


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="sweeps.json")
    ap.add_argument("--frames", type=int, default=16)
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    rows = []

    def emit(**kw):
        rows.append(kw)
        print(json.dumps(kw), flush=True)

    for (H, W, name) in ((576, 768, "768x576"), (1080, 1920, "1920x1080")):
        specs = _frames(args.frames, H, W, 1, 2000 + H)
        imgs = [s.image_torch(dev) for s in specs]
        for b in range(2, 21):
            mse, ssim, ms = run_point(specs, imgs, None, dev, b, b, 16, 0.5)
            emit(sweep="grid", frames=name, b=b, m=16, eps=0.5, mse=mse, ssim=ssim, gpu_ms_per_frame=ms)
        for m in (4, 8, 16, 32, 64, 128, 256):
            mse, ssim, ms = run_point(specs, imgs, None, dev, 16, 16, m, 0.5)
            emit(sweep="m", frames=name, b=16, m=m, eps=0.5, mse=mse, ssim=ssim, gpu_ms_per_frame=ms)
        for eps in (0.1, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0):
            mse, ssim, ms = run_point(specs, imgs, None, dev, 16, 16, 16, eps)
            emit(sweep="eps", frames=name, b=16, m=16, eps=eps, mse=mse, ssim=ssim, gpu_ms_per_frame=ms)
        del imgs
    specs = _frames(args.frames, 512, 512, 3, 3000, masks=True)
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    for b in (8, 16, 32, 64):
        for n in (1, 2, 4, 8):
            if b % n:
                continue
            mse, ssim, ms = run_point(specs, imgs, masks, dev, b, b // n, 32, 0.5)
            emit(sweep="region", frames="512x512x3", b=b, n=n, m=32, eps=0.5, mse=mse, ssim=ssim,
                 gpu_ms_per_frame=ms)
    with open(args.out, "w") as f:
        json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
