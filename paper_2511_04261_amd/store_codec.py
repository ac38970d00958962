"""Compact-store codec and storage study.

The paper keeps, instead of the pixelated frame, only the noisy cell means,
the region indicator per grid cell, the two grid sizes and the frame size
(Table III, Table IV, Sec. V-D and VI-F), saved as compressed arrays with the
means quantised to uint8.  This codec writes one frame's store in that spirit:

  magic "DPPX", version, header (geometry, the frame's privacy ledger, its
  noise counter, counts), deflate-compressed payload = region flags packed
  to bits, then the statistics as uint8 (rounded half to even, exactly the
  values the uint8 reconstruction shows) or as fp32.

The generator's key (the seed) is never written: whoever knows it can
regenerate the noise and subtract it.  The frame_index (the counter) may be
published; it identifies the draws without revealing them.

A uint8 store rebuilds exactly the uint8 reconstruction; an fp32 store keeps
the released values themselves.  ``storage_study`` measures encoded sizes
against PNG of the reconstructed frame over grid sizes and subgrid factors.
"""
from __future__ import annotations

import io
import math
import struct
import zlib
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

MAGIC = b"DPPX"
VERSION = 2
Q_U8, Q_F32 = 0, 1
# magic, version, quant, H, W, C, b, sb, pad, m, eps_bg, eps_fg, eps_frame, eps_pixel, frame_index, n_bg, n_fg
_HDR = struct.Struct("<4sBBxx7i4dQ2I")


def privacy_ledger(channels: int, m: int, eps_bg: float, eps_fg: float) -> dict:
    """Privacy accounting of one released frame.

    Simple cells and complex subcells cover disjoint pixels and each draws its
    own noise, so by parallel composition (Thm. 1) the frame is
    max(eps_bg, eps_fg)-DP for neighbouring frames that differ in at most m
    values of one channel (the paper's grayscale setting, per channel).  For
    neighbours differing in m whole pixels, all C channels' statistics move
    and compose sequentially: C * max(eps_bg, eps_fg).  (The paper's scale
    ignores mirrored duplicates at padded borders; such a cell can leak up to
    four times its budget, and none at all when b divides the frame.)"""
    e = max(float(eps_bg), float(eps_fg))
    return dict(m=int(m), eps_bg=float(eps_bg), eps_fg=float(eps_fg), eps_frame=e,
                eps_pixel=channels * e if not math.isinf(e) else math.inf)


def encode(store: dict, height: int, width: int, channels: int, b: int, sb: int, m: int, eps_bg: float,
           eps_fg: float, frame_index: int = 0, pad_mode: int = 0, quant: int = Q_U8, level: int = 9) -> bytes:
    """One frame's store (dict with flags (G_R, G_C), bg (n_bg, C), fg (n_fg, n*n, C)) -> bytes."""
    flags = np.ascontiguousarray(store["flags"], np.uint8)
    bg = np.asarray(store["bg"], np.float32)
    fg = np.asarray(store["fg"], np.float32)
    n_bg, n_fg = bg.shape[0], fg.shape[0]
    if int(flags.sum()) != n_fg or flags.size != n_bg + n_fg:
        raise ValueError("flags do not match the statistic counts")
    led = privacy_ledger(channels, m, eps_bg, eps_fg)
    hdr = _HDR.pack(MAGIC, VERSION, quant, height, width, channels, b, sb, pad_mode, m, led["eps_bg"],
                    led["eps_fg"], led["eps_frame"], led["eps_pixel"], frame_index & (2**64 - 1), n_bg, n_fg)
    if quant == Q_U8:
        stats = np.concatenate([np.rint(bg).reshape(-1), np.rint(fg).reshape(-1)]).astype(np.uint8)
    elif quant == Q_F32:
        stats = np.concatenate([bg.reshape(-1), fg.reshape(-1)]).astype("<f4")
    else:
        raise ValueError("unknown quantisation")
    payload = np.packbits(flags.reshape(-1)).tobytes() + stats.tobytes()
    return hdr + zlib.compress(payload, level)


def decode(blob: bytes) -> Tuple[dict, dict]:
    """bytes -> (header dict with the privacy ledger, store dict with flags, bg, fg as float32)."""
    if len(blob) < _HDR.size:
        raise ValueError("truncated store")
    (magic, ver, quant, H, W, C, b, sb, pad, m, eps_bg, eps_fg, eps_frame, eps_pixel, fi, n_bg,
     n_fg) = _HDR.unpack_from(blob)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("not a dppix store (magic %r, version %d)" % (magic, ver))
    if b < 1 or sb < 1 or b % sb or H < 1 or W < 1 or C < 1:
        raise ValueError("invalid geometry in the header")
    GR, GC, n = -(-H // b), -(-W // b), b // sb
    if n_bg + n_fg != GR * GC:
        raise ValueError("counts do not cover the grid")
    payload = zlib.decompress(blob[_HDR.size:])
    nflag = (GR * GC + 7) // 8
    flags = np.unpackbits(np.frombuffer(payload[:nflag], np.uint8))[: GR * GC].reshape(GR, GC)
    if int(flags.sum()) != n_fg:
        raise ValueError("flags do not match the counts")
    rest = payload[nflag:]
    count = n_bg * C + n_fg * n * n * C
    if quant == Q_U8:
        stats = np.frombuffer(rest, np.uint8, count).astype(np.float32)
    else:
        stats = np.frombuffer(rest, "<f4", count).astype(np.float32)
    bg = stats[: n_bg * C].reshape(n_bg, C)
    fg = stats[n_bg * C:].reshape(n_fg, n * n, C)
    hdr = dict(height=H, width=W, channels=C, b=b, sb=sb, pad_mode=pad, frame_index=fi, quant=quant,
               ledger=dict(m=m, eps_bg=eps_bg, eps_fg=eps_fg, eps_frame=eps_frame, eps_pixel=eps_pixel))
    return hdr, dict(flags=flags, bg=bg, fg=fg, counts=(n_bg, n_fg))


def png_size(image: np.ndarray) -> int:
    """Bytes of a PNG of an (H, W) or (H, W, C) uint8 frame (PIL, default settings)."""
    from PIL import Image
    buf = io.BytesIO()
    arr = image[:, :, 0] if image.ndim == 3 and image.shape[2] == 1 else image
    Image.fromarray(np.ascontiguousarray(arr)).save(buf, format="PNG")
    return buf.tell()


def storage_study(specs: Sequence, grid_sizes: Sequence[int] = (4, 8, 16, 32, 64, 128),
                  factors: Sequence[int] = (1, 2, 4, 8), device=None, m: int = 16, eps: float = 0.5,
                  keep_blobs: bool = False) -> list:
    """Encoded store size vs PNG of the reconstruction, per (b, n), summed over
    the given frames (synth.FrameSpec with masks).  Runs the GPU path.  With
    keep_blobs, each row also carries the encoded stores ("blobs_u8",
    "blobs_f32", one per frame) and the frame parameters ("frames")."""
    import torch
    import paper_2511_04261_amd as dp
    dev = torch.device(device if device is not None else "cuda:0")
    rows = []
    imgs = [s.image_torch(dev) for s in specs]
    masks = [s.mask_torch(dev) for s in specs]
    for b in grid_sizes:
        for nf in factors:
            if b % nf:
                continue
            sb = b // nf
            frames = [dp.FrameParams(s.height, s.width, s.channels, dp.U8_HWC, b, sb, m, eps, eps, 1,
                                     dp.PAD_SYMMETRIC, s.seed, s.frame_index) for s in specs]
            plan = dp.Plan(frames, device=dev)
            outs = [torch.empty_like(t) for t in imgs]
            plan.plan(masks)
            plan.forward(imgs, out=outs)
            torch.cuda.synchronize()
            st = plan.store_host()
            u8 = f32 = png = 0
            b8, b32 = [], []
            for k, s in enumerate(specs):
                kw = dict(height=s.height, width=s.width, channels=s.channels, b=b, sb=sb, m=m, eps_bg=eps,
                          eps_fg=eps, frame_index=s.frame_index)
                e8, e32 = encode(st[k], quant=Q_U8, **kw), encode(st[k], quant=Q_F32, **kw)
                u8 += len(e8)
                f32 += len(e32)
                png += png_size(outs[k].cpu().numpy())
                if keep_blobs:
                    b8.append(e8)
                    b32.append(e32)
            row = dict(b=b, n=nf, sb=sb, store_u8=u8, store_f32=f32, png=png, ratio_u8_png=round(u8 / png, 4),
                       frames=len(specs))
            if keep_blobs:
                row.update(blobs_u8=b8, blobs_f32=b32, frames_params=frames)
            rows.append(row)
            plan.close()
    return rows
