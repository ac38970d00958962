"""Shared test plumbing: run frames through the HIP path and through the
oracle on the same seeded inputs, and compare to the bar:
  - flags, store counts and exact sums: bit-exact;
  - noisy fp32 statistics: within 1e-3 absolute (same Philox words, fp64
    transform; only the last bit of the fp64 log may differ);
  - reconstructed uint8: within 1 LSB.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

STAT_TOL = 1e-3
LSB_TOL = 1


def oracle_params(fp):
    """oracle.Params from a paper_2511_04261_amd.FrameParams."""
    sb = fp.b if fp.sb is None else fp.sb
    eps_fg = fp.eps_bg if fp.eps_fg is None else fp.eps_fg
    return oracle.Params(fp.height, fp.width, fp.channels, b=fp.b, sb=sb, m=fp.m, eps_simple=fp.eps_bg,
                         eps_complex=eps_fg, tau=fp.tau, pad_mode=fp.pad_mode, seed=fp.seed,
                         frame_index=fp.frame_index)


def run_gpu(frames, images, masks, device, threads=0, persistent=False, fused=True, reconstruct=True,
            sums=False):
    """frames: FrameParams; images: numpy HWC uint8 (or CHW float32); masks: numpy or None.
    Returns dict(store=[per-frame], fused=[np], recon=[np], coarse=..., fine=...)."""
    import torch
    import paper_2511_04261_amd as dp
    plan = dp.Plan(frames, device=device, threads=threads, persistent=persistent)
    ti = [torch.from_numpy(np.ascontiguousarray(x)).to(device) for x in images]
    tm = None if masks is None else [None if m is None else torch.from_numpy(np.ascontiguousarray(m)).to(device)
                                      for m in masks]
    plan.plan(tm)
    res = {}
    fo = [torch.empty_like(t) for t in ti] if fused else None
    if sums:
        coarse, fine = plan.debug_sums(ti)
        res["coarse"] = coarse.cpu().numpy().view(np.uint32)
        res["fine"] = fine.cpu().numpy().view(np.uint32)
    if fused or not sums:
        plan.forward(ti, out=fo)
    ro = None
    if reconstruct:
        ro = [torch.empty_like(t) for t in ti]
        plan.reconstruct(ro)
    torch.cuda.synchronize()
    res["store"] = plan.store_host()
    res["fused"] = None if fo is None else [t.cpu().numpy() for t in fo]
    res["recon"] = None if ro is None else [t.cpu().numpy() for t in ro]
    res["info"] = plan.info
    res["plan"] = plan
    return res


def compare_frame(got_store, want, got_recon=None, tag=""):
    assert np.array_equal(got_store["flags"], want["flags"]), "%s flags differ" % tag
    assert tuple(got_store["counts"]) == tuple(want["counts"]), "%s counts %s vs %s" % (
        tag, got_store["counts"], want["counts"])
    for k in ("bg", "fg"):
        g, w = got_store[k], want[k]
        assert g.shape == w.shape, "%s %s shape %s vs %s" % (tag, k, g.shape, w.shape)
        if g.size:
            d = np.abs(g.astype(np.float64) - w.astype(np.float64)).max()
            assert d <= STAT_TOL, "%s %s max diff %g" % (tag, k, d)
    if got_recon is not None:
        if got_recon.dtype == np.uint8:
            r = got_recon.reshape(want["recon_u8"].shape)
            d = np.abs(r.astype(np.int16) - want["recon_u8"].astype(np.int16)).max()
            assert d <= LSB_TOL, "%s recon max diff %d" % (tag, d)
        else:
            d = np.abs(got_recon - want["recon_f32"]).max()
            assert d <= STAT_TOL, "%s recon f32 max diff %g" % (tag, d)


def exact_fraction(got_store, want):
    """Fraction of statistics that are bit-identical (expected ~1)."""
    n = eq = 0
    for k in ("bg", "fg"):
        n += want[k].size
        eq += int((got_store[k] == want[k]).sum())
    return 1.0 if n == 0 else eq / n


def chw_to_hwc(x):
    return np.ascontiguousarray(np.transpose(x, (1, 2, 0)))


def hwc_to_chw(x):
    return np.ascontiguousarray(np.transpose(x, (2, 0, 1)))
