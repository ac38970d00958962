"""Region-adaptive differentially private pixelization on AMD MI355X.

Python face of libdppix (``include/dppix.h``).  The method (Liu, arXiv
2511.04261, Algorithms 2 and 3): cut each frame into b x b cells, split cells
a foreground mask marks as complex into n x n subcells of size s_b = b / n,
release every cell or subcell mean plus Laplace noise of scale
255 m / (area * eps), clipped to [0, 255], keep only those statistics and the
layout (Table IV), and rebuild the frame by broadcasting them.

PyTorch supplies device memory and streams; every step of the method runs in
the HIP kernels of libdppix.  Names follow the paper: ``b`` (grid size of
simple cells), ``sb`` (s_b, subgrid size of complex cells), ``m``, ``eps``.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

from . import _lib
from ._lib import DppixError, F32_CHW, PAD_NONE, PAD_REFLECT, PAD_SYMMETRIC, U8_HWC

__all__ = ["FrameParams", "Plan", "Graph", "DppixError", "pixelize", "DPPixFn", "debug_philox",
           "U8_HWC", "F32_CHW", "PAD_SYMMETRIC", "PAD_REFLECT", "PAD_NONE"]


def _torch():
    import torch
    return torch


@dataclass
class FrameParams:
    """Parameters of one frame (Algorithm 3 inputs).

    ``b``: grid size of simple cells; ``sb``: subgrid size of complex cells
    (defaults to ``b``: Algorithm 2); ``eps_bg`` / ``eps_fg``: budgets of the
    two regions (``math.inf``: no noise); ``tau``: a cell is complex when at
    least ``tau`` of its mask pixels are nonzero (0: the paper's majority rule).
    """
    height: int
    width: int
    channels: int = 1
    layout: int = U8_HWC
    b: int = 16
    sb: Optional[int] = None
    m: int = 16
    eps_bg: float = 0.5
    eps_fg: Optional[float] = None
    tau: int = 0
    pad_mode: int = PAD_SYMMETRIC
    seed: int = 0
    frame_index: int = 0
    pitch: Optional[int] = None
    tile_cells: int = 0

    def desc(self) -> _lib.FrameDesc:
        sb = self.b if self.sb is None else self.sb
        eps_fg = self.eps_bg if self.eps_fg is None else self.eps_fg
        if self.pitch is not None:
            pitch = self.pitch
        else:
            pitch = self.width * self.channels if self.layout == U8_HWC else self.width
        return _lib.FrameDesc(self.height, self.width, self.channels, self.layout, pitch, self.pad_mode,
                              self.b, sb, self.m, float(self.eps_bg), float(eps_fg), self.tau, self.tile_cells,
                              self.seed & (2**64 - 1), self.frame_index & (2**64 - 1))

    @classmethod
    def from_spec(cls, spec, layout: int = U8_HWC) -> "FrameParams":
        """From a ``synth.FrameSpec``."""
        return cls(spec.height, spec.width, spec.channels, layout, spec.b, spec.sb, spec.m, spec.eps_simple,
                   spec.eps_complex, spec.tau, PAD_SYMMETRIC, spec.seed, spec.frame_index)


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Plan of a batch of frames bound to device workspace and store buffers.

    A plan is used by one call sequence at a time (plan -> forward ->
    reconstruct/backward); calls are stream-ordered and never synchronise.
    """

    def __init__(self, frames: Sequence[FrameParams], device=None, threads: int = 0, persistent: int = 0):
        torch = _torch()
        self.lib = _lib.load()
        self.frames = list(frames)
        n = len(self.frames)
        descs = (_lib.FrameDesc * n)(*[f.desc() for f in self.frames])
        h = ctypes.c_void_p()
        _lib.check(self.lib.dp_pix_plan_create(descs, n, ctypes.byref(h)))
        self.handle = h
        self.device = torch.device(device if device is not None else "cuda")
        sz = _lib.Sizes()
        _lib.check(self.lib.dp_pix_plan_sizes(self.handle, ctypes.byref(sz)))
        self.sizes = sz
        self.info = []
        for i in range(n):
            fi = _lib.FrameInfo()
            _lib.check(self.lib.dp_pix_plan_frame_info(self.handle, i, ctypes.byref(fi)))
            self.info.append(fi)
        dev = self.device
        self.workspace = torch.empty(max(sz.workspace_bytes, 256), dtype=torch.uint8, device=dev)
        self.bg = torch.empty(max(sz.bg_capacity, 1), dtype=torch.float32, device=dev)
        self.fg = torch.empty(max(sz.fg_capacity, 1), dtype=torch.float32, device=dev)
        self.flags = torch.empty(max(sz.flag_bytes, 1), dtype=torch.uint8, device=dev)
        self.counts = torch.zeros((n, 4), dtype=torch.int64, device=dev)
        self.store = _lib.Store(self.bg.data_ptr(), self.fg.data_ptr(), self.flags.data_ptr(), self.counts.data_ptr())
        self.set_launch(threads, persistent)
        _lib.check(self.lib.dp_pix_plan_bind(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                             self.workspace.numel(), _stream_handle()))
        self._tables = {}

    # -- plumbing ---------------------------------------------------------
    def set_launch(self, threads: int = 0, persistent: int = 0):
        """threads per workgroup (0: default); persistent: 0 one workgroup per
        tile, 1 a resident grid pulling tiles from a ticket, k >= 2 k per CU."""
        _lib.check(self.lib.dp_pix_plan_set_launch(self.handle, int(threads), int(persistent)))
        self.threads, self.persistent = threads, int(persistent)

    def pointer_table(self, tensors: Optional[Sequence]):
        """Device array of device pointers (None entries -> NULL)."""
        torch = _torch()
        if tensors is None:
            return None
        ptrs = [0 if t is None else t.data_ptr() for t in tensors]
        if len(ptrs) != len(self.frames):
            raise ValueError("need one tensor per frame (%d), got %d" % (len(self.frames), len(ptrs)))
        key = tuple(ptrs)
        tab = self._tables.get(key)
        if tab is None:
            tab = torch.tensor(ptrs, dtype=torch.int64).to(self.device)
            self._tables[key] = tab
        return tab

    def _check_images(self, tensors, what):
        torch = _torch()
        for fp, t in zip(self.frames, tensors):
            if t.device.type != "cuda":
                raise ValueError("%s must be on the GPU" % what)
            if fp.layout == U8_HWC:
                if t.dtype != torch.uint8 or tuple(t.shape[:2]) != (fp.height, fp.width) or \
                        (t.dim() == 3 and t.shape[2] != fp.channels) or (t.dim() == 2 and fp.channels != 1):
                    raise ValueError("%s: expected uint8 (%d, %d, %d)" % (what, fp.height, fp.width, fp.channels))
                pitch = fp.pitch if fp.pitch is not None else fp.width * fp.channels
                if t.stride(0) != pitch or (t.dim() == 3 and (t.stride(1) != fp.channels or t.stride(2) != 1)):
                    raise ValueError("%s: row pitch must be %d bytes, pixels interleaved" % (what, pitch))
            else:
                if t.dtype != torch.float32 or tuple(t.shape) != (fp.channels, fp.height, fp.width):
                    raise ValueError("%s: expected float32 (%d, %d, %d)" % (what, fp.channels, fp.height, fp.width))
                pitch = fp.pitch if fp.pitch is not None else fp.width
                if t.stride(2) != 1 or t.stride(1) != pitch or t.stride(0) != pitch * fp.height:
                    raise ValueError("%s: CHW planes with row pitch %d floats expected" % (what, pitch))

    # -- the method ----------------------------------------------------------
    def plan(self, masks=None, stream=None):
        """Classify cells from the masks (Algorithm 3 steps 3-6) and lay out the store."""
        torch = _torch()
        if masks is not None:
            for fp, mk in zip(self.frames, masks):
                if mk is not None and (mk.dtype != torch.uint8 or tuple(mk.shape) != (fp.height, fp.width)
                                       or not mk.is_contiguous()):
                    raise ValueError("mask must be contiguous uint8 (%d, %d)" % (fp.height, fp.width))
        tab = self.pointer_table(masks)
        _lib.check(self.lib.dp_pix_plan(self.handle, None if tab is None else ctypes.c_void_p(tab.data_ptr()),
                                        ctypes.byref(self.store), _stream_handle(stream)))

    def edge_masks(self, images, threshold: int, out=None, stream=None):
        """Sobel complexity labels of uint8 frames (one (H, W) uint8 mask per
        frame, 1 where |Gx| + |Gy| of the channel sum >= threshold * C), ready
        for ``plan``."""
        torch = _torch()
        self._check_images(images, "images")
        if out is None:
            out = [torch.empty((fp.height, fp.width), dtype=torch.uint8, device=self.device) for fp in self.frames]
        it = self.pointer_table(images)
        mt = self.pointer_table(out)
        _lib.check(self.lib.dp_pix_edge_mask(self.handle, ctypes.c_void_p(it.data_ptr()), int(threshold),
                                             ctypes.c_void_p(mt.data_ptr()), _stream_handle(stream)))
        return out

    def metrics(self, images, recons, stream=None):
        """Per-frame (MSE, SSIM) between uint8 frames and their reconstructions,
        computed on the GPU; returns a (n_frames, 2) float64 tensor on the device."""
        torch = _torch()
        self._check_images(images, "images")
        self._check_images(recons, "recons")
        scratch = torch.empty(max(self.sizes.metrics_scratch_bytes, 256), dtype=torch.uint8, device=self.device)
        out = torch.empty((len(self.frames), 2), dtype=torch.float64, device=self.device)
        it = self.pointer_table(images)
        rt = self.pointer_table(recons)
        _lib.check(self.lib.dp_pix_metrics(self.handle, ctypes.c_void_p(it.data_ptr()), ctypes.c_void_p(rt.data_ptr()),
                                           ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def forward(self, images, out=None, clip=None, stream=None):
        """Noisy statistics into the store; with ``out`` also the reconstruction.
        ``clip``: optional (clip_bg, clip_fg) uint8 tensors of the store's capacities."""
        self._check_images(images, "images")
        if out is not None:
            self._check_images(out, "out")
        it = self.pointer_table(images)
        ot = self.pointer_table(out)
        cb = ctypes.c_void_p(clip[0].data_ptr()) if clip is not None else None
        cf = ctypes.c_void_p(clip[1].data_ptr()) if clip is not None else None
        _lib.check(self.lib.dp_pix_forward(self.handle, ctypes.c_void_p(it.data_ptr()), ctypes.byref(self.store), cb,
                                           cf, None if ot is None else ctypes.c_void_p(ot.data_ptr()),
                                           _stream_handle(stream)))

    def reconstruct(self, out, stream=None):
        """Rebuild frames from the store (Sec. VI-F)."""
        self._check_images(out, "out")
        ot = self.pointer_table(out)
        _lib.check(self.lib.dp_pix_reconstruct(self.handle, ctypes.byref(self.store), ctypes.c_void_p(ot.data_ptr()),
                                               _stream_handle(stream)))

    def backward(self, grad_out, grad_in, clip, scratch=None, stream=None):
        """Adjoint for F32_CHW frames (noise and mask fixed)."""
        torch = _torch()
        self._check_images(grad_out, "grad_out")
        self._check_images(grad_in, "grad_in")
        if scratch is None:
            scratch = torch.empty(max(self.sizes.grad_scratch_bytes, 256), dtype=torch.uint8, device=self.device)
        gt = self.pointer_table(grad_out)
        it = self.pointer_table(grad_in)
        _lib.check(self.lib.dp_pix_backward(self.handle, ctypes.byref(self.store), ctypes.c_void_p(gt.data_ptr()),
                                            ctypes.c_void_p(clip[0].data_ptr()), ctypes.c_void_p(clip[1].data_ptr()),
                                            ctypes.c_void_p(it.data_ptr()), ctypes.c_void_p(scratch.data_ptr()),
                                            scratch.numel(), _stream_handle(stream)))

    def debug_sums(self, images, stream=None):
        """Forward that also returns dense exact sums (coarse, fine) as uint32 tensors."""
        torch = _torch()
        self._check_images(images, "images")
        ncell = sum(fi.grid_rows * fi.grid_cols * fp.channels for fi, fp in zip(self.info, self.frames))
        nfine = sum(fi.grid_rows * fi.grid_cols * fi.n * fi.n * fp.channels for fi, fp in zip(self.info, self.frames))
        coarse = torch.zeros(max(ncell, 1), dtype=torch.int32, device=self.device)
        fine = torch.zeros(max(nfine, 1), dtype=torch.int32, device=self.device)
        it = self.pointer_table(images)
        _lib.check(self.lib.dp_pix_debug_sums(self.handle, ctypes.c_void_p(it.data_ptr()), ctypes.byref(self.store),
                                              ctypes.c_void_p(coarse.data_ptr()), ctypes.c_void_p(fine.data_ptr()),
                                              _stream_handle(stream)))
        return coarse, fine

    def clip_buffers(self):
        torch = _torch()
        return (torch.empty(max(self.sizes.clip_bytes_bg, 1), dtype=torch.uint8, device=self.device),
                torch.empty(max(self.sizes.clip_bytes_fg, 1), dtype=torch.uint8, device=self.device))

    def bound_calls(self, masks, images, out=None, stream=None, clip=None):
        """Validate once and return zero-argument callables ``(plan, forward)``
        that issue dp_pix_plan / dp_pix_forward on ``stream`` with the
        arguments already marshalled (for back-to-back launches)."""
        self._check_images(images, "images")
        if out is not None:
            self._check_images(out, "out")
        mt = self.pointer_table(masks)
        it = self.pointer_table(images)
        ot = self.pointer_table(out)
        lib, h, st, s = self.lib, self.handle, ctypes.byref(self.store), _stream_handle(stream)
        mp = None if mt is None else ctypes.c_void_p(mt.data_ptr())
        ip = ctypes.c_void_p(it.data_ptr())
        op = None if ot is None else ctypes.c_void_p(ot.data_ptr())
        cb = None if clip is None else ctypes.c_void_p(clip[0].data_ptr())
        cf = None if clip is None else ctypes.c_void_p(clip[1].data_ptr())
        keep = (mt, it, ot, clip)

        def plan_call():
            _lib.check(lib.dp_pix_plan(h, mp, st, s))

        def forward_call():
            _lib.check(lib.dp_pix_forward(h, ip, st, cb, cf, op, s))

        plan_call.keep = forward_call.keep = keep
        return plan_call, forward_call

    def bound_backward(self, grad_out, grad_in, clip, scratch, stream=None):
        """Validate once and return a zero-argument callable issuing
        dp_pix_backward with the arguments already marshalled."""
        self._check_images(grad_out, "grad_out")
        self._check_images(grad_in, "grad_in")
        gt = self.pointer_table(grad_out)
        it = self.pointer_table(grad_in)
        lib, h, st, s = self.lib, self.handle, ctypes.byref(self.store), _stream_handle(stream)
        args = (ctypes.c_void_p(gt.data_ptr()), ctypes.c_void_p(clip[0].data_ptr()),
                ctypes.c_void_p(clip[1].data_ptr()), ctypes.c_void_p(it.data_ptr()),
                ctypes.c_void_p(scratch.data_ptr()), scratch.numel())

        def backward_call():
            _lib.check(lib.dp_pix_backward(h, st, args[0], args[1], args[2], args[3], args[4], args[5], s))

        backward_call.keep = (gt, it, clip, scratch)
        return backward_call

    def graph(self, masks, images, out=None, stream=None) -> "Graph":
        """Capture plan + forward (+ fused reconstruction) into a HIP graph."""
        return Graph(self, masks, images, out, stream)

    # -- host views --------------------------------------------------------
    def store_host(self):
        """Copy the store to the host and split it per frame (synchronises)."""
        import numpy as np
        counts = self.counts.cpu().numpy()
        bg = self.bg.cpu().numpy()
        fg = self.fg.cpu().numpy()
        flags = self.flags.cpu().numpy()
        out = []
        for f, (fp, fi) in enumerate(zip(self.frames, self.info)):
            nb, nf, ob, of = (int(x) for x in counts[f])
            C, nn = fp.channels, fi.n * fi.n
            out.append(dict(
                flags=flags[fi.cell_offset: fi.cell_offset + fi.grid_rows * fi.grid_cols].reshape(fi.grid_rows, fi.grid_cols),
                bg=bg[ob: ob + nb * C].reshape(nb, C), fg=fg[of: of + nf * nn * C].reshape(nf, nn, C),
                counts=(nb, nf), offsets=(ob, of)))
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.dp_pix_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """plan + forward (+ fused reconstruction) captured once, replayed per step.
    The kernels read the pointer tables at replay time: refill the same image,
    mask and output buffers between launches."""

    def __init__(self, plan: Plan, masks, images, out=None, stream=None):
        self.plan = plan
        plan._check_images(images, "images")
        self.mt = plan.pointer_table(masks)
        self.it = plan.pointer_table(images)
        self.ot = plan.pointer_table(out)
        h = ctypes.c_void_p()
        _lib.check(plan.lib.dp_pix_graph_create(
            plan.handle, None if self.mt is None else ctypes.c_void_p(self.mt.data_ptr()),
            ctypes.c_void_p(self.it.data_ptr()), ctypes.byref(plan.store),
            None if self.ot is None else ctypes.c_void_p(self.ot.data_ptr()), _stream_handle(stream),
            ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _lib.check(self.plan.lib.dp_pix_graph_launch(self.handle, _stream_handle(stream)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.plan.lib.dp_pix_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_philox(blocks):
    """Raw Philox4x32-10 words for an (n, 6) uint32 tensor of (ctr0..3, key0, key1) on the GPU."""
    torch = _torch()
    lib = _lib.load()
    x = blocks.to(torch.int32).contiguous()
    out = torch.empty((x.shape[0], 4), dtype=torch.int32, device=x.device)
    _lib.check(lib.dp_pix_debug_philox(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.shape[0],
                                       _stream_handle()))
    return out


def pixelize(image, mask=None, b: int = 16, sb: Optional[int] = None, m: int = 16, eps_bg: float = 0.5,
             eps_fg: Optional[float] = None, tau: int = 0, seed: int = 0, frame_index: int = 0,
             pad_mode: int = PAD_SYMMETRIC):
    """One frame, end to end: returns (reconstruction, per-frame store dict on the host).
    (seed, frame_index) is the frame's Philox counter: every released frame
    needs its own, or frames released with equal noise give away the exact
    difference of their true cell means."""
    torch = _torch()
    if image.dtype == torch.uint8:
        img = image if image.dim() == 3 else image.unsqueeze(-1)
        H, W, C = img.shape
        fp = FrameParams(H, W, C, U8_HWC, b, sb, m, eps_bg, eps_fg, tau, pad_mode, seed, frame_index)
    else:
        img = image
        C, H, W = img.shape
        fp = FrameParams(H, W, C, F32_CHW, b, sb, m, eps_bg, eps_fg, tau, pad_mode, seed, frame_index)
    img = img.contiguous()
    plan = Plan([fp], device=img.device)
    plan.plan(None if mask is None else [mask.contiguous()])
    out = torch.empty_like(img)
    plan.forward([img], out=[out])
    store = plan.store_host()[0]
    return (out if image.dim() == img.dim() else out.squeeze(-1)), store


from .autograd import DPPixFn, DPPixLayer  # noqa: E402
