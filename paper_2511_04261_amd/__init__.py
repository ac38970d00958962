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

__all__ = ["FrameParams", "Plan", "Store", "Graph", "DppixError", "pixelize", "DPPixFn", "debug_philox",
           "check_masks", "check_no_alias",
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


_SETUP_STREAMS = {}


def _setup_stream(device):
    """A non-blocking stream per device for plan set-up (the table upload that
    dp_pix_plan_bind waits for), so binding a plan never waits for work
    queued on the caller's streams."""
    torch = _torch()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    s = _SETUP_STREAMS.get(idx)
    if s is None:
        s = torch.cuda.Stream(device=torch.device("cuda", idx))
        _SETUP_STREAMS[idx] = s
    return s


def _use_on(tensors, seen, stream):
    """Tell torch's caching allocator that `tensors` are used on `stream` (once
    per stream), so their memory is not handed to another allocation while
    work queued there may still touch it."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    if s.cuda_stream in seen:
        return
    seen.add(s.cuda_stream)
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def _on_device(t, device) -> bool:
    """t is a CUDA tensor on `device` (any CUDA device when it has no index)."""
    return t.device.type == "cuda" and (device.index is None or t.device.index in (None, device.index))


def check_masks(frames, masks, device):
    """Masks must be contiguous uint8 (H, W) CUDA tensors on the plan's
    device (or None): a host tensor's address in the device pointer table
    would be dereferenced by the plan kernel."""
    torch = _torch()
    if masks is None:
        return
    if len(masks) != len(frames):
        raise ValueError("need one mask (or None) per frame (%d), got %d" % (len(frames), len(masks)))
    for fp, mk in zip(frames, masks):
        if mk is None:
            continue
        if not _on_device(mk, device):
            raise ValueError("masks must be CUDA tensors on %s, got one on %s" % (device, mk.device))
        if mk.dtype != torch.uint8 or tuple(mk.shape) != (fp.height, fp.width) or not mk.is_contiguous():
            raise ValueError("mask must be contiguous uint8 (%d, %d)" % (fp.height, fp.width))


def _span(t):
    """Byte range [lo, hi) that a tensor view touches."""
    if t.numel() == 0:
        return (t.data_ptr(), t.data_ptr())
    last = sum((n - 1) * st for n, st in zip(t.shape, t.stride()))
    return (t.data_ptr(), t.data_ptr() + (last + 1) * t.element_size())


def check_no_alias(images, outs):
    """A fused reconstruction must not overlap its image: with mirror padding
    a tile reads rows and columns that other tiles of the same launch write."""
    for i, (x, y) in enumerate(zip(images, outs)):
        a0, a1 = _span(x)
        b0, b1 = _span(y)
        if a0 < b1 and b0 < a1:
            raise ValueError("out[%d] overlaps images[%d]: the forward cannot run in place" % (i, i))


class Store:
    """Device buffers of one compact store of a plan (Table IV: flags, simple
    cell statistics, complex subcell statistics, per-frame counts) and its
    per-call state.  Every call sequence in flight at once (another stream,
    a forward whose backward is still to come) uses its own store.

    ``noise``: optional (n_frames, 2) int64 CUDA tensor of (seed,
    frame_index) per frame, read by the kernels when they run (see
    ``Plan.noise_counters``); None draws with the frames' own parameters."""

    def __init__(self, plan: "Plan", noise=None):
        torch = _torch()
        sz, dev, n = plan.sizes, plan.device, len(plan.frames)
        self.plan_info = (plan.frames, plan.info)
        self.bg = torch.empty(max(sz.bg_capacity, 1), dtype=torch.float32, device=dev)
        self.fg = torch.empty(max(sz.fg_capacity, 1), dtype=torch.float32, device=dev)
        self.flags = torch.empty(max(sz.flag_bytes, 1), dtype=torch.uint8, device=dev)
        self.counts = torch.zeros((n, 4), dtype=torch.int64, device=dev)
        self.state = torch.empty(max(sz.store_state_bytes, 256), dtype=torch.uint8, device=dev)
        self.noise = None
        self._streams = set()
        self.c = _lib.Store(self.bg.data_ptr(), self.fg.data_ptr(), self.flags.data_ptr(), self.counts.data_ptr(),
                            self.state.data_ptr(), None)
        if noise is not None:
            self.set_noise(noise)

    def set_noise(self, noise):
        torch = _torch()
        n = len(self.plan_info[0])
        if noise is not None:
            if noise.dtype != torch.int64 or tuple(noise.shape) != (n, 2) or not noise.is_contiguous() \
                    or noise.device.type != "cuda":
                raise ValueError("noise must be a contiguous (%d, 2) int64 CUDA tensor" % n)
        self.noise = noise
        self.c.noise = None if noise is None else noise.data_ptr()
        self._streams = set()

    def used_on(self, stream):
        """Record that calls with this store run on `stream`."""
        _use_on((self.bg, self.fg, self.flags, self.counts, self.state, self.noise), self._streams, stream)

    def host(self):
        """Copy the store to the host and split it per frame (synchronises).
        Each frame's dict carries its privacy ledger (budgets per region, the
        frame's eps by parallel composition, m, C times it for neighbours that
        differ in whole pixels, and its Philox counter)."""
        from .store_codec import privacy_ledger
        counts = self.counts.cpu().numpy()
        bg = self.bg.cpu().numpy()
        fg = self.fg.cpu().numpy()
        flags = self.flags.cpu().numpy()
        frames, info = self.plan_info
        out = []
        for f, (fp, fi) in enumerate(zip(frames, info)):
            nb, nf, ob, of = (int(x) for x in counts[f])
            C, nn = fp.channels, fi.n * fi.n
            eps_fg = fp.eps_bg if fp.eps_fg is None else fp.eps_fg
            out.append(dict(
                flags=flags[fi.cell_offset: fi.cell_offset + fi.grid_rows * fi.grid_cols].reshape(fi.grid_rows, fi.grid_cols),
                bg=bg[ob: ob + nb * C].reshape(nb, C), fg=fg[of: of + nf * nn * C].reshape(nf, nn, C),
                counts=(nb, nf), offsets=(ob, of),
                ledger=dict(privacy_ledger(C, fp.m, fp.eps_bg, eps_fg), frame_index=fp.frame_index)))
        return out

    def load_host(self, per_frame):
        """Fill flags and statistics from per-frame host dicts (flags (G_R,
        G_C), bg (n_bg, C), fg (n_fg, n*n, C)), packed back to back in batch
        order; call ``Plan.index_store`` before reconstructing from it."""
        import numpy as np
        torch = _torch()
        frames, info = self.plan_info
        flags = np.zeros(self.flags.numel(), np.uint8)
        bgs, fgs = [], []
        for fp, fi, d in zip(frames, info, per_frame):
            cells = fi.grid_rows * fi.grid_cols
            fl = np.asarray(d["flags"], np.uint8).reshape(-1)
            if fl.size != cells:
                raise ValueError("flags of a frame must have G_R * G_C = %d entries" % cells)
            flags[fi.cell_offset: fi.cell_offset + cells] = fl
            nf = int((fl != 0).sum())
            b = np.asarray(d["bg"], np.float32).reshape(-1)
            g = np.asarray(d["fg"], np.float32).reshape(-1)
            if b.size != (cells - nf) * fp.channels or g.size != nf * fi.n * fi.n * fp.channels:
                raise ValueError("statistics do not match the flags")
            bgs.append(b)
            fgs.append(g)
        bg = np.concatenate(bgs) if bgs else np.zeros(0, np.float32)
        fg = np.concatenate(fgs) if fgs else np.zeros(0, np.float32)
        self.flags.copy_(torch.from_numpy(flags))
        if bg.size:
            self.bg[: bg.size].copy_(torch.from_numpy(bg))
        if fg.size:
            self.fg[: fg.size].copy_(torch.from_numpy(fg))


class Plan:
    """Plan of a batch of frames: geometry, tiles and store capacities, bound
    to a device workspace that holds only immutable tables.

    A plan can be used by any number of call sequences at once, each with its
    own ``Store`` (``new_store``); methods use the plan's default store when
    none is given.  Calls are stream-ordered and never synchronise."""

    MAX_TABLES = 64

    def __init__(self, frames: Sequence[FrameParams], device=None, threads: int = 0, persistent: int = 0,
                 default_store: bool = True):
        """default_store=False: no store is allocated for the plan itself
        (every call then names its own ``Store``)."""
        import collections
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
        # the workspace belongs to the set-up stream, which uploads its tables;
        # every stream a call runs on is recorded against it (see _use_on)
        setup = _setup_stream(self.device)
        with torch.cuda.stream(setup):
            self.workspace = torch.empty(max(sz.workspace_bytes, 256), dtype=torch.uint8, device=self.device)
        self._streams = set()
        self.set_launch(threads, persistent)
        _lib.check(self.lib.dp_pix_plan_bind(self.handle, ctypes.c_void_p(self.workspace.data_ptr()),
                                             self.workspace.numel(), _stream_handle(setup)))
        self._tables = collections.OrderedDict()
        self._default = Store(self) if default_store else None

    @property
    def store(self) -> Store:
        """The plan's default store (allocated on first use when the plan was
        made without one)."""
        if self._default is None:
            self._default = Store(self)
        return self._default

    # default store's buffers, for callers that use one store per plan
    @property
    def bg(self):
        return self.store.bg

    @property
    def fg(self):
        return self.store.fg

    @property
    def flags(self):
        return self.store.flags

    @property
    def counts(self):
        return self.store.counts

    def new_store(self, noise=None) -> Store:
        return Store(self, noise)

    def noise_counters(self):
        """(n_frames, 2) int64 CUDA tensor of the frames' (seed, frame_index),
        for ``Store(noise=...)``; advance it with ``advance_noise``."""
        torch = _torch()
        rows = [[f.seed & (2**64 - 1), f.frame_index & (2**64 - 1)] for f in self.frames]
        arr = torch.tensor([[v - 2**64 if v >= 2**63 else v for v in r] for r in rows], dtype=torch.int64)
        return arr.to(self.device)

    def advance_noise(self, noise, step: int = 1, stream=None):
        """Add `step` to every frame_index of a noise-counter tensor, on the GPU."""
        if noise.dtype != _torch().int64 or noise.dim() != 2 or noise.shape[1] != 2 or not noise.is_contiguous():
            raise ValueError("noise must be a contiguous (n, 2) int64 tensor")
        _lib.check(self.lib.dp_pix_noise_advance(ctypes.c_void_p(noise.data_ptr()), noise.shape[0],
                                                 int(step) & (2**64 - 1), _stream_handle(stream)))

    def _store(self, store, stream=None):
        """The store of a call (default: the plan's), with the call's stream
        recorded against its buffers and the plan's workspace."""
        st = self.store if store is None else store
        st.used_on(stream)
        _use_on((self.workspace,), self._streams, stream)
        return st

    # -- plumbing ---------------------------------------------------------
    def set_launch(self, threads: int = 0, persistent: int = 0):
        """threads per workgroup (0: default); persistent: 0 one workgroup per
        tile, 1 a resident grid pulling tiles from a ticket, k >= 2 k per CU."""
        _lib.check(self.lib.dp_pix_plan_set_launch(self.handle, int(threads), int(persistent)))
        self.threads, self.persistent = threads, int(persistent)

    def pointer_table(self, tensors: Optional[Sequence], stream=None):
        """Device array of device pointers (None entries -> NULL).  The last
        MAX_TABLES tables are kept for reuse; a table used on a stream other
        than the current one is recorded on it, so evicting it cannot hand
        its memory to another allocation while a kernel may still read it."""
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
            while len(self._tables) > self.MAX_TABLES:
                self._tables.popitem(last=False)
        else:
            self._tables.move_to_end(key)
        if stream is not None and stream != torch.cuda.current_stream(self.device):
            tab.record_stream(stream)
        return tab

    def _check_images(self, tensors, what):
        torch = _torch()
        if len(tensors) != len(self.frames):
            raise ValueError("%s: need one tensor per frame (%d), got %d" % (what, len(self.frames), len(tensors)))
        for fp, t in zip(self.frames, tensors):
            if not _on_device(t, self.device):
                raise ValueError("%s must be CUDA tensors on %s" % (what, self.device))
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

    def _ptr(self, tab):
        return None if tab is None else ctypes.c_void_p(tab.data_ptr())

    # -- the method ----------------------------------------------------------
    def plan(self, masks=None, stream=None, store: Optional[Store] = None):
        """Classify cells from the masks (Algorithm 3 steps 3-6) and lay out the store."""
        check_masks(self.frames, masks, self.device)
        st = self._store(store, stream)
        tab = self.pointer_table(masks, stream)
        _lib.check(self.lib.dp_pix_plan(self.handle, self._ptr(tab), ctypes.byref(st.c), _stream_handle(stream)))

    def plan_labels(self, images, threshold: int, stream=None, store: Optional[Store] = None):
        """Classify cells from the frames' Sobel labels in the same pass (no
        mask written): the flags ``edge_masks`` followed by ``plan`` would give."""
        self._check_images(images, "images")
        st = self._store(store, stream)
        it = self.pointer_table(images, stream)
        _lib.check(self.lib.dp_pix_plan_labels(self.handle, self._ptr(it), int(threshold), ctypes.byref(st.c),
                                               _stream_handle(stream)))

    def index_store(self, store: Optional[Store] = None, stream=None):
        """Rebuild a store's counts and state from its flags (a store loaded
        with ``Store.load_host``)."""
        st = self._store(store, stream)
        _lib.check(self.lib.dp_pix_store_index(self.handle, ctypes.byref(st.c), _stream_handle(stream)))

    def edge_masks(self, images, threshold: int, out=None, stream=None):
        """Sobel complexity labels of uint8 frames (one (H, W) uint8 mask per
        frame, 1 where |Gx| + |Gy| of the channel sum >= threshold * C), ready
        for ``plan``."""
        torch = _torch()
        self._check_images(images, "images")
        if out is None:
            out = [torch.empty((fp.height, fp.width), dtype=torch.uint8, device=self.device) for fp in self.frames]
        else:
            check_masks(self.frames, out, self.device)
            if any(o is None for o in out):
                raise ValueError("edge_masks needs an output tensor per frame")
        _use_on((self.workspace,), self._streams, stream)
        it = self.pointer_table(images, stream)
        mt = self.pointer_table(out, stream)
        _lib.check(self.lib.dp_pix_edge_mask(self.handle, self._ptr(it), int(threshold), self._ptr(mt),
                                             _stream_handle(stream)))
        return out

    def metrics(self, images, recons, stream=None):
        """Per-frame (MSE, SSIM) between uint8 frames and their reconstructions,
        computed on the GPU; returns a (n_frames, 2) float64 tensor on the device."""
        torch = _torch()
        self._check_images(images, "images")
        self._check_images(recons, "recons")
        scratch = torch.empty(max(self.sizes.metrics_scratch_bytes, 256), dtype=torch.uint8, device=self.device)
        out = torch.empty((len(self.frames), 2), dtype=torch.float64, device=self.device)
        _use_on((self.workspace,), self._streams, stream)
        it = self.pointer_table(images, stream)
        rt = self.pointer_table(recons, stream)
        _lib.check(self.lib.dp_pix_metrics(self.handle, self._ptr(it), self._ptr(rt),
                                           ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def forward(self, images, out=None, clip=None, stream=None, store: Optional[Store] = None):
        """Noisy statistics into the store; with ``out`` also the reconstruction.
        ``clip``: optional (clip_bg, clip_fg) uint8 tensors of the store's capacities."""
        self._check_images(images, "images")
        if out is not None:
            self._check_images(out, "out")
            check_no_alias(images, out)
        st = self._store(store, stream)
        it = self.pointer_table(images, stream)
        ot = self.pointer_table(out, stream)
        cb = ctypes.c_void_p(clip[0].data_ptr()) if clip is not None else None
        cf = ctypes.c_void_p(clip[1].data_ptr()) if clip is not None else None
        _lib.check(self.lib.dp_pix_forward(self.handle, self._ptr(it), ctypes.byref(st.c), cb, cf, self._ptr(ot),
                                           _stream_handle(stream)))

    def reconstruct(self, out, stream=None, store: Optional[Store] = None):
        """Rebuild frames from a store alone (Sec. VI-F)."""
        self._check_images(out, "out")
        st = self._store(store, stream)
        ot = self.pointer_table(out, stream)
        _lib.check(self.lib.dp_pix_reconstruct(self.handle, ctypes.byref(st.c), self._ptr(ot),
                                               _stream_handle(stream)))

    def backward(self, grad_out, grad_in, clip, scratch=None, stream=None, store: Optional[Store] = None):
        """Adjoint for F32_CHW frames (noise and mask fixed), through the cell
        classes and offsets of the store the matching forward wrote."""
        torch = _torch()
        self._check_images(grad_out, "grad_out")
        self._check_images(grad_in, "grad_in")
        st = self._store(store, stream)
        if scratch is None:
            scratch = torch.empty(max(self.sizes.grad_scratch_bytes, 256), dtype=torch.uint8, device=self.device)
        gt = self.pointer_table(grad_out, stream)
        it = self.pointer_table(grad_in, stream)
        _lib.check(self.lib.dp_pix_backward(self.handle, ctypes.byref(st.c), self._ptr(gt),
                                            ctypes.c_void_p(clip[0].data_ptr()), ctypes.c_void_p(clip[1].data_ptr()),
                                            self._ptr(it), ctypes.c_void_p(scratch.data_ptr()),
                                            scratch.numel(), _stream_handle(stream)))

    def backward_static(self, grad_out, grad_in, clip, stream=None, store: Optional[Store] = None):
        """``backward`` through dp_pix_backward_static: the library's fixed
        device scratch instead of a scratch tensor (nothing is allocated by
        the call; calls overlapping on one GPU race)."""
        self._check_images(grad_out, "grad_out")
        self._check_images(grad_in, "grad_in")
        st = self._store(store, stream)
        gt = self.pointer_table(grad_out, stream)
        it = self.pointer_table(grad_in, stream)
        _lib.check(self.lib.dp_pix_backward_static(self.handle, ctypes.byref(st.c), self._ptr(gt),
                                                   ctypes.c_void_p(clip[0].data_ptr()),
                                                   ctypes.c_void_p(clip[1].data_ptr()), self._ptr(it),
                                                   _stream_handle(stream)))

    def debug_sums(self, images, stream=None, store: Optional[Store] = None):
        """Forward that also returns dense exact sums (coarse, fine) as uint32 tensors."""
        torch = _torch()
        self._check_images(images, "images")
        st = self._store(store, stream)
        ncell = sum(fi.grid_rows * fi.grid_cols * fp.channels for fi, fp in zip(self.info, self.frames))
        nfine = sum(fi.grid_rows * fi.grid_cols * fi.n * fi.n * fp.channels for fi, fp in zip(self.info, self.frames))
        coarse = torch.zeros(max(ncell, 1), dtype=torch.int32, device=self.device)
        fine = torch.zeros(max(nfine, 1), dtype=torch.int32, device=self.device)
        it = self.pointer_table(images, stream)
        _lib.check(self.lib.dp_pix_debug_sums(self.handle, self._ptr(it), ctypes.byref(st.c),
                                              ctypes.c_void_p(coarse.data_ptr()), ctypes.c_void_p(fine.data_ptr()),
                                              _stream_handle(stream)))
        return coarse, fine

    def clip_buffers(self):
        torch = _torch()
        return (torch.empty(max(self.sizes.clip_bytes_bg, 1), dtype=torch.uint8, device=self.device),
                torch.empty(max(self.sizes.clip_bytes_fg, 1), dtype=torch.uint8, device=self.device))

    def bound_calls(self, masks, images, out=None, stream=None, clip=None, store: Optional[Store] = None):
        """Validate once and return zero-argument callables ``(plan, forward)``
        that issue dp_pix_plan / dp_pix_forward on ``stream`` with the
        arguments already marshalled (for back-to-back launches)."""
        check_masks(self.frames, masks, self.device)
        self._check_images(images, "images")
        if out is not None:
            self._check_images(out, "out")
            check_no_alias(images, out)
        st = self._store(store, stream)
        mt = self.pointer_table(masks, stream)
        it = self.pointer_table(images, stream)
        ot = self.pointer_table(out, stream)
        lib, h, sc, s = self.lib, self.handle, ctypes.byref(st.c), _stream_handle(stream)
        mp, ip, op = self._ptr(mt), self._ptr(it), self._ptr(ot)
        cb = None if clip is None else ctypes.c_void_p(clip[0].data_ptr())
        cf = None if clip is None else ctypes.c_void_p(clip[1].data_ptr())
        keep = (mt, it, ot, clip, st)

        def plan_call():
            _lib.check(lib.dp_pix_plan(h, mp, sc, s))

        def forward_call():
            _lib.check(lib.dp_pix_forward(h, ip, sc, cb, cf, op, s))

        plan_call.keep = forward_call.keep = keep
        return plan_call, forward_call

    def bound_reconstruct(self, out, stream=None, store: Optional[Store] = None):
        """Validate once and return a zero-argument callable issuing
        dp_pix_reconstruct with the arguments already marshalled."""
        self._check_images(out, "out")
        st = self._store(store, stream)
        ot = self.pointer_table(out, stream)
        lib, h, sc, s, op = self.lib, self.handle, ctypes.byref(st.c), _stream_handle(stream), self._ptr(ot)

        def reconstruct_call():
            _lib.check(lib.dp_pix_reconstruct(h, sc, op, s))

        reconstruct_call.keep = (ot, st)
        return reconstruct_call

    def bound_backward(self, grad_out, grad_in, clip, scratch, stream=None, store: Optional[Store] = None):
        """Validate once and return a zero-argument callable issuing
        dp_pix_backward with the arguments already marshalled."""
        self._check_images(grad_out, "grad_out")
        self._check_images(grad_in, "grad_in")
        st = self._store(store, stream)
        gt = self.pointer_table(grad_out, stream)
        it = self.pointer_table(grad_in, stream)
        lib, h, sc, s = self.lib, self.handle, ctypes.byref(st.c), _stream_handle(stream)
        args = (self._ptr(gt), ctypes.c_void_p(clip[0].data_ptr()),
                ctypes.c_void_p(clip[1].data_ptr()), self._ptr(it),
                ctypes.c_void_p(scratch.data_ptr()), scratch.numel())

        def backward_call():
            _lib.check(lib.dp_pix_backward(h, sc, args[0], args[1], args[2], args[3], args[4], args[5], s))

        backward_call.keep = (gt, it, clip, scratch, st)
        return backward_call

    def graph(self, masks, images, out=None, stream=None, store: Optional[Store] = None) -> "Graph":
        """Capture plan + forward (+ fused reconstruction) into a HIP graph."""
        return Graph(self, masks, images, out, stream, store)

    # -- host views --------------------------------------------------------
    def store_host(self, store: Optional[Store] = None):
        """Copy a store (default: the plan's) to the host and split it per frame (synchronises)."""
        return (self.store if store is None else store).host()

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

    def __init__(self, plan: Plan, masks, images, out=None, stream=None, store: Optional[Store] = None):
        self.plan = plan
        check_masks(plan.frames, masks, plan.device)
        plan._check_images(images, "images")
        if out is not None:
            plan._check_images(out, "out")
            check_no_alias(images, out)
        self.store = plan._store(store, stream)
        # tables held by the graph for its lifetime (its kernels read them at replay)
        self.mt = plan.pointer_table(masks, stream)
        self.it = plan.pointer_table(images, stream)
        self.ot = plan.pointer_table(out, stream)
        h = ctypes.c_void_p()
        _lib.check(plan.lib.dp_pix_graph_create(
            plan.handle, plan._ptr(self.mt), plan._ptr(self.it), ctypes.byref(self.store.c), plan._ptr(self.ot),
            _stream_handle(stream), ctypes.byref(h)))
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
    if blocks.device.type != "cuda" or blocks.dim() != 2 or blocks.shape[1] != 6:
        raise ValueError("blocks must be an (n, 6) CUDA tensor")
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
