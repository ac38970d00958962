"""Differentiable DP pixelization (not in the paper): forward and a
hand-written adjoint behind ``torch.autograd.Function``.

With the noise frozen by its counter (seed, frame_index) and the mask held
constant, the layer is piecewise linear in its input: each output pixel is its
statistic clip(mean + noise) and the adjoint spreads the statistic's gradient
over the padded cell, divided by the cell area, where the clip did not bind.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import F32_CHW, FrameParams, Plan


class DPPixFn(torch.autograd.Function):
    """y = pixelize(x) for a batch x of shape (B, C, H, W), float32, on the GPU.

    Every call plans into a store of its own, which its backward reads: the
    adjoint goes through the cell classes and store offsets of the forward it
    belongs to, however many other forwards of the same plan (other masks)
    ran in between — gradient accumulation, two-branch losses, recomputation.
    """

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan, masks: Optional[Sequence[torch.Tensor]] = None):
        if x.dim() != 4 or x.dtype != torch.float32:
            raise ValueError("x must be float32 (B, C, H, W)")
        x = x.contiguous()
        frames = [x[i] for i in range(x.shape[0])]
        y = torch.empty_like(x)
        outs = [y[i] for i in range(x.shape[0])]
        clip = plan.clip_buffers()
        store = plan.new_store()
        plan.plan(masks, store=store)
        plan.forward(frames, out=outs, clip=clip, store=store)
        ctx.plan = plan
        ctx.store = store
        ctx.save_for_backward(clip[0], clip[1])
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        clip_bg, clip_fg = ctx.saved_tensors
        gy = gy.contiguous()
        gx = torch.empty_like(gy)
        ctx.plan.backward([gy[i] for i in range(gy.shape[0])], [gx[i] for i in range(gx.shape[0])],
                          (clip_bg, clip_fg), store=ctx.store)
        return gx, None, None


class DPPixLayer(torch.nn.Module):
    """Module wrapper: one plan per batch geometry, masks given per call.

    Image i of every call draws its noise with counter first_frame_index + i
    under `seed`: the noise is frozen, as training through the layer needs.
    Outputs meant as privacy releases must not reuse a counter for different
    images (equal noise gives away the exact difference of their true cell
    means): give each released batch its own first_frame_index or seed."""

    def __init__(self, b: int = 16, sb: Optional[int] = None, m: int = 8, eps_bg: float = 1.0,
                 eps_fg: Optional[float] = None, tau: int = 1, seed: int = 0, first_frame_index: int = 0):
        super().__init__()
        self.kw = dict(b=b, sb=sb, m=m, eps_bg=eps_bg, eps_fg=eps_fg, tau=tau, seed=seed)
        self.first_frame_index = first_frame_index
        self._plans = {}

    def plan_for(self, x: torch.Tensor) -> Plan:
        key = (tuple(x.shape), x.device)
        p = self._plans.get(key)
        if p is None:
            B, C, H, W = x.shape
            frames = [FrameParams(H, W, C, F32_CHW, frame_index=self.first_frame_index + i, **self.kw)
                      for i in range(B)]
            p = Plan(frames, device=x.device)
            self._plans[key] = p
        return p

    def forward(self, x: torch.Tensor, masks: Optional[Sequence[torch.Tensor]] = None) -> torch.Tensor:
        return DPPixFn.apply(x, self.plan_for(x), masks)
