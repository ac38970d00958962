"""GPU test of dp_pix_backward_static, the adjoint entry point that takes no
scratch argument and allocates nothing (its scratch is a fixed device array
inside the library).  Called through the C ABI, it must give exactly what
dp_pix_backward gives with a caller-provided scratch buffer, and both must
match the oracle's adjoint, on two calls in a row whose second plan is
smaller than the first (the fixed array keeps the first call's contents)."""
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import chw_to_hwc, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dp = pytest.importorskip("paper_2511_04261_amd")
from paper_2511_04261_amd import _lib, synth  # noqa: E402

GRAD_TOL = 1e-5   # relative to the largest gradient, as in the adjoint parity tests


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(dev, shapes, seed):
    """Forward + both backward entry points on fp32 CHW frames of `shapes`
    ((H, W, pad_mode) each); returns per-frame (static, scratch, oracle)
    gradients as HWC arrays."""
    r = np.random.Generator(np.random.PCG64(seed))
    frames = [dp.FrameParams(H, W, 3, dp.F32_CHW, b=16, sb=8, m=8, eps_bg=1.0, eps_fg=0.5, tau=1, pad_mode=pm,
                             seed=seed, frame_index=i) for i, (H, W, pm) in enumerate(shapes)]
    xs = [synth.uniform_f32(r, (3, H, W)) for (H, W, _) in shapes]
    ms = [synth.rect_mask(r, H, W, n_rects=2, rect_frac=0.1, cover=(0.05, 0.5)) for (H, W, _) in shapes]
    ws = [r.standard_normal((3, H, W)).astype(np.float32) for (H, W, _) in shapes]
    plan = dp.Plan(frames, device=dev)
    tx = [torch.from_numpy(x).to(dev) for x in xs]
    tm = [torch.from_numpy(m).to(dev) for m in ms]
    tw = [torch.from_numpy(w).to(dev) for w in ws]
    plan.plan(tm)
    clip = plan.clip_buffers()
    plan.forward(tx, out=[torch.empty_like(t) for t in tx], clip=clip)
    # NaN-filled outputs: every real pixel must be written by the adjoint
    g_static = [torch.full_like(t, float("nan")) for t in tx]
    g_scratch = [torch.full_like(t, float("nan")) for t in tx]
    plan.backward_static(tw, g_static, clip)
    plan.backward(tw, g_scratch, clip)
    torch.cuda.synchronize()
    out = []
    for i, fp in enumerate(frames):
        want = oracle.backward(chw_to_hwc(xs[i]).astype(np.float64), ms[i], chw_to_hwc(ws[i]).astype(np.float64),
                               oracle_params(fp))
        out.append((chw_to_hwc(g_static[i].cpu().numpy()), chw_to_hwc(g_scratch[i].cpu().numpy()), want))
    return plan, out


def test_backward_static_matches_backward_twice(dev):
    """Two calls in a row, the second on a smaller plan: each equals
    dp_pix_backward bit for bit and the oracle gradient within 1e-5."""
    cases = [
        ("three frames, mixed padding", [(64, 64, dp.PAD_SYMMETRIC), (61, 57, dp.PAD_REFLECT),
                                         (33, 70, dp.PAD_NONE)], 11),
        ("one smaller frame", [(29, 37, dp.PAD_SYMMETRIC)], 12),
    ]
    for tag, shapes, seed in cases:
        say("case: backward_static,", tag, shapes, "seed", seed)
        plan, res = _run(dev, shapes, seed)
        assert plan.sizes.grad_scratch_bytes <= 32 << 20
        for i, (got, ref, want) in enumerate(res):
            assert np.array_equal(got, ref), "%s frame %d: static scratch differs from dp_pix_backward" % (tag, i)
            d = np.abs(got.astype(np.float64) - want).max()
            assert d <= GRAD_TOL * max(1.0, np.abs(want).max()), "%s frame %d: %g from the oracle" % (tag, i, d)


def test_backward_static_rejects_plans_beyond_its_scratch(dev):
    """A plan needing more than the fixed 32 MiB is refused with ENOMEM
    before any launch; the grad_in buffer keeps its contents."""
    H = W = 2048
    say("case: backward_static over-size plan", H, W)
    fp = dp.FrameParams(H, W, 3, dp.F32_CHW, b=2, sb=1, m=1, eps_bg=1.0, eps_fg=1.0, tau=1, seed=1)
    plan = dp.Plan([fp], device=dev)
    assert plan.sizes.grad_scratch_bytes > 32 << 20
    x = torch.zeros((3, H, W), dtype=torch.float32, device=dev)
    plan.plan(None)
    clip = plan.clip_buffers()
    plan.forward([x], clip=clip)
    g = torch.full_like(x, 7.0)
    with pytest.raises(_lib.DppixError) as ei:
        plan.backward_static([x], [g], clip)
    assert ei.value.status == _lib.DPPIX_ENOMEM
    torch.cuda.synchronize()
    assert bool((g == 7.0).all())
