"""GPU tests of the rows after the hot path: utility metrics (MSE, SSIM) of a
release against the oracle, and the storage study."""
import sys

import numpy as np
import pytest

import oracle
from tests.helpers import oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dp = pytest.importorskip("paper_2511_04261_amd")
from paper_2511_04261_amd import synth  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("threads", [0, 512])
def test_metrics_match_oracle(dev, threads):
    """MSE exact (integer squared errors), SSIM within 1e-9 of the oracle, on
    a mixed batch of frames and their DP reconstructions (every channel count,
    rows with and without 16-byte alignment, frames at and below the 7 x 7
    window, tiles taller than one chunk of window rows at b = 64)."""
    say("case: metrics, threads", threads)
    r = np.random.Generator(np.random.PCG64(31))
    shapes = [(64, 80, 3), (37, 300, 1), (270, 480, 3), (7, 7, 2), (5, 30, 3), (1080, 1920, 3), (45, 71, 4),
              (33, 50, 2), (200, 130, 3)]
    frames, imgs = [], []
    for i, (H, W, C) in enumerate(shapes):
        b = 64 if (H, W) == (200, 130) else 16
        frames.append(dp.FrameParams(H, W, C, dp.U8_HWC, b=b, sb=4, m=16, eps_bg=1.0, eps_fg=0.3, tau=1, seed=4,
                                     frame_index=i))
        imgs.append(synth.gradient_image(r, H, W, C))
    plan = dp.Plan(frames, device=dev, threads=threads)
    ti = [torch.from_numpy(x).to(dev) for x in imgs]
    outs = [torch.empty_like(t) for t in ti]
    plan.plan(None)
    plan.forward(ti, out=outs)
    got = plan.metrics(ti, outs).cpu().numpy()
    for i, (H, W, C) in enumerate(shapes):
        rec = outs[i].cpu().numpy()
        if H >= 7 and W >= 7:
            mse, ssim = oracle.metrics(imgs[i], rec)
            assert got[i, 0] == pytest.approx(mse, rel=1e-15, abs=0), i
            assert abs(got[i, 1] - ssim) <= 1e-9, (i, got[i, 1], ssim)
        else:
            assert got[i, 0] == pytest.approx(((imgs[i].astype(float) - rec.astype(float)) ** 2).mean(), rel=1e-15)
            assert got[i, 1] == 0.0
    same = plan.metrics(ti, ti).cpu().numpy()
    assert (same[:, 0] == 0).all() and np.allclose(same[[0, 1, 2, 3, 5, 6, 7, 8], 1], 1.0, atol=1e-12)


def test_storage_study_small(dev):
    """Encoded store vs PNG of the reconstruction over grid sizes and subgrid
    factors: the store shrinks with b, grows with n; every store the GPU
    wrote decodes to the oracle's store of the same frame (flags exact, fp32
    statistics within 1e-3, uint8 statistics within one level of the
    oracle's rounded ones) with the frame's privacy ledger in its header."""
    say("case: storage study")
    from paper_2511_04261_amd import store_codec as sc
    specs = synth.region_batch(2, height=270, width=480)
    rows = sc.storage_study(specs, grid_sizes=(4, 16, 64), factors=(1, 4), device=dev, keep_blobs=True)
    by = {(r["b"], r["n"]): r for r in rows}
    assert by[(64, 1)]["store_u8"] < by[(16, 1)]["store_u8"] < by[(4, 1)]["store_u8"]
    assert by[(16, 4)]["store_u8"] > by[(16, 1)]["store_u8"]
    assert all(r["store_u8"] < r["png"] for r in rows if r["b"] >= 16)
    imgs = [s.image_torch(dev).cpu().numpy() for s in specs]
    for r in rows:
        for k, (s, fp) in enumerate(zip(specs, r["frames_params"])):
            say("  decode b=%d n=%d frame %d" % (r["b"], r["n"], k))
            want = oracle.forward(imgs[k], s.mask, oracle_params(fp))
            for blob, tol, quant in ((r["blobs_f32"][k], 1e-3, "f32"), (r["blobs_u8"][k], 1.0, "u8")):
                hdr, st = sc.decode(blob)
                assert hdr["ledger"] == sc.privacy_ledger(3, fp.m, fp.eps_bg, fp.eps_fg)
                assert np.array_equal(st["flags"], want["flags"]) and st["counts"] == want["counts"]
                for key in ("bg", "fg"):
                    ref = want[key] if quant == "f32" else np.rint(want[key])
                    if ref.size:
                        assert np.abs(st[key] - ref).max() <= tol, (r["b"], r["n"], k, quant, key)
