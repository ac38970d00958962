"""The seeded input generators: host (numpy) and device (torch) renderers give
identical bytes, masks cover what they claim, values have the stated ranges."""
import numpy as np
import pytest

from paper_2511_04261_amd import synth

torch = pytest.importorskip("torch")


def test_host_and_torch_render_identical():
    rng = np.random.Generator(np.random.PCG64(5))
    for (H, W) in [(1, 1), (7, 300), (576, 768), (123, 45)]:
        ramps = [synth.draw_ramp(rng) for _ in range(3)]
        a = synth.render_image(ramps, H, W)
        b = synth.render_image_torch(ramps, H, W, "cpu").numpy()
        assert np.array_equal(a, b)
        rects = synth.draw_rects(rng, H, W, n_rects=4)
        assert np.array_equal(synth.paint_mask(rects, H, W), synth.paint_mask_torch(rects, H, W, "cpu").numpy())


def test_union_area_and_cover():
    rng = np.random.Generator(np.random.PCG64(6))
    for _ in range(20):
        H, W = int(rng.integers(50, 400)), int(rng.integers(50, 400))
        rects = synth.draw_rects(rng, H, W)
        assert synth.union_area(rects) == int(synth.paint_mask(rects, H, W).sum())
    for spec in synth.region_batch(4):
        frac = synth.union_area(spec.rects) / (spec.height * spec.width)
        assert 0.13 <= frac <= 0.17


def test_value_ranges():
    img = synth.single_gray(1000)
    assert img.shape == (256, 256, 1) and img.dtype == np.uint8
    # noise U{-20..20}: the residual around the row/column ramp spans that range
    rng = np.random.Generator(np.random.PCG64(1))
    r = synth.Ramp(0, 0, 0, 12345)   # flat ramp at 128: image = 128 + noise
    flat = synth.render_image([r], 300, 300)[:, :, 0].astype(int) - 128
    assert flat.min() == -20 and flat.max() == 20
    counts = np.bincount(flat.ravel() + 20, minlength=41)
    assert counts.min() > 0.8 * counts.mean()


def test_uneven_batch_recipe():
    fr = synth.uneven_batch(32)
    assert {(f.height, f.width) for f in fr} <= set(synth.MIXED_RESOLUTIONS)
    assert all(f.b in (16, 32) and f.sb in (4, 8) and 0.1 <= f.eps_complex <= 0.5 and 0.5 <= f.eps_simple <= 2.0
               for f in fr)
    assert [f.frame_index for f in fr] == list(range(32))
