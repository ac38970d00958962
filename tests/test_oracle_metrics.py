"""Pins of the oracle's utility metrics (MSE, SSIM) against independent
formulations: numpy for MSE; a vectorised SSIM built from
scipy.ndimage.uniform_filter (the same definition, different code path);
closed forms for identical, constant and shifted images."""
import numpy as np
import pytest

import oracle

C1 = (0.01 * 255) ** 2
C2 = (0.03 * 255) ** 2


def ssim_ref(x, y):
    ndi = pytest.importorskip("scipy.ndimage")
    vals = []
    for ch in range(x.shape[2]):
        a = x[:, :, ch].astype(np.float64)
        b = y[:, :, ch].astype(np.float64)
        f = lambda z: ndi.uniform_filter(z, size=7, mode="reflect")
        ux, uy = f(a), f(b)
        k = 49.0 / 48.0
        vx = k * (f(a * a) - ux * ux)
        vy = k * (f(b * b) - uy * uy)
        vxy = k * (f(a * b) - ux * uy)
        S = ((2 * ux * uy + C1) * (2 * vxy + C2)) / ((ux ** 2 + uy ** 2 + C1) * (vx + vy + C2))
        vals.append(S[3:-3, 3:-3].mean())
    return float(np.mean(vals))


@pytest.mark.parametrize("H,W,C", [(7, 7, 1), (20, 31, 3), (64, 48, 1), (33, 90, 2)])
def test_metrics_match_independent_formulation(H, W, C):
    r = np.random.Generator(np.random.PCG64(H * W * C))
    x = r.integers(0, 256, (H, W, C)).astype(np.uint8)
    y = np.clip(x.astype(int) + r.integers(-40, 41, (H, W, C)), 0, 255).astype(np.uint8)
    mse, ssim = oracle.metrics(x, y)
    assert mse == pytest.approx(((x.astype(float) - y.astype(float)) ** 2).mean(), rel=1e-13)
    assert ssim == pytest.approx(ssim_ref(x, y), abs=1e-10)
    assert oracle.metrics(y, x)[1] == pytest.approx(ssim, abs=1e-12)


def test_metrics_closed_forms():
    r = np.random.Generator(np.random.PCG64(3))
    x = r.integers(0, 256, (30, 40, 3)).astype(np.uint8)
    mse, ssim = oracle.metrics(x, x)
    assert mse == 0.0 and ssim == pytest.approx(1.0, abs=1e-12)
    for a, b in [(10, 200), (128, 128), (0, 255)]:
        mse, ssim = oracle.metrics(np.full((12, 9), a, np.uint8), np.full((12, 9), b, np.uint8))
        assert mse == (a - b) ** 2
        assert ssim == pytest.approx((2 * a * b + C1) / (a * a + b * b + C1), rel=1e-12)
    with pytest.raises(ValueError):
        oracle.metrics(np.zeros((6, 30), np.uint8), np.zeros((6, 30), np.uint8))
