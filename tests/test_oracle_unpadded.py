"""Pins of the oracle's unpadded border mode (Algorithm 1: a border cell keeps
only its h x w real pixels and its mean divides by h*w; no mirror padding).

Each expected value is computed here from the image itself with numpy slicing
(no padding, no oracle arithmetic), or from a pinned primitive (Philox words,
the Laplace inverse CDF, sigma), or by finite differences of the forward.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import Params, INF

NONE = oracle.PAD_NONE


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _expected_noise_off(img, mk, b, sb, tau):
    """Algorithm 1 cell means (and subcell means of complex cells) by slicing
    the unpadded image; flags from the real mask pixels of each cell."""
    M, N, C = img.shape
    GR, GC, n = -(-M // b), -(-N // b), b // sb
    flags = np.zeros((GR, GC), np.uint8)
    bg, fg = [], []
    recon = np.zeros((M, N, C), np.float32)
    for r in range(GR):
        for c in range(GC):
            y0, x0 = r * b, c * b
            cell_m = mk[y0:y0 + b, x0:x0 + b]
            t = tau if tau > 0 else (cell_m.size + 1) // 2
            flags[r, c] = int((cell_m != 0).sum() >= t)
            if not flags[r, c]:
                blk = img[y0:y0 + b, x0:x0 + b].astype(np.float64)
                v = blk.reshape(-1, C).mean(axis=0).astype(np.float32)
                bg.append(v)
                recon[y0:y0 + b, x0:x0 + b] = v
            else:
                sub = np.zeros((n * n, C), np.float32)
                for i in range(n):
                    for j in range(n):
                        ys, xs = y0 + i * sb, x0 + j * sb
                        blk = img[ys:ys + sb, xs:xs + sb].astype(np.float64)
                        if blk.size:
                            sub[i * n + j] = blk.reshape(-1, C).mean(axis=0)
                            recon[ys:ys + sb, xs:xs + sb] = sub[i * n + j]
                fg.append(sub)
    bg = np.array(bg, np.float32).reshape(-1, C)
    fg = np.array(fg, np.float32).reshape(-1, n * n, C)
    return flags, bg, fg, recon


@pytest.mark.parametrize("M,N,C,b,sb,tau", [
    (45, 70, 3, 16, 4, 1),    # partial cells on both borders, some subcells empty
    (13, 17, 1, 8, 2, 1),
    (5, 3, 2, 8, 4, 1),       # frame smaller than one cell
    (50, 61, 3, 12, 3, 0),    # majority rule on partial cells
    (33, 65, 3, 32, 8, 0),
    (1, 1, 1, 4, 1, 1),
])
def test_noise_off_is_cropped_block_mean(M, N, C, b, sb, tau):
    r = rng(M * 131 + N)
    img = r.integers(0, 256, (M, N, C)).astype(np.uint8)
    mk = (r.random((M, N)) < 0.25).astype(np.uint8)
    mk[: M // 3, : N // 3] = 1
    p = Params(M, N, C, b=b, sb=sb, m=4, eps_simple=INF, eps_complex=INF, tau=tau, pad_mode=NONE)
    o = oracle.forward(img, mk, p)
    flags, bg, fg, recon = _expected_noise_off(img, mk, b, sb, tau)
    assert np.array_equal(o["flags"], flags)
    assert np.array_equal(o["bg"], bg)
    assert np.array_equal(o["fg"], fg)
    assert np.array_equal(o["recon_f32"], recon)
    assert np.array_equal(o["recon_u8"], np.rint(recon).astype(np.uint8))
    # subcells with no real pixel release nothing and never pass a gradient
    n = b // sb
    GR, GC = -(-M // b), -(-N // b)
    k = 0
    for rr, cc in itertools.product(range(GR), range(GC)):
        if not flags[rr, cc]:
            continue
        for i, j in itertools.product(range(n), range(n)):
            if rr * b + i * sb >= M or cc * b + j * sb >= N:
                assert (o["fg"][k, i * n + j] == 0).all()
                assert (o["pass_fg"][k, i * n + j] == 0).all()
        k += 1


@pytest.mark.parametrize("M,N,C,b,sb", [(48, 80, 3, 16, 4), (64, 64, 1, 8, 8), (24, 36, 2, 12, 3)])
def test_equals_padded_mode_when_b_divides(M, N, C, b, sb):
    """Without border cells there is nothing to pad: both modes give the same
    store and output, noise included."""
    r = rng(M + N + C)
    img = r.integers(0, 256, (M, N, C)).astype(np.uint8)
    mk = (r.random((M, N)) < 0.1).astype(np.uint8)
    base = dict(b=b, sb=sb, m=16, eps_simple=0.7, eps_complex=0.4, tau=1, seed=21, frame_index=5)
    a = oracle.forward(img, mk, Params(M, N, C, pad_mode=oracle.PAD_SYMMETRIC, **base))
    z = oracle.forward(img, mk, Params(M, N, C, pad_mode=NONE, **base))
    for key in ("flags", "bg", "fg", "recon_u8", "recon_f32", "pass_bg", "pass_fg"):
        assert np.array_equal(a[key], z[key]), key


def test_border_noise_uses_papers_sigma():
    """Algorithm 1 draws every cell's noise at the one sigma = 255 m / (b^2 eps),
    border cells included: on a constant frame the released value minus the
    constant is exactly that Laplace draw of the cell's Philox block."""
    M, N, b, m, eps = 37, 23, 8, 2, 50.0
    img = np.full((M, N, 1), 128, np.uint8)
    p = Params(M, N, 1, b=b, sb=b, m=m, eps_simple=eps, eps_complex=eps, pad_mode=NONE, seed=3, frame_index=9)
    o = oracle.forward(img, None, p)
    GC = -(-N // b)
    sigma = 255.0 * m / (b * b) / eps
    assert oracle.sigma(b, m, eps) == sigma
    for k, (r, c) in enumerate(itertools.product(range(-(-M // b)), range(GC))):
        w = oracle.noise_words(3, 9, r * GC + c, 0, 0)
        eta = oracle.laplace(oracle.uniform(w[0], w[1]), sigma)
        assert o["bg"][k, 0] == np.float32(128.0 + eta)


@pytest.mark.parametrize("M,N,C,b,sb", [(11, 13, 2, 4, 2), (7, 10, 1, 8, 2), (9, 6, 1, 4, 4)])
def test_backward_matches_central_fd(M, N, C, b, sb):
    r = rng(M * N * C + 7)
    img = r.uniform(0, 255, (M, N, C))
    mk = (r.random((M, N)) < 0.3).astype(np.uint8)
    w = r.standard_normal((M, N, C))
    p = Params(M, N, C, b=b, sb=sb, m=2, eps_simple=2.0, eps_complex=1.0, tau=1, pad_mode=NONE, seed=4)
    g = oracle.backward(img, mk, w, p)
    h = 1e-3
    f = lambda x: float((oracle.forward(x, mk, p)["recon_f64"] * w).sum())
    for idx in itertools.product(range(M), range(N), range(C)):
        e = np.zeros_like(img)
        e[idx] = h
        fd = (f(img + e) - f(img - e)) / (2 * h)
        assert fd == pytest.approx(g[idx], abs=1e-7), idx


def test_store_reconstructs_forward_output():
    r = rng(77)
    M, N, C, b, sb = 29, 45, 3, 16, 4
    img = r.integers(0, 256, (M, N, C)).astype(np.uint8)
    mk = (r.random((M, N)) < 0.2).astype(np.uint8)
    p = Params(M, N, C, b=b, sb=sb, m=8, eps_simple=1.0, eps_complex=0.5, tau=1, pad_mode=NONE, seed=2)
    o = oracle.forward(img, mk, p)
    rf, ru = oracle.reconstruct(o["flags"], o["bg"], o["fg"], p)
    assert np.array_equal(ru, o["recon_u8"])
    assert np.array_equal(rf, o["recon_f32"])
