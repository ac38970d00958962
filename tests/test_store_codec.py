"""Store codec on the CPU: round trips, the uint8 store rebuilds the uint8
reconstruction exactly (Table IV: the stored metadata suffices to rebuild the
frame), headers survive, corrupt input is refused."""
import zlib

import numpy as np
import pytest

import oracle
from paper_2511_04261_amd import store_codec as sc
from paper_2511_04261_amd import synth


def frame(seed=0, H=70, W=101, b=16, sb=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    img = synth.gradient_image(rng, H, W, 3)
    mk = synth.rect_mask(rng, H, W, n_rects=3, rect_frac=0.05, cover=(0.05, 0.4))
    p = oracle.Params(H, W, 3, b=b, sb=sb, m=16, eps_simple=1.0, eps_complex=0.3, tau=1, seed=3, frame_index=7)
    return img, mk, p, oracle.forward(img, mk, p)


def kw(p):
    return dict(height=p.height, width=p.width, channels=p.channels, b=p.b, sb=p.sb, m=p.m, eps_bg=p.eps_simple,
                eps_fg=p.eps_complex, frame_index=p.frame_index)


@pytest.mark.parametrize("b,sb", [(16, 4), (8, 8), (32, 8), (4, 1)])
def test_round_trip_f32_exact_and_u8_rebuilds_u8(b, sb):
    img, mk, p, o = frame(b, b=b, sb=sb)
    hdr, st = sc.decode(sc.encode(o, quant=sc.Q_F32, **kw(p)))
    assert np.array_equal(st["flags"], o["flags"]) and np.array_equal(st["bg"], o["bg"])
    assert np.array_equal(st["fg"], o["fg"]) and st["counts"] == o["counts"]
    assert hdr["b"] == b and hdr["sb"] == sb and hdr["frame_index"] == 7
    led = hdr["ledger"]
    assert led["eps_fg"] == 0.3 and led["eps_bg"] == 1.0 and led["m"] == 16
    assert led["eps_frame"] == 1.0 and led["eps_pixel"] == 3.0      # Thm. 1: max over regions; x C whole pixels
    assert "seed" not in hdr and b"seed" not in sc.encode(o, **kw(p))
    _, st8 = sc.decode(sc.encode(o, quant=sc.Q_U8, **kw(p)))
    _, ru = oracle.reconstruct(st8["flags"], st8["bg"], st8["fg"], p)
    assert np.array_equal(ru, o["recon_u8"])


def test_store_is_smaller_than_the_frame():
    img, mk, p, o = frame(1, H=270, W=480, b=32, sb=8)
    blob = sc.encode(o, quant=sc.Q_U8, **kw(p))
    assert len(blob) < img.size / 20
    assert len(blob) < sc.png_size(o["recon_u8"])


def test_corrupt_and_inconsistent_input_refused():
    img, mk, p, o = frame(2)
    blob = sc.encode(o, **kw(p))
    with pytest.raises(ValueError):
        sc.decode(b"XXXX" + blob[4:])
    with pytest.raises(ValueError):
        sc.decode(blob[:10])
    with pytest.raises(zlib.error):
        sc.decode(blob[: sc._HDR.size] + b"not deflate")
    bad = dict(o)
    bad["flags"] = np.zeros_like(o["flags"])
    with pytest.raises(ValueError):
        sc.encode(bad, **kw(p))


def test_ledger_and_no_key_in_the_bytes():
    """The header carries the ledger (budgets, m, max over the regions by
    parallel composition, C times that for whole-pixel neighbours) and the
    noise counter, never the generator's key: the encoded bytes are the same
    for two seeds."""
    img, mk, p, o = frame(3)
    blob = sc.encode(o, **kw(p))
    hdr, _ = sc.decode(blob)
    assert hdr["ledger"] == sc.privacy_ledger(3, 16, 1.0, 0.3)
    import inspect
    assert "seed" not in inspect.signature(sc.encode).parameters
    led = sc.privacy_ledger(1, 4, 0.5, float("inf"))
    assert led["eps_frame"] == float("inf") and led["eps_pixel"] == float("inf")
    assert sc.privacy_ledger(1, 4, 0.5, 0.25)["eps_pixel"] == 0.5
