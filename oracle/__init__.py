"""CPU oracle for region-adaptive DP pixelization (arXiv 2511.04261).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product package never does.
The arithmetic lives in ``dppix_oracle.c`` (plain C, fp64, written step by step
from Algorithms 2 and 3, Eq. (1)-(4), (8)-(11) and (16)-(17) of the paper).
This module only marshals numpy arrays into it and out of it.

Parameter names follow the paper: ``b`` is the grid size of simple regions,
``sb`` the subgrid size of complex regions (b = n * sb, Eq. 16), ``m`` the
number of pixels neighbouring images may differ in, ``eps_simple`` and
``eps_complex`` the budgets (``math.inf`` switches the noise off).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dppix_oracle.c")
_LIB = os.path.join(_HERE, "libdppix_oracle.so")

PAD_SYMMETRIC = 0
PAD_REFLECT = 1
PAD_NONE = 2          # Algorithm 1: border cells keep only their real pixels


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math) into ``oracle/``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("b", ctypes.c_int32), ("sb", ctypes.c_int32), ("m", ctypes.c_int32),
                ("eps_simple", ctypes.c_double), ("eps_complex", ctypes.c_double),
                ("tau", ctypes.c_int32), ("pad_mode", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("frame_index", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        lib.orc_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        lib.orc_philox4x32_10.restype = None
        lib.orc_noise_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                        ctypes.c_int32, P(ctypes.c_uint32)]
        lib.orc_noise_words.restype = None
        lib.orc_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.orc_uniform.restype = ctypes.c_double
        lib.orc_laplace.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_laplace.restype = ctypes.c_double
        lib.orc_sigma.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double]
        lib.orc_sigma.restype = ctypes.c_double
        lib.orc_fold.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
        lib.orc_fold.restype = ctypes.c_int64
        lib.orc_check.argtypes = [P(_Params)]
        lib.orc_check.restype = ctypes.c_int32
        lib.orc_geometry.argtypes = [P(_Params), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
        lib.orc_geometry.restype = ctypes.c_int32
        lib.orc_forward.argtypes = [P(_Params), vp, vp, vp, vp, vp, P(ctypes.c_int64), vp, vp, vp, vp, vp, vp, vp]
        lib.orc_forward.restype = ctypes.c_int32
        lib.orc_reconstruct.argtypes = [P(_Params), vp, vp, vp, vp, vp]
        lib.orc_reconstruct.restype = ctypes.c_int32
        lib.orc_backward.argtypes = [P(_Params), vp, vp, vp, vp]
        lib.orc_backward.restype = ctypes.c_int32
        lib.orc_edge_mask.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32,
                                      ctypes.c_int32, vp]
        lib.orc_edge_mask.restype = ctypes.c_int32
        lib.orc_metrics.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, P(ctypes.c_double),
                                    P(ctypes.c_double)]
        lib.orc_metrics.restype = ctypes.c_int32
        _lib = lib
    return _lib


@dataclass
class Params:
    height: int
    width: int
    channels: int = 1
    b: int = 16
    sb: int = 16
    m: int = 16
    eps_simple: float = 0.5
    eps_complex: float = 0.5
    tau: int = 0
    pad_mode: int = PAD_SYMMETRIC
    seed: int = 0
    frame_index: int = 0

    def _c(self) -> _Params:
        return _Params(self.height, self.width, self.channels, self.b, self.sb, self.m,
                       float(self.eps_simple), float(self.eps_complex), self.tau, self.pad_mode,
                       self.seed & (2**64 - 1), self.frame_index & (2**64 - 1))

    def geometry(self):
        """(G_R, G_C, n); raises ValueError on invalid parameters."""
        a, b_, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        if _load().orc_geometry(ctypes.byref(self._c()), ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c)):
            raise ValueError("invalid oracle parameters: %r" % (self,))
        return a.value, b_.value, c.value


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def philox4x32_10(ctr, key):
    ctr = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    key = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (ctypes.c_uint32 * 4)()
    _load().orc_philox4x32_10(ctr, key, out)
    return tuple(int(v) for v in out)


def noise_words(seed, frame_index, cell_id, ch, level):
    out = (ctypes.c_uint32 * 4)()
    _load().orc_noise_words(seed & (2**64 - 1), frame_index & (2**64 - 1), cell_id, ch, level, out)
    return tuple(int(v) for v in out)


def uniform(w0, w1) -> float:
    return _load().orc_uniform(w0 & 0xFFFFFFFF, w1 & 0xFFFFFFFF)


def laplace(u, sigma) -> float:
    return _load().orc_laplace(u, sigma)


def sigma(b, m, eps) -> float:
    return _load().orc_sigma(b, m, float(eps))


def fold(x, L, mode=PAD_SYMMETRIC) -> int:
    return _load().orc_fold(x, L, mode)


def _as_hwc(img, p: Params):
    a = np.asarray(img)
    if a.ndim == 2:
        a = a[:, :, None]
    if a.shape != (p.height, p.width, p.channels):
        raise ValueError("image shape %r does not match params %r" % (a.shape, (p.height, p.width, p.channels)))
    return np.ascontiguousarray(a, dtype=np.float64)


def _as_mask(mask, p: Params):
    if mask is None:
        return None
    mk = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    if mk.shape != (p.height, p.width):
        raise ValueError("mask shape %r does not match (%d, %d)" % (mk.shape, p.height, p.width))
    return mk


def forward(img, mask, p: Params, sums: bool = False):
    """Run the oracle forward pass on one HWC (or HW) image.

    Returns a dict with ``flags`` (G_R, G_C) uint8, ``bg`` (n_bg, C) float32,
    ``fg`` (n_fg, n*n, C) float32, ``counts`` (n_bg, n_fg), ``recon_f32`` and
    ``recon_u8`` (M, N, C), ``recon_f64`` (before fp32 rounding), ``pass_bg``/``pass_fg`` and, with ``sums``, the
    padded ``coarse_sum`` (G_R, G_C, C) and ``fine_sum`` (G_R*n, G_C*n, C).
    """
    GR, GC, n = p.geometry()
    C = p.channels
    x = _as_hwc(img, p)
    mk = _as_mask(mask, p)
    cells = GR * GC
    flags = np.zeros(cells, np.uint8)
    bg = np.zeros(cells * C, np.float32)
    fg = np.zeros(cells * n * n * C, np.float32)
    pbg = np.zeros(cells * C, np.uint8)
    pfg = np.zeros(cells * n * n * C, np.uint8)
    counts = (ctypes.c_int64 * 2)()
    rf = np.zeros((p.height, p.width, C), np.float32)
    ru = np.zeros((p.height, p.width, C), np.uint8)
    rd = np.zeros((p.height, p.width, C), np.float64)
    cs = np.zeros((GR, GC, C), np.float64) if sums else None
    fs = np.zeros((GR * n, GC * n, C), np.float64) if sums else None
    rc = _load().orc_forward(ctypes.byref(p._c()), _ptr(x), _ptr(mk), _ptr(flags), _ptr(bg), _ptr(fg), counts,
                             _ptr(rf), _ptr(ru), _ptr(rd), _ptr(cs), _ptr(fs), _ptr(pbg), _ptr(pfg))
    if rc:
        raise RuntimeError("orc_forward failed (%d)" % rc)
    nb, nf = int(counts[0]), int(counts[1])
    out = dict(flags=flags.reshape(GR, GC), bg=bg[: nb * C].reshape(nb, C),
               fg=fg[: nf * n * n * C].reshape(nf, n * n, C), counts=(nb, nf),
               recon_f32=rf, recon_u8=ru, recon_f64=rd, pass_bg=pbg[: nb * C].reshape(nb, C),
               pass_fg=pfg[: nf * n * n * C].reshape(nf, n * n, C), geometry=(GR, GC, n))
    if sums:
        out["coarse_sum"] = cs
        out["fine_sum"] = fs
    return out


def reconstruct(flags, bg, fg, p: Params):
    """Rebuild (recon_f32, recon_u8) from the compact store alone."""
    GR, GC, n = p.geometry()
    fl = np.ascontiguousarray(np.asarray(flags, np.uint8).reshape(-1))
    if fl.size != GR * GC:
        raise ValueError("flags size mismatch")
    b_ = np.ascontiguousarray(np.asarray(bg, np.float32).reshape(-1))
    f_ = np.ascontiguousarray(np.asarray(fg, np.float32).reshape(-1))
    if b_.size == 0:
        b_ = np.zeros(1, np.float32)
    if f_.size == 0:
        f_ = np.zeros(1, np.float32)
    rf = np.zeros((p.height, p.width, p.channels), np.float32)
    ru = np.zeros((p.height, p.width, p.channels), np.uint8)
    if _load().orc_reconstruct(ctypes.byref(p._c()), _ptr(fl), _ptr(b_), _ptr(f_), _ptr(rf), _ptr(ru)):
        raise RuntimeError("orc_reconstruct failed")
    return rf, ru


def edge_mask(img, threshold: int, pad_mode: int = PAD_SYMMETRIC):
    """uint8 (H, W) Sobel edge mask of an HWC (or HW) image: 1 where
    |Gx| + |Gy| of the channel sum reaches threshold * C."""
    a = np.asarray(img)
    if a.ndim == 2:
        a = a[:, :, None]
    H, W, C = a.shape
    x = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros((H, W), np.uint8)
    if _load().orc_edge_mask(H, W, C, _ptr(x), int(threshold), pad_mode, _ptr(out)):
        raise ValueError("bad edge-mask arguments")
    return out


def metrics(x, y):
    """(MSE, SSIM) between two HWC (or HW) images of the same shape."""
    a = np.asarray(x)
    b = np.asarray(y)
    if a.ndim == 2:
        a, b = a[:, :, None], b[:, :, None]
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    H, W, C = a.shape
    xa = np.ascontiguousarray(a, dtype=np.float64)
    ya = np.ascontiguousarray(b, dtype=np.float64)
    mse, ssim = ctypes.c_double(), ctypes.c_double()
    if _load().orc_metrics(H, W, C, _ptr(xa), _ptr(ya), ctypes.byref(mse), ctypes.byref(ssim)):
        raise ValueError("metrics need frames of at least 7 x 7")
    return mse.value, ssim.value


def backward(img, mask, grad_out, p: Params):
    """fp64 adjoint (HWC): gradient of sum(grad_out * forward(img)) w.r.t. img."""
    x = _as_hwc(img, p)
    mk = _as_mask(mask, p)
    g = _as_hwc(grad_out, p)
    gi = np.zeros_like(x)
    if _load().orc_backward(ctypes.byref(p._c()), _ptr(x), _ptr(mk), _ptr(g), _ptr(gi)):
        raise RuntimeError("orc_backward failed")
    return gi


INF = math.inf
