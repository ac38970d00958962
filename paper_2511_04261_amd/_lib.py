"""ctypes binding of libdppix (include/dppix.h): structure layouts, prototypes
and status checking.  Argument marshalling only — every step of the method
runs in the HIP kernels behind the C ABI.  There is no fallback: if the
library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdppix.so")

DPPIX_OK, DPPIX_EINVAL, DPPIX_ENOMEM, DPPIX_EDEVICE, DPPIX_ENOTSUP = 0, 1, 2, 3, 4
U8_HWC, F32_CHW = 0, 1
PAD_SYMMETRIC, PAD_REFLECT, PAD_NONE = 0, 1, 2


class DppixError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__("libdppix status %d: %s" % (status, detail))
        self.status = status
        self.detail = detail


class FrameDesc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("pitch", ctypes.c_int64), ("pad_mode", ctypes.c_int32),
                ("b_bg", ctypes.c_int32), ("b_fg", ctypes.c_int32), ("m", ctypes.c_int32),
                ("eps_bg", ctypes.c_double), ("eps_fg", ctypes.c_double),
                ("fg_min_count", ctypes.c_int32), ("tile_cells", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("frame_index", ctypes.c_uint64)]


class Store(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_void_p), ("fg", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("state", ctypes.c_void_p), ("noise", ctypes.c_void_p)]


class Sizes(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("bg_capacity", ctypes.c_size_t),
                ("fg_capacity", ctypes.c_size_t), ("flag_bytes", ctypes.c_size_t),
                ("clip_bytes_bg", ctypes.c_size_t), ("clip_bytes_fg", ctypes.c_size_t),
                ("grad_scratch_bytes", ctypes.c_size_t), ("n_tiles", ctypes.c_int64),
                ("total_pixels", ctypes.c_int64), ("metrics_scratch_bytes", ctypes.c_size_t),
                ("store_state_bytes", ctypes.c_size_t), ("forward_launches", ctypes.c_int64)]


class FrameInfo(ctypes.Structure):
    _fields_ = [("grid_rows", ctypes.c_int32), ("grid_cols", ctypes.c_int32), ("n", ctypes.c_int32),
                ("pad_rows", ctypes.c_int32), ("pad_cols", ctypes.c_int32),
                ("tile_cells", ctypes.c_int32), ("tiles_per_band", ctypes.c_int32),
                ("fg_min_count", ctypes.c_int32), ("cell_offset", ctypes.c_int64),
                ("fine_offset", ctypes.c_int64), ("sigma_bg", ctypes.c_double), ("sigma_fg", ctypes.c_double)]


#: every symbol the header declares, with (restype, argtypes)
_vp = ctypes.c_void_p
_st = ctypes.c_int
_P = ctypes.POINTER
SYMBOLS = {
    "dp_pix_plan_create": (_st, [_P(FrameDesc), ctypes.c_int32, _P(_vp)]),
    "dp_pix_plan_destroy": (None, [_vp]),
    "dp_pix_plan_sizes": (_st, [_vp, _P(Sizes)]),
    "dp_pix_plan_workspace_size": (_st, [_P(FrameDesc), ctypes.c_int32, _P(Sizes)]),
    "dp_pix_plan_frame_info": (_st, [_vp, ctypes.c_int32, _P(FrameInfo)]),
    "dp_pix_plan_bind": (_st, [_vp, _vp, ctypes.c_size_t, _vp]),
    "dp_pix_plan": (_st, [_vp, _vp, _P(Store), _vp]),
    "dp_pix_plan_labels": (_st, [_vp, _vp, ctypes.c_int32, _P(Store), _vp]),
    "dp_pix_store_index": (_st, [_vp, _P(Store), _vp]),
    "dp_pix_noise_advance": (_st, [_vp, ctypes.c_int32, ctypes.c_uint64, _vp]),
    "dp_pix_edge_mask": (_st, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
    "dp_pix_forward": (_st, [_vp, _vp, _P(Store), _vp, _vp, _vp, _vp]),
    "dp_pix_reconstruct": (_st, [_vp, _P(Store), _vp, _vp]),
    "dp_pix_backward": (_st, [_vp, _P(Store), _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dp_pix_backward_static": (_st, [_vp, _P(Store), _vp, _vp, _vp, _vp, _vp]),
    "dp_pix_plan_set_launch": (_st, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "dp_pix_graph_create": (_st, [_vp, _vp, _vp, _P(Store), _vp, _vp, _P(_vp)]),
    "dp_pix_graph_launch": (_st, [_vp, _vp]),
    "dp_pix_graph_destroy": (None, [_vp]),
    "dp_pix_debug_sums": (_st, [_vp, _vp, _P(Store), _vp, _vp, _vp]),
    "dp_pix_debug_philox": (_st, [_vp, _vp, ctypes.c_int64, _vp]),
    "dp_pix_metrics": (_st, [_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
    "dp_pix_status_string": (ctypes.c_char_p, [_st]),
    "dp_pix_last_error": (ctypes.c_char_p, []),
    "dp_pix_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libdppix and declare its prototypes.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libdppix.so is not built at %s; run __graft_entry__.build() "
                           "(there is no CPU fallback)" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != DPPIX_OK:
        detail = _lib.dp_pix_last_error().decode(errors="replace") if _lib is not None else ""
        raise DppixError(status, detail)
