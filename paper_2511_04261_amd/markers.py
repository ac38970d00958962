"""ROCTx ranges around host-side phases, for the profiler's marker trace
(``rocprofv3 --marker-trace``): the serving loop's completions, admissions
and batch launches then appear on the timeline beside the kernels they
issue.

The ROCTx library is opened on first use from the ROCm installation
(``ROCM_PATH``, default /opt/rocm); where it is absent, or ``DPPIX_ROCTX=0``
is set, every range is a no-op.  Ranges nest per host thread; a range is
popped on the way out of its ``with`` block even when the block raises.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import threading

_NAMES = ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4", "libroctx64.so")
_lock = threading.Lock()
_lib = None
_tried = False


def library():
    """The opened ROCTx library, or None when markers are off or it is absent."""
    global _lib, _tried
    if _tried:
        return _lib
    with _lock:
        if _tried:
            return _lib
        if os.environ.get("DPPIX_ROCTX", "1") != "0":
            root = os.environ.get("ROCM_PATH", "/opt/rocm")
            for name in _NAMES:
                path = os.path.join(root, "lib", name)
                if not os.path.exists(path):
                    continue
                try:
                    lib = ctypes.CDLL(path)
                    lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                    lib.roctxRangePushA.restype = ctypes.c_int
                    lib.roctxRangePop.argtypes = []
                    lib.roctxRangePop.restype = ctypes.c_int
                    lib.roctxMarkA.argtypes = [ctypes.c_char_p]
                    lib.roctxMarkA.restype = None
                except (OSError, AttributeError):
                    continue
                _lib = lib
                break
        _tried = True
    return _lib


@contextlib.contextmanager
def marker_range(name: str):
    """A ROCTx range named ``name`` around the block."""
    lib = library()
    if lib is None:
        yield
        return
    lib.roctxRangePushA(name.encode())
    try:
        yield
    finally:
        lib.roctxRangePop()


def mark(name: str):
    """A single ROCTx marker."""
    lib = library()
    if lib is not None:
        lib.roctxMarkA(name.encode())
