"""The streaming probes' library (the HBM ceilings bench.py --ceilings
measures) loads and refuses shapes it does not cover before any launch; no
GPU is needed for that."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_04261_amd", "libdppix_probes.so")
INVALID = 1   # hipErrorInvalidValue


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libdppix_probes.so is not built")
    L = ctypes.CDLL(LIB)
    L.dppix_probe_stream.restype = ctypes.c_int
    L.dppix_probe_stream.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32,
                                     ctypes.c_void_p]
    L.dppix_probe_tiles.restype = ctypes.c_int
    L.dppix_probe_tiles.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    return L


def test_stream_probe_refuses_bad_shapes(lib):
    a, b = 0x100000, 0x200000          # never dereferenced: every call below is refused first
    assert lib.dppix_probe_stream(0, a, b, 0, 0, None) == INVALID          # empty
    assert lib.dppix_probe_stream(0, a, b, 24, 0, None) == INVALID         # not whole 16-byte words
    assert lib.dppix_probe_stream(3, a, b, 32, 0, None) == INVALID         # no such mode
    assert lib.dppix_probe_stream(0, a + 8, b, 32, 0, None) == INVALID     # misaligned
    assert lib.dppix_probe_stream(0, None, b, 32, 0, None) == INVALID      # copy without a source
    assert lib.dppix_probe_stream(2, None, None, 32, 0, None) == INVALID   # write without a destination


def test_tile_probe_refuses_bad_shapes(lib):
    a, b = 0x100000, 0x200000
    ok = dict(frames=2, frame_bytes=1088 * 5760, pitch=5760, rows=1088, row_bytes=5760, tile_rows=32, tile_bytes=1920)

    def call(**kw):
        k = dict(ok, **kw)
        return lib.dppix_probe_tiles(a, b, k["frames"], k["frame_bytes"], k["pitch"], k["rows"], k["row_bytes"],
                                     k["tile_rows"], k["tile_bytes"], None)
    assert call(tile_rows=64, tile_bytes=1040) == INVALID    # more strips than a workgroup holds (4160 > 4096)
    assert call(tile_bytes=1000) == INVALID                  # not whole strips
    assert call(pitch=5000) == INVALID                       # rows shorter than their bytes
    assert call(frame_bytes=1088 * 5760 - 16) == INVALID     # frames overlapping
    assert call(frames=0) == INVALID
