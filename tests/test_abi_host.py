"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/dppix.h declares, validates arguments before touching
the device, and lays out geometry, tiles and store capacities as the paper's
formulas say."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

dp = pytest.importorskip("paper_2511_04261_amd")
from paper_2511_04261_amd import _lib  # noqa: E402


def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2511_04261_amd import build
        build.build()
    return _lib.load()


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "dppix.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_pix_\w+)\s*\(", txt)))


def test_library_exports_every_header_symbol():
    L = lib()
    syms = header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
        assert s in _lib.SYMBOLS, "binding misses %s" % s
    assert set(_lib.SYMBOLS) == set(syms)
    assert L.dp_pix_version().startswith(b"dppix")


LAYOUT_PROG = r"""
#include <stddef.h>
#include <stdio.h>
#include "dppix.h"
#define F(T, m) printf(#T " " #m " %zu %zu\n", offsetof(T, m), sizeof(((T*)0)->m))
int main(void) {
  printf("dppix_frame_desc_t size %zu 0\n", sizeof(dppix_frame_desc_t));
  printf("dppix_store_t size %zu 0\n", sizeof(dppix_store_t));
  printf("dppix_sizes_t size %zu 0\n", sizeof(dppix_sizes_t));
  printf("dppix_frame_info_t size %zu 0\n", sizeof(dppix_frame_info_t));
  F(dppix_frame_desc_t, pitch); F(dppix_frame_desc_t, eps_bg); F(dppix_frame_desc_t, seed);
  F(dppix_frame_desc_t, frame_index); F(dppix_frame_desc_t, tile_cells);
  F(dppix_sizes_t, n_tiles); F(dppix_sizes_t, total_pixels); F(dppix_sizes_t, store_state_bytes); F(dppix_sizes_t, forward_launches);
  F(dppix_store_t, counts); F(dppix_store_t, state); F(dppix_store_t, noise);
  F(dppix_frame_info_t, cell_offset); F(dppix_frame_info_t, sigma_fg);
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the C compiler's sizes and field offsets."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_PROG)
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    names = {"dppix_frame_desc_t": _lib.FrameDesc, "dppix_store_t": _lib.Store, "dppix_sizes_t": _lib.Sizes,
             "dppix_frame_info_t": _lib.FrameInfo}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        t, field, off, size = line.split()
        cls = names[t]
        if field == "size":
            assert ctypes.sizeof(cls) == int(off), t
        else:
            assert getattr(cls, field).offset == int(off), (t, field)
            assert getattr(cls, field).size == int(size), (t, field)


def create(frames):
    L = lib()
    n = len(frames)
    d = (_lib.FrameDesc * n)(*[f.desc() for f in frames])
    h = ctypes.c_void_p()
    st = L.dp_pix_plan_create(d, n, ctypes.byref(h))
    return st, h, L


def info(h, L, f=0):
    fi = _lib.FrameInfo()
    assert L.dp_pix_plan_frame_info(h, f, ctypes.byref(fi)) == 0
    return fi


@pytest.mark.parametrize("kw,status", [
    (dict(height=0, width=10), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, channels=5), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, b=16, sb=5), _lib.DPPIX_EINVAL),        # b % s_b != 0 (Eq. 16)
    (dict(height=10, width=10, b=8, sb=16), _lib.DPPIX_EINVAL),        # s_b > b
    (dict(height=10, width=10, m=0), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, eps_bg=0.0), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, eps_bg=-1.0), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, eps_bg=float("nan")), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, tau=257, b=16), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, pitch=5), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, pad_mode=3), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, layout=7), _lib.DPPIX_EINVAL),
    (dict(height=10, width=10, b=512, sb=512), _lib.DPPIX_ENOTSUP),
    (dict(height=1 << 25, width=10), _lib.DPPIX_ENOTSUP),
])
def test_invalid_descriptors_rejected_on_host(kw, status):
    st, h, L = create([dp.FrameParams(**kw)])
    assert st == status
    assert not h.value
    assert len(L.dp_pix_last_error()) > 0


def test_null_and_empty_arguments():
    L = lib()
    h = ctypes.c_void_p()
    assert L.dp_pix_plan_create(None, 1, ctypes.byref(h)) == _lib.DPPIX_EINVAL
    d = (_lib.FrameDesc * 1)(dp.FrameParams(8, 8).desc())
    assert L.dp_pix_plan_create(d, 0, ctypes.byref(h)) == _lib.DPPIX_EINVAL
    assert L.dp_pix_plan_create(d, 1, None) == _lib.DPPIX_EINVAL
    st, h, L = create([dp.FrameParams(8, 8)])
    assert st == 0
    # unbound plan: device calls refuse before enqueueing anything
    s = _lib.Store()
    assert L.dp_pix_plan(h, None, ctypes.byref(s), None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_forward(h, None, ctypes.byref(s), None, None, None, None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_reconstruct(h, ctypes.byref(s), None, None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_store_index(h, ctypes.byref(s), None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_noise_advance(None, 1, 1, None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_noise_advance(None, -1, 1, None) == _lib.DPPIX_EINVAL
    assert L.dp_pix_noise_advance(None, 0, 1, None) == 0          # nothing to do, nothing enqueued
    assert L.dp_pix_plan_set_launch(h, 96, 0) == _lib.DPPIX_EINVAL
    assert L.dp_pix_plan_set_launch(h, 1024, 0) == _lib.DPPIX_EINVAL
    assert L.dp_pix_plan_set_launch(h, 128, 1) == 0
    assert L.dp_pix_plan_frame_info(h, 1, ctypes.byref(_lib.FrameInfo())) == _lib.DPPIX_EINVAL
    assert L.dp_pix_debug_philox(None, None, -1, None) == _lib.DPPIX_EINVAL
    L.dp_pix_plan_destroy(h)
    L.dp_pix_plan_destroy(None)
    L.dp_pix_graph_destroy(None)


@pytest.mark.parametrize("H,W,b,sb", [(256, 256, 16, 16), (1080, 1920, 32, 8), (2160, 3840, 16, 4),
                                      (4000, 6000, 32, 4), (5, 3, 8, 2), (1, 1, 1, 1), (17, 33, 16, 8)])
def test_geometry_and_capacities(H, W, b, sb):
    C = 3
    st, h, L = create([dp.FrameParams(H, W, C, b=b, sb=sb, m=16, eps_bg=1.0, eps_fg=0.3)])
    assert st == 0
    fi = info(h, L)
    GR, GC, n = math.ceil(H / b), math.ceil(W / b), b // sb       # Alg. 3 step 1, Eq. 16
    assert (fi.grid_rows, fi.grid_cols, fi.n) == (GR, GC, n)
    assert (fi.pad_rows, fi.pad_cols) == (GR * b - H, GC * b - W)  # Alg. 3 step 2
    assert fi.fg_min_count == (b * b + 1) // 2                     # tau = 0 -> paper's majority rule
    assert fi.sigma_bg == pytest.approx(255 * 16 / (b * b * 1.0), rel=1e-15)   # Eq. 11
    assert fi.sigma_fg == pytest.approx(255 * 16 / (sb * sb * 0.3), rel=1e-15)
    sz = _lib.Sizes()
    assert L.dp_pix_plan_sizes(h, ctypes.byref(sz)) == 0
    assert sz.flag_bytes == GR * GC
    assert sz.bg_capacity == GR * GC * C
    assert sz.fg_capacity == GR * GC * n * n * C
    assert sz.total_pixels == H * W
    assert fi.tiles_per_band * fi.tile_cells >= GC and (fi.tiles_per_band - 1) * fi.tile_cells < GC
    assert sz.n_tiles == GR * fi.tiles_per_band
    L.dp_pix_plan_destroy(h)


def test_noise_off_has_zero_sigma_and_batch_offsets():
    frames = [dp.FrameParams(100, 90, 3, b=16, sb=4, eps_bg=math.inf, eps_fg=math.inf),
              dp.FrameParams(33, 7, 1, b=8, sb=8), dp.FrameParams(64, 64, 3, b=32, sb=8, tile_cells=1)]
    st, h, L = create(frames)
    assert st == 0
    fi = [info(h, L, f) for f in range(3)]
    assert fi[0].sigma_bg == 0.0 and fi[0].sigma_fg == 0.0
    cells = [x.grid_rows * x.grid_cols for x in fi]
    assert [x.cell_offset for x in fi] == [0, cells[0], cells[0] + cells[1]]
    fines = [x.grid_rows * x.grid_cols * x.n * x.n for x in fi]
    assert [x.fine_offset for x in fi] == [0, fines[0], fines[0] + fines[1]]
    assert fi[2].tile_cells == 1 and fi[2].tiles_per_band == 2
    L.dp_pix_plan_destroy(h)


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load(str(tmp_path / "missing.so"))


def test_unpadded_mode_geometry():
    """Algorithm 1 border mode: same grid, no padding, tau 0 = per-cell majority."""
    st, h, L = create([dp.FrameParams(45, 70, 3, b=16, sb=4, pad_mode=dp.PAD_NONE)])
    assert st == 0
    fi = info(h, L)
    assert (fi.grid_rows, fi.grid_cols) == (3, 5)
    assert fi.fg_min_count == 0
    L.dp_pix_plan_destroy(h)
    st, h, L = create([dp.FrameParams(45, 70, 3, b=16, sb=4, pad_mode=dp.PAD_NONE, tau=3)])
    assert st == 0 and info(h, L).fg_min_count == 3
    L.dp_pix_plan_destroy(h)


def test_plans_for_extreme_and_mixed_batches():
    """Host layout of batches that stress the tile and plan-unit arithmetic:
    very wide and very tall frames, b = 1 and b = 256, every (layout,
    channels) pair in one batch (the most launch groups), explicit tile
    widths from 1 to far past the grid.  Plan creation succeeds, the
    workspace covers the tables, and the frames' cells are laid out back to
    back."""
    frames = [dp.FrameParams(3, 1 << 20, 1, b=1, sb=1), dp.FrameParams(1 << 16, 7, 4, b=256, sb=16),
              dp.FrameParams(600, 900, 2, b=3, sb=1, tile_cells=1), dp.FrameParams(17, 4001, 3, b=12, sb=4,
                                                                                  tile_cells=100000)]
    for C in (1, 2, 3, 4):
        frames.append(dp.FrameParams(40, 50, C, dp.U8_HWC, b=8, sb=4))
        frames.append(dp.FrameParams(40, 50, C, dp.F32_CHW, b=8, sb=4))
        frames.append(dp.FrameParams(300, 520, C, dp.U8_HWC, b=16, sb=4))   # small tiles: 128-lane group
    st, h, L = create(frames)
    assert st == 0, L.dp_pix_last_error()
    sz = _lib.Sizes()
    assert L.dp_pix_plan_sizes(h, ctypes.byref(sz)) == 0
    cells = 0
    tiles = 0
    for f, fp in enumerate(frames):
        fi = info(h, L, f)
        assert fi.cell_offset == cells
        cells += fi.grid_rows * fi.grid_cols
        assert 1 <= fi.tile_cells <= fi.grid_cols
        assert fi.tiles_per_band == -(-fi.grid_cols // fi.tile_cells)
        tiles += fi.grid_rows * fi.tiles_per_band
    assert sz.flag_bytes == cells and sz.n_tiles == tiles
    # the workspace holds the frame records and the tile and plan-unit maps;
    # each store's state holds two per-tile counters and the ticket words
    assert sz.workspace_bytes >= 144 * len(frames) + 8 * tiles
    assert sz.store_state_bytes >= 8 * tiles + 4 * 33
    L.dp_pix_plan_destroy(h)


def test_workspace_size_without_a_plan():
    """dp_pix_plan_workspace_size gives the sizes of dp_pix_plan_sizes for the
    same descriptors, host only, and the status of dp_pix_plan_create for
    invalid ones."""
    L = lib()
    frames = [dp.FrameParams(1080, 1920, 3, b=32, sb=8, eps_bg=1.0, eps_fg=0.3, tau=1),
              dp.FrameParams(576, 768, 3, b=16, sb=4), dp.FrameParams(37, 41, 1, dp.F32_CHW, b=8, sb=2)]
    d = (_lib.FrameDesc * 3)(*[f.desc() for f in frames])
    a = _lib.Sizes()
    assert L.dp_pix_plan_workspace_size(d, 3, ctypes.byref(a)) == 0
    st, h, L = create(frames)
    assert st == 0
    b = _lib.Sizes()
    assert L.dp_pix_plan_sizes(h, ctypes.byref(b)) == 0
    L.dp_pix_plan_destroy(h)
    for name, _ in _lib.Sizes._fields_:
        assert getattr(a, name) == getattr(b, name), name
    assert a.store_state_bytes > 0 and a.workspace_bytes > 0
    bad = (_lib.FrameDesc * 1)(dp.FrameParams(10, 10, b=16, sb=5).desc())
    assert L.dp_pix_plan_workspace_size(bad, 1, ctypes.byref(a)) == _lib.DPPIX_EINVAL
    assert L.dp_pix_plan_workspace_size(d, 0, ctypes.byref(a)) == _lib.DPPIX_EINVAL
    assert L.dp_pix_plan_workspace_size(d, 3, None) == _lib.DPPIX_EINVAL


def test_host_masks_and_in_place_outputs_are_refused():
    """The Python face refuses, before any launch, masks that are not CUDA
    tensors (their host address would reach the plan kernel) and fused
    outputs that overlap their images."""
    torch = pytest.importorskip("torch")
    frames = [dp.FrameParams(8, 12, 3)]
    cuda0 = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="CUDA"):
        dp.check_masks(frames, [torch.zeros((8, 12), dtype=torch.uint8)], cuda0)
    with pytest.raises(ValueError, match="one mask"):
        dp.check_masks(frames, [None, None], cuda0)
    dp.check_masks(frames, [None], cuda0)
    dp.check_masks(frames, None, cuda0)
    x = torch.zeros((8, 12, 3), dtype=torch.uint8)
    with pytest.raises(ValueError, match="overlaps"):
        dp.check_no_alias([x], [x])
    with pytest.raises(ValueError, match="overlaps"):
        big = torch.zeros((16, 12, 3), dtype=torch.uint8)
        dp.check_no_alias([big[:8]], [big[4:12]])
    big = torch.zeros((16, 12, 3), dtype=torch.uint8)
    dp.check_no_alias([big[:8]], [big[8:]])
    dp.check_no_alias([x], [torch.zeros_like(x)])


@pytest.mark.parametrize("H,W,b,K", [(576, 768, 16, 24), (576, 768, 32, 12), (1080, 1920, 32, 20), (1080, 1920, 16, 40),
                                     (4000, 6000, 16, 42), (4000, 6000, 32, 21), (2160, 3840, 16, 40)])
def test_default_tile_width(H, W, b, K):
    """The library's tile width for RGB frames: each band's padded row cut
    into the fewest tiles of at most about 2 KB (a band of 2304 bytes is two
    tiles), the widths the profiled batches ran with."""
    st, h, L = create([dp.FrameParams(H, W, 3, b=b, sb=b // 4, m=16, eps_bg=1.0, eps_fg=0.3)])
    assert st == 0
    assert info(h, L).tile_cells == K
    L.dp_pix_plan_destroy(h)
