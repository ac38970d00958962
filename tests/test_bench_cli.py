"""bench.py's contract on the host: more than one GPU is refused with a
message before anything touches a device, and the HBM traffic of the
roofline block is taken from the committed counter summary only for the
build and launch shapes it was measured on."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _plan(tile_cells=20, threads=0):
    fp = SimpleNamespace(height=1080, width=1920, channels=3, b=32, sb=8)
    return SimpleNamespace(frames=[fp], info=[SimpleNamespace(tile_cells=tile_cells)], threads=threads, persistent=0)


def test_traffic_only_for_the_measured_build(monkeypatch):
    plan = _plan()
    kv = {"kernel_source_sha256_16": bench.kernel_source_hash(), "launch_signature": bench.launch_signature(plan),
          "fetch_kib_per_dispatch": "1000.0", "fetch_scale": "2.0", "write_kib_per_dispatch": "500.0",
          "write_scale": "1.0"}
    monkeypatch.setattr(bench, "read_counters", lambda path=None: dict(kv))
    assert bench.read_traffic(plan) == pytest.approx(1000.0 * 1024 * 2.0 + 500.0 * 1024 * 1.0)
    # other tile widths or launch shape: not the measured launches
    assert bench.read_traffic(_plan(tile_cells=21)) is None
    assert bench.read_traffic(_plan(threads=128)) is None
    # other kernels
    monkeypatch.setattr(bench, "read_counters", lambda path=None: dict(kv, kernel_source_sha256_16="0" * 16))
    assert bench.read_traffic(plan) is None
    # a malformed summary is no summary
    monkeypatch.setattr(bench, "read_counters", lambda path=None: {k: v for k, v in kv.items() if k != "fetch_scale"})
    assert bench.read_traffic(plan) is None


def test_source_hash_ignores_comments(tmp_path):
    csrc = tmp_path / "paper_2511_04261_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in ("dppix_kernels.hip", "dppix_internal.h", "dppix_tiles.h", "dppix_api.hip"):
        (csrc / name).write_text("int f(int x) { return x + 1; }\n")
    h0 = bench.kernel_source_hash(str(tmp_path))
    (csrc / "dppix_kernels.hip").write_text("// a comment\nint f(int x) { return x + 1; }  /* same code */\n\n")
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    (csrc / "dppix_kernels.hip").write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash(str(tmp_path)) != h0
