"""Build libdppix.so in-tree for gfx950 with hipcc (no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "dppix_kernels.hip"), os.path.join(HERE, "csrc", "dppix_api.hip")]
OUT = os.path.join(HERE, "libdppix.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "dppix_probes.hip")]
PROBE_OUT = os.path.join(HERE, "libdppix_probes.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed fp32 instructions are disabled: hipcc would form them from plain
# float code, and the kernels do not need them.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    """libdppix.so, then the streaming probes' libdppix_probes.so (the HBM
    ceilings bench.py --ceilings measures)."""
    _compile(SOURCES, OUT, verbose)
    _compile(PROBE_SOURCES, PROBE_OUT, verbose)
    return OUT


def _compile(sources, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + sources
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    noise = [ln for ln in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(noise))
    if verbose and noise:
        print("\n".join(noise), file=sys.stderr)
    os.replace(tmp, out)


if __name__ == "__main__":
    print(build(verbose=True))
