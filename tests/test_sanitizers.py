"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code.

- The oracle (oracle/dppix_oracle.c), compiled with gcc and both
  sanitizers, runs every one of its functions over random small frames and
  the degenerate cases (tests/sanitize/oracle_driver.c).
- The host side of libdppix (descriptor validation, plan layout, sizes,
  frame information, refusals of unbound plans), compiled with the
  sanitizers on its host code only, is driven with valid and invalid
  descriptors (tests/sanitize/abi_host_driver.c).  No GPU is needed.

Any invalid access or undefined operation aborts the program
(-fno-sanitize-recover=all), which fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                           os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "dppix_oracle.c"),
                           "-o", exe, "-lm"])
    _run(exe)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang")
def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2511_04261_amd", "csrc")
    lib = str(tmp_path / "libdppix_san.so")
    # sanitizers on the host pass only: the device code is built as usual
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-Xarch_host", "-fno-sanitize-recover=all",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", lib,
                        os.path.join(csrc, "dppix_kernels.hip"), os.path.join(csrc, "dppix_api.hip")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "abi_driver")
    subprocess.check_call([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"), os.path.join(SAN, "abi_host_driver.c"),
                           "-L", str(tmp_path), "-ldppix_san", "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe])
    _run(exe)
