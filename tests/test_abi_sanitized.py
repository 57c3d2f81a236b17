"""The C entry points' host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): tests/abi_driver.cpp exercises every
call's validation, error codes, workspace sizes and the exchange-grid rule,
and the batch tune cache's handling of malformed entries.
capi.cpp and the driver are compiled with the sanitizers on the host side;
the kernel objects of the regular build are linked unchanged."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1305_7313_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_is_clean_under_sanitizers(tmp_path):
    objs = [os.path.join(PKG, "_build", f) for f in ("kernels_c128.o", "kernels_c64.o", "kernels_common.o")]
    if not all(os.path.exists(o) for o in objs):
        import sys
        sys.path.insert(0, PKG)
        import build
        build.build(verbose=False)
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")] + SAN
    capi = str(tmp_path / "capi.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "abi_driver")
    for src, obj in ((os.path.join(PKG, "csrc", "capi.cpp"), capi), (os.path.join(ROOT, "tests", "abi_driver.cpp"), drv)):
        r = subprocess.run([HIPCC] + common + ["-x", "hip", "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + SAN + [drv, capi] + objs + ["-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "0 failure(s)" in out
