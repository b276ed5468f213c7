"""The library's host code (gpcg_host.cpp with the kernel sources linked as
usual) built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
side only, driving the host preparation passes through the C ABI on 300
seeded random grids and on malformed inputs (tests/sanitize/host_passes.cpp).
CPU only: no GPU call is made."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1803_03290_amd", "csrc")


def test_host_passes_under_address_and_ub_sanitizers():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    tmp = tempfile.mkdtemp(prefix="gpcg_san_")
    try:
        exe = os.path.join(tmp, "host_passes")
        # sanitizers on the host code only (each flag right after -Xarch_host)
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined",
               "-I", os.path.join(ROOT, "include"),
               os.path.join(CSRC, "gpcg_host.cpp"), os.path.join(CSRC, "gpcg_tile.hip"),
               os.path.join(CSRC, "gpcg_kernels.hip"), os.path.join(ROOT, "tests", "sanitize", "host_passes.cpp"),
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and "ok" in r.stdout, out[-3000:]
        assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
