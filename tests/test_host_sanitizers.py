"""Host-side sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer,
no recovery): the oracle's C++ on small random operands of every semiring
and layout, and the C ABI's host code (plan creation, workspace layouts,
option and descriptor checks) built with the sanitizers on the host side
only.  CPU only: no device work is done."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(exe, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)


def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "san_oracle"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", *SAN, "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "oracle.cpp"), os.path.join(ROOT, "tests", "host", "sanitize_oracle.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = _run(exe, leaks=True)
    assert r.returncode == 0 and "oracle sanitize ok" in r.stdout, r.stdout + r.stderr


def test_abi_host_code_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "san_abi"
    csrc = os.path.join(ROOT, "paper_2106_14402_amd", "csrc")
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]  # host side only
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", *host_san, "-I", os.path.join(ROOT, "include"),
           os.path.join(csrc, "spg_api.hip"), os.path.join(csrc, "spg_kernels.hip"), os.path.join(csrc, "spg_batch.hip"),
           os.path.join(ROOT, "tests", "host", "sanitize_abi.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # leaks: the HIP runtime's own allocations at exit are not the library's
    r = _run(exe, leaks=False)
    assert r.returncode == 0 and "abi sanitize ok" in r.stdout, r.stdout + r.stderr
