"""Host run of the per-slice index logic of the kernels (panel index on
sorted, descending and shuffled slices; the sorting network that orders the
slices of unsorted operands), compiled from the library's own header."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rowlogic_on_host(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "rowlogic_test"
    src = os.path.join(ROOT, "tests", "host", "rowlogic_test.cpp")
    inc = os.path.join(ROOT, "paper_2106_14402_amd", "csrc")
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I", inc, src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "rowlogic ok" in r.stdout
