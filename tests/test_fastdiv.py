"""The multiply-shift division behind the fused kernels' cell indices
(Granlund and Montgomery's Thm. 4.2 with N = 31: m = ceil(2^(31+l) / d),
l = ceil(log2 d)), compiled from the library's own header for the host and
checked against integer division (tests/fastdiv_check.cpp).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_fastdiv_matches_integer_division(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = tmp_path / "fastdiv_check"
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
           "-I", os.path.join(ROOT, "paper_1711_10885_amd", "csrc"),
           os.path.join(ROOT, "tests", "fastdiv_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert int(r.stdout.split()[-1]) > 1_000_000
