"""Host-only checks built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU; no GPU and no HIP compiler involved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_14372_amd", "csrc")
SANITIZE = ["-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-fsanitize=address,undefined"]


def test_host_propagator_construction(tmp_path):
    """The host-side propagator tables and their separable factors
    (csrc/pty_prop.hpp) against the Fresnel propagator written out in double."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "propagator_check"
    src = os.path.join(ROOT, "tests", "host", "propagator_check.cpp")
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-g", *SANITIZE, "-I", CSRC, src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
