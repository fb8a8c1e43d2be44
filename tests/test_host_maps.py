"""Host-side checks of the kernels' index maps: `tests/host_maps_check.cpp`
includes the library's internal header and is compiled by hipcc as a host
program (no device code runs)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_host_maps(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_maps_check"
    src = os.path.join(ROOT, "tests", "host_maps_check.cpp")
    r = subprocess.run([HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-4000:]
