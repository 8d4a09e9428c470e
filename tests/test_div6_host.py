"""The library's FP64 division by 6 (`gs::div6` in the device header, a
host-and-device function) compiled for the host and compared bit for bit with
the IEEE quotient x / 6 (Eq. 3 divides the neighbour sum by 6 with true
division): every subnormal argument m 2^-1074 with m < 2^20, the normal
arguments whose quotient is subnormal or just normal, a band around 6 2^-1022,
20 million random finite doubles, and Laplacian numerators built from
subnormal neighbours. The documented differences are checked too: both zeros
give +0 (no stored value of the step depends on that sign) and +-Inf give
NaN."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_div6_matches_ieee_division(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "div6_check"
    cmd = [hipcc, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-ffp-contract=off",
           os.path.join(ROOT, "tests", "aux", "div6_host_check.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert out.stdout.startswith("ok"), out.stdout
