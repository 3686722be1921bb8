"""The device sine/cosine (own quarter-turn reduction and Taylor polynomials, used by every
cone step) built for the host and checked against FP64 sin/cos over every heading grid
point and every Box-Muller uniform: within 1.5 * 2^-24.  The helpers use only fma, mul, add
and rint, so the host build computes the same bits as the GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1405_3331_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_device_sincos_error_bound(tmp_path):
    exe = str(tmp_path / "sincos_driver")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-ffp-contract=off", "-x", "hip",
                    "--cuda-host-only", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "device_math", "sincos_driver.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    fields = out.split()
    angle, turn = float(fields[1]), float(fields[3])
    print(out.strip())
    assert angle <= 1.5, out
    assert turn <= 1.5, out
