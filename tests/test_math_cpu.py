"""The kernels' sine/cosine (pf_math.h), compiled for the host from the same
source, against 80-bit sinl/cosl over many argument ranges; and the kernels'
wave-wide shortcut for quadrant count 0 (the series alone on x),
which must reproduce the full function's bits."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_sincos_accuracy(tmp_path):
    exe = tmp_path / "sincos_check"
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.fail("hipcc is required to compile the kernel math header")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", os.path.join(HERE, "native", "sincos_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    max_abs, max_ulp, n = float(out[0]), float(out[1]), int(out[2])
    n0, n0_diff = int(out[3]), int(out[4])
    assert n > 2_000_000
    assert n0 > 400_000, n0
    assert n0_diff == 0, n0_diff
    assert max_abs <= 3.0e-16, max_abs   # absolute, results in [-1, 1]
    assert max_ulp <= 2.5, max_ulp       # relative where |result| >= 2^-10
