"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only, no GPU): tests/native/host_checks.c drives pattern building, the
tile and lane tables of every tile size, pattern export, the Algorithm 2
index map and the argument checks through the C ABI on host-only handles.
The sanitizers instrument host code only; the kernels are compiled as usual
and never launched."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2302_10736_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
COMMON = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=off", "-I", os.path.join(ROOT, "include")]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_under_sanitizers(tmp_path):
    objs = []
    for src in ("pf_api.cpp", "pf_kernels.hip", "pf_probe.hip"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([HIPCC, *COMMON, "-std=c++17", *HOST_SAN, "-c", os.path.join(CSRC, src), "-o", obj],
                       check=True, capture_output=True, timeout=600)
        objs.append(obj)
    drv = str(tmp_path / "host_checks.o")
    subprocess.run([HIPCC, "-x", "c", "-O1", "-g", *HOST_SAN, "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(ROOT, "tests", "native", "host_checks.c"), "-o", drv],
                   check=True, capture_output=True, timeout=300)
    exe = str(tmp_path / "host_checks")
    subprocess.run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, drv, *objs, "-o", exe], check=True,
                   capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-6000:]
    assert "host checks passed" in p.stdout
