"""Host logic of bench.py (no GPU): the algorithmic byte counts the roofline
divides by, the counter-file scaling of the traffic figure, and the refusal
of multi-GPU runs."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("args, kw, want", [
    # 100k buses, one state, element-wise S+J:
    # 16 nb (v, theta) + 16 nb (P, Q) + 8 nnzJ + 48 nl + 16 nb + 4 (nb + 1)
    ((100_000, 130_000, 360_000, 1), {}, 3_200_000 + 11_520_000 + 6_240_000 + 1_600_000 + 400_004),
    # the same outputs by the Ybus method: 20 nnzY of grid data instead
    ((100_000, 130_000, 360_000, 1), {"method": "ybus"}, 3_200_000 + 11_520_000 + 7_200_000 + 400_004),
    # 512 states of the 20k-bus grid
    ((20_000, 27_000, 74_000, 512), {}, 512 * (640_000 + 2_368_000) + 1_296_000 + 320_000 + 80_004),
    # 32 states of the 100k-bus grid: injections only, and the adjoint (32 nb in, 16 nb out)
    ((100_000, 130_000, 360_000, 32), {"with_j": False}, 32 * 3_200_000 + 8_240_004),
    ((100_000, 130_000, 360_000, 32), {"vjp": True}, 32 * 4_800_000 + 8_240_004),
])
def test_algorithmic_bytes(args, kw, want):
    assert bench.algorithmic_bytes(*args, **kw) == want


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, v in rows:
            f.write(f'{d},"{name}",{counter},{v}\n')


def test_traffic_from_counter_files(tmp_path):
    head = "void pf::k_ew<256, false, true, true, false>(pf::DevGrid, int)"
    copy = "__amd_rocclr_copyBuffer"
    copy_kib = 8 * bench.COPY_PROBE_DOUBLES / 1024.0
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    # FETCH_SIZE: the copy reads half its bytes by the counter (scale 2);
    # two dispatches of the headline kernel, counted in two parts each
    _counter_csv(f, "FETCH_SIZE", [(1, head, 2000.0), (1, head, 1000.0), (2, head, 3000.0),
                                   (3, copy, 0.5 * copy_kib), (4, copy, 10.0)])
    # WRITE_SIZE: exact
    _counter_csv(w, "WRITE_SIZE", [(1, head, 4000.0), (2, head, 6000.0), (3, copy, copy_kib)])
    r = bench.traffic_from_csv(str(f), str(w))
    assert r["FETCH_SIZE"]["dispatches"] == 2
    assert r["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert r["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(3000.0 * 1024 * 2)
    assert r["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    assert r["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(5000.0 * 1024)
    assert r["bytes_per_launch"] == pytest.approx(3000.0 * 1024 * 2 + 5000.0 * 1024)
    assert r["kernel_sha256_16"] == bench.kernel_hash()


def test_recorded_traffic_needs_the_same_kernel_sources(tmp_path):
    import json
    good = tmp_path / "t.json"
    good.write_text(json.dumps({"kernel_sha256_16": bench.kernel_hash(), "bytes_per_launch": 123.0}))
    assert bench.recorded_traffic(str(good)) == 123.0
    stale = tmp_path / "s.json"
    stale.write_text(json.dumps({"kernel_sha256_16": "0" * 16, "bytes_per_launch": 123.0}))
    assert bench.recorded_traffic(str(stale)) is None
    assert bench.recorded_traffic(str(tmp_path / "missing.json")) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stdout + p.stderr
