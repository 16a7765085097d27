"""CPU: the benchmark's host-side contract (no GPU needed).

- More than one GPU is refused with a message (this build measures one GPU).
- The roofline figure is algorithmic work per launch over the average launch time.
- The M2L flop count per interaction-list entry is the one the kernel performs (4p^2 + 14p).
- Counter-derived traffic is reported only for a kernel with a committed counter record.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_roofline_is_work_per_launch_over_launch_time():
    prof = {"ms_total": 2.0, "launches": 4, "pairs": 4.0e9}
    rl = bench.roofline(prof, 0, 11, "f64", bound="alu", kernel=None)
    assert rl["avg_launch_ms"] == pytest.approx(0.5)
    assert rl["units_per_launch"] == pytest.approx(1.0e9)
    # 11 flops x 1e9 units in 0.5 ms = 22 TFLOP/s against the 78.6 TFLOP/s float64 peak
    assert rl["achieved"] == pytest.approx(22.0)
    assert rl["frac"] == pytest.approx(22.0 / 78.6)
    assert rl["traffic"] is None and rl["unit"] == "TFLOP/s"


def test_m2l_flops_per_entry():
    # p complex scalings (6 flops each), the real p x p Hankel product on the real and imaginary
    # parts (4 p^2), p complex multiply-adds (8 flops each)
    for p in (8, 24, 40, 64):
        assert bench.m2l_flops_per_entry(p) == 6 * p + 4 * p * p + 8 * p
    assert bench.m2l_flops_per_entry(40) == 6960


def test_traffic_only_for_recorded_kernels():
    assert bench.traffic_bytes(None) is None
    assert bench.traffic_bytes("no_such_kernel<1>") is None
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for name, r in rec.items():
        v = bench.traffic_bytes(name)
        # a number while the kernel's source is the one the counters were taken on, else None
        assert v is None or v == pytest.approx(r["fetch_bytes"] + r["write_bytes"])


def test_percentile_helper():
    v = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.pct(v, 0.5) == 3.0
    assert bench.pct(v, 0.99) == 5.0
    assert bench.pct(v, 0.0) == 1.0
