"""Host-side checks of bench.py's contract (no GPU needed)."""

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_range_flops_convention():
    b = _bench()
    # per Doppler row: forward DFT_N of N_cp taps 5 N log2 N_cp, window 2 N,
    # inverse N'-point DFT of N values 5 N' log2 N, |.|^2 3 N'
    n, ncp, pad, m = 1024, 256, 4, 1024
    per_row = 5 * n * 8 + 2 * n + 5 * pad * n * 10 + 3 * pad * n
    assert per_row == 260096
    assert b.k3_flops_per_frame() == pad * m * per_row
    assert b.k3_flops_per_frame(256, 64, 4, 32) == 4 * 64 * (5 * 256 * 5 + 2 * 256 + 5 * 1024 * 8 + 3 * 1024)


def test_traffic_only_for_the_measured_sources(monkeypatch):
    b = _bench()
    with open(os.path.join(ROOT, "profiles", "k3_range_power_full_frame_traffic.json")) as fh:
        rec = json.load(fh)
    if rec["source_hash"] != b.kernel_source_hash():
        # counters taken on other kernel sources are not reported
        assert b.measured_traffic(128) is None
        return
    per_frame = rec["hbm_bytes_per_launch"] / rec["frames_per_launch"]
    assert b.measured_traffic(128) == pytest.approx(128 * per_frame)
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 16)
    assert b.measured_traffic(128) is None
