"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the
algorithmic byte and flop counts the roofline divides by, and the rule that
measured HBM traffic is reported only for the kernel sources it was taken on.
"""
import importlib.util
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no bench line


def test_algorithmic_bytes_and_flops(bench):
    """Per position: delta and beta read in both sweeps and their gradients
    written (24 B per voxel), the measured intensity read (4 B per pixel),
    a complex64 checkpoint written and read every C slices (16 B per pixel)."""
    n, s = 128, 64
    voxels = n * n * s
    expect = 2 * 8 * voxels + 8 * voxels + 4 * n * n + 16 * n * n * math.ceil(s / 16)
    assert bench.algorithmic_bytes_per_position(n, s) == expect == 26_279_936
    assert bench.algorithmic_bytes_per_position(n, s, 1) - bench.algorithmic_bytes_per_position(n, s) \
        == 16 * n * n * (64 - 4)
    # 6 S 2D FFT-equivalents of 5 N^2 log2 N^2 flops plus 60 flops per voxel
    assert bench.algorithmic_flops_per_position(n, s) == pytest.approx(6 * s * 5 * n * n * 14 + 60 * voxels)


def test_traffic_is_reported_only_for_the_measured_sources(bench, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "multislice_n128_s64_b50_traffic.json")))
    assert {"csrc_sha256", "read_bytes", "write_bytes"} <= set(rec)
    assert len(bench.kernel_source_hash()) == 64
    # sources as measured: the recorded read + write bytes
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["csrc_sha256"])
    assert bench.measured_traffic() == rec["read_bytes"] + rec["write_bytes"]
    # any other sources: no traffic figure
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic() is None


def test_copy_peak_is_added_only_to_hbm_rooflines(bench, monkeypatch):
    monkeypatch.setattr(bench, "measured_copy_gbs", lambda reps=10: 5000.0)
    line = {"roofline": {"unit": "GB/s", "achieved": 1000.0}}
    out = bench.with_copy_peak(line)
    assert out["roofline"]["measured_copy_GBps"] == 5000.0
    assert out["roofline"]["frac_of_measured_copy"] == pytest.approx(0.2)
    assert bench.with_copy_peak({"value": 1.0}) == {"value": 1.0}
