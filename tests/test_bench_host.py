"""Host-side checks of bench.py (no GPU): the one-GPU guard, the flop count
of the roofline, and the committed-traffic lookup that nulls the traffic
figure once the contraction's sources differ from the profiled ones."""
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


def test_flops_per_sample_of_the_benchmark_point():
    # 4 flop per (detector, mode) and bin, 16 n_det n_lm^2 per sample
    assert bench.flops_per_sample(3, 21, 1601) == 4 * 3 * 21 * 1601 + 16 * 3 * 21 * 21
    assert bench.flops_per_sample(3, 21, 1601) == 424620


def test_traffic_lookup_needs_matching_sources(monkeypatch, tmp_path):
    assert bench.committed_traffic("fp64", "phased", 999) is None
    assert bench.committed_traffic("bf16", "pipelined", 128) is None
    # a record is found only for its own sources, precision, engine and shape
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.md").write_text("traffic-record: source_sha256=abc precision=fp64 "
                               "engine=phased threads=512 bytes=123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.committed_traffic("fp64", "phased", 512) == 123
    assert bench.committed_traffic("fp64", "pipelined", 512) is None
    assert bench.committed_traffic("fp32", "phased", 512) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.committed_traffic("fp64", "phased", 512) is None


def test_profiles_hold_text_only():
    d = os.path.join(ROOT, "profiles")
    for f in os.listdir(d):
        assert f.endswith((".md", ".txt")), f
        assert os.path.getsize(os.path.join(d, f)) < 64 * 1024
