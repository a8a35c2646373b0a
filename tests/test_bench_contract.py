"""Host-side checks of bench.py's output contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    recorded = dict(bench.MEASURED_TRAFFIC)
    # the recorded bytes of every form are per launch and well above the compulsory W bytes
    for form in ("fp32", "bf16x3", "bf16"):
        assert recorded["bytes"][form] > 2e6
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", dict(recorded, sources_sha256="0" * 64))
    assert bench.measured_traffic("bf16") is None


def test_cpu_baseline_fields_on_a_small_sample():
    from paper_2411_03289_amd import workloads as W
    pr = W.make_config(2)
    summary, tr = bench.cpu_baseline(pr, 2)
    assert summary["kind"] == "oracle"
    assert summary["unit"] == "sample-steps/s"
    assert summary["value"] > 0 and summary["cores"] >= 1
    assert "K=16384" in summary["sample"] and "T=100" in summary["sample"]
    assert tr.x.shape[1] == 2
