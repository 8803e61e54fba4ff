"""Host-side checks of bench.py (no GPU): the single-GPU rule and the HBM
traffic field, which is reported only while the DTW kernel's sources are the
ones its counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_reported_for_the_measured_sources():
    traffic, src = bench.measured_traffic()
    assert traffic is not None and traffic > 0, src
    assert src == bench.source_digest()


def test_traffic_dropped_when_the_sources_change(monkeypatch):
    # a digest over other files stands for kernel sources edited after the counters were taken
    monkeypatch.setattr(bench, "DTW_KERNEL_SOURCES", ("bounds.hip",))
    real = bench.source_digest
    monkeypatch.setattr(bench, "source_digest", lambda names=("bounds.hip",): real(names))
    traffic, reason = bench.measured_traffic()
    assert traffic is None
    assert "changed" in reason
