"""Host-side checks of bench.py's contract (no GPU needed)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counted_traffic_is_reported_only_for_the_measured_source(monkeypatch):
    for name, rec in bench.COUNTED_TRAFFIC.items():
        with open(os.path.join(ROOT, rec["file"]), "rb") as f:
            current = hashlib.sha256(f.read()).hexdigest()
        assert bench.counted_traffic(name) == (rec["bytes"] if current == rec["sha256"] else None)
        # a stale record (another source hash) reports null, never an old figure
        monkeypatch.setitem(bench.COUNTED_TRAFFIC, name, dict(rec, sha256="0" * 64))
        assert bench.counted_traffic(name) is None
    assert bench.counted_traffic("no such kernel") is None


def test_defaults_finish_within_minutes(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.size == 4096
    assert 1 <= a.steps <= 10 and 0 <= a.warmup <= 5
    assert a.precision_reps <= 10
