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


def test_defaults_finish_within_minutes():
    a = bench.parse([])
    assert a.gpus == 1 and a.size == 4096
    assert 1 <= a.steps <= 10 and 0 <= a.warmup <= 5
    assert a.cpu_seconds <= 30  # the bounded CPU-oracle sample
    assert a.serve_requests == 2000


def test_headline_is_the_metric_configuration():
    # the headline compares split configurations with the plain FP64 GEMM
    names = [h[0] for h in bench.HEADLINE]
    assert "dgemm" in names and any(n.startswith("split_bf16") for n in names)
    assert any(n.startswith("split_int8") for n in names) and any(n.startswith("split_fp16") for n in names)
    assert bench.FP64_GRADE == 1e-13
    assert set(bench.SECTIONS) >= {"headline", "latency", "allmethods", "batch", "serve"}


def test_tile_tuner_split_keys(tmp_path):
    from paper_1106_1347_amd import tune
    from paper_1106_1347_amd._lib import Config

    t = tune.TileTuner(path=str(tmp_path / "t.json"))
    cfg = Config(split_type="bf16", split_slices=6)
    k = t.key((9, 8), "split", cfg)
    assert k.endswith("/split/bf16_s6/n9_p8") and k != t.key((9, 8))
    t.table[k] = "narrow"
    assert t.tile_for(300, 200, 400, "split", cfg) == tune.SPLIT_TILE_CODES["narrow"]
    assert t.tile_for(300, 200, 400, "split", Config(split_type="int8", split_slices=7)) == 0
