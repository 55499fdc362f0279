"""Host logic of bench.py (no GPU): the kernel-source hash that ties the
committed counter record to the source it was taken on, the record's parsing,
the serial-queue model of the served comparison, and the one-GPU guard."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    src = open(bench.KERNEL_SRC).read()
    h0 = bench.kernel_hash()
    edited = tmp_path / "k.hip"
    edited.write_text("// a new comment line\n" + src.replace("\n", "\n  ", 5) + "\n/* block\n comment */\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(edited))
    assert bench.kernel_hash() == h0
    edited.write_text(src.replace("kWave = 64", "kWave = 32", 1))
    assert bench.kernel_hash() != h0


def test_traffic_record_parses_and_is_tied_to_the_source(tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_FILE).read()
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    cal = rec["calibration"]
    assert cal["read_factor"] > 0 and cal["write_factor"] > 0
    for name in ("k_plain_x", "k_combine", "k_bricks", "k_pom_x", "k_dist_lines<false>",
                 "k_dist_lines<true>"):
        k = rec["kernels"][name]
        assert k["hbm_bytes_per_launch"] > 0 and k["launches"] >= 1
    # a record is used only for the source it was taken on
    other = tmp_path / "k.hip"
    other.write_text(open(bench.KERNEL_SRC).read() + "\nint unrelated_symbol;\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(other))
    assert bench.load_traffic() is None


def test_serial_queue_latencies():
    class R:
        def __init__(self, arrival, vol_id):
            self.arrival, self.vol_id = arrival, vol_id

    # two requests 0.5 s apart on a server taking 1 s each: the second waits
    out = bench.serial_queue([R(0.0, 0), R(0.5, 0)], {0: 1.0})
    assert out["p50_ms"] == pytest.approx(1250.0)
    assert out["updates_per_s"] == pytest.approx(1.0)
    # spaced out beyond the service time: no waiting
    out = bench.serial_queue([R(0.0, 0), R(2.0, 1), R(4.0, 0)], {0: 0.1, 1: 0.2})
    assert out["p50_ms"] == pytest.approx(100.0) and out["p99_ms"] == pytest.approx(198.0)


def test_pct_of_nothing_is_nan():
    assert math.isnan(bench.pct([], 50))
    assert bench.pct([1.0, 2.0, 3.0], 50) == 2.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
