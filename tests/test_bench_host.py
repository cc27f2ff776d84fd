"""Host logic of bench.py that needs no GPU: the HBM traffic record of the
dominant kernel (read from the committed counter summary, valid only while
the kernel source is the one the counters were taken on) and the refusal of
more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# 4 fields of 127^3 interior points, 24 bytes each (read u and b, write u)
SWEEP_ALGO_BYTES = 24 * 4 * 127 ** 3


def test_traffic_record_matches_the_kernel_source():
    rec = bench.measured_traffic()
    assert rec is not None, "the counter record does not match rbgs_fused.hip: take the counters again"
    assert rec["algorithmic_bytes_per_launch"] == SWEEP_ALGO_BYTES
    assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    # the output is written once: the write counter cannot fall below the
    # bytes of u'; and every input byte is read at least once
    assert rec["write_bytes_per_launch"] >= 8 * 4 * 127 ** 3
    assert rec["fetch_bytes_per_launch"] >= 16 * 4 * 127 ** 3


def test_traffic_record_is_dropped_when_the_source_changes(tmp_path, monkeypatch):
    src = tmp_path / "rbgs_fused.hip"
    with open(bench.KERNEL_SOURCE, "rb") as f:
        src.write_bytes(f.read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    assert bench.measured_traffic() is None


def test_traffic_record_missing_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None


def test_traffic_record_takes_the_last_line(tmp_path, monkeypatch):
    rec = bench.measured_traffic()
    assert rec is not None
    older = dict(rec, hbm_bytes_per_launch=1)
    p = tmp_path / "traffic.md"
    p.write_text("text\nbench-traffic: " + json.dumps(older) + "\nmore text\nbench-traffic: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic() == rec


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
