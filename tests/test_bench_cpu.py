"""The bench's host-side contract (no GPU): it refuses more than one GPU with
a message, and it reports HBM traffic only from counters taken on the
current Gauss-point kernel source."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_from_counters_on_the_current_source(tmp_path, monkeypatch):
    digest = bench.source_digest(bench.GP_SOURCES)
    rec = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic() is None  # no record
    rec.write_text("{not json")
    assert bench.measured_traffic() is None
    rec.write_text(json.dumps({"source_digest": digest, "bytes_per_launch": 123.0}))
    assert bench.measured_traffic() == 123.0
    rec.write_text(json.dumps({"source_digest": "0" * 16, "bytes_per_launch": 123.0}))
    assert bench.measured_traffic() is None


def test_source_digest_follows_every_kernel_source(tmp_path, monkeypatch):
    files = []
    for i in range(2):
        p = tmp_path / f"k{i}.hip"
        p.write_text(f"// source {i}\nint k{i}(int a) {{ return a + {i}; }}\n")
        files.append(str(p))
    d0 = bench.source_digest(files)
    assert d0 == bench.source_digest(files)
    # comments and blank lines do not change the code the counters were taken on
    with open(files[0], "a") as f:
        f.write("\n// a remark\n/* a block\n   remark */\n\n")
    assert bench.source_digest(files) == d0
    with open(files[1], "a") as f:
        f.write("int x;\n")
    assert bench.source_digest(files) != d0
