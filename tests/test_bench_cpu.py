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


def test_live_tree_counts_match_the_oracles_compressed_tree():
    """The compressed-tree counts that credit only live work in the bench equal
    the live laminates and leaves of the oracle's compressed model, and with
    no dead leaf the live flop count is the full tree's."""
    import numpy as np
    import synthetic as S
    from oracle.compression import CompressedDmnModel
    from paper_2103_08253_amd import roofline as R
    for K in (1, 3, 5, 8):
        net = S.random_dmn(S.streams(5)["dmn"], K, 0.25)
        w = net.w.copy()
        rng = np.random.default_rng(K)
        if K > 1:
            w[rng.choice(len(w), len(w) // 3, replace=False)] = 0.0
        if K >= 3:
            w[0:4] = 0.0
        m = CompressedDmnModel(K, w, net.normals, S.FIBER, S.MATRIX)
        live_mat = sum(1 for j in m.live_leaves if j % 2 == 1)
        live_fib = sum(1 for j in m.live_leaves if j % 2 == 0)
        assert R.live_tree_counts(w) == (len(m.live_lams), live_mat, live_fib), K
        L, M = 2 ** K - 1, 2 ** (K - 1)
        assert R.live_tree_counts(net.w) == (L, M, M)
        assert R.gp_update_flops_live(L, M, M, 3) == R.gp_update_flops(K, 3)
