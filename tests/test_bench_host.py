"""Host-side parts of bench.py (no GPU): the one-GPU contract, the
comment-blind source digest that ties counter summaries to kernel code, and
the geometry check on those summaries."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for extra in ([], ["--workload", "batched2d"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"] + extra,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2 and "one GPU" in r.stderr


def test_digest_ignores_comments_and_layout(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one more\n}\n")
    b.write_text("/* doc */\nint f(int x) {\n\n    return x + 1;\n}\n")
    assert bench.src_digest([str(a)]) == bench.src_digest([str(b)])
    b.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.src_digest([str(a)]) != bench.src_digest([str(b)])


def test_counters_need_matching_source_and_geometry(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int k;\n")
    ctr = tmp_path / "c.json"
    ctr.write_text(json.dumps({"source_digest": bench.src_digest([str(src)]), "geometry": [8, 1],
                               "hbm_bytes_per_launch": 1.0}))
    wk = {"counters": str(ctr), "sources": [str(src)]}
    monkeypatch.setattr(bench, "ROOT", "/")
    assert bench.load_counters(wk, (8, 1))["hbm_bytes_per_launch"] == 1.0
    assert bench.load_counters(wk, (16, 1)) is None
    src.write_text("int k2;\n")
    assert bench.load_counters(wk, (8, 1)) is None
