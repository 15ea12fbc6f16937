"""Host-side bookkeeping of the benchmark: recorded counter summaries are
used only while the kernel sources they were taken with are unchanged
(comments and blank lines aside), and the multi-GPU request is refused."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_digest_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    a.write_text("int x = 1;  // one\n\n// note\nint y = 2;\n")
    b = tmp_path / "b.hip"
    b.write_text("int x = 1;\n// other note\nint y = 2;   \n\n")
    c = tmp_path / "c.hip"
    c.write_text("int x = 1;\nint y = 3;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_digest(["a.hip"]) == bench.source_digest(["b.hip"])
    assert bench.source_digest(["a.hip"]) != bench.source_digest(["c.hip"])


def test_recorded_figure_needs_matching_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int k;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d = {"sources": ["k.hip"], "source_sha256": bench.source_digest(["k.hip"]), "x": 42.0}
    md = tmp_path / "p.md"
    md.write_text("text\n```json\n" + json.dumps(d) + "\n```\n")
    assert bench.recorded(str(md), "x") == 42.0
    src.write_text("int k2;\n")
    assert bench.recorded(str(md), "x") is None
    assert bench.recorded(str(tmp_path / "missing.md"), "x") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
