"""bench.py's command-line contract that needs no GPU: it measures one GPU
and refuses more, and its kernel-source hash ignores comments but not code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_1808_01478_amd" / "csrc"
    csrc.mkdir(parents=True)
    k = csrc / "dh_kernels.hip"
    h = csrc / "dh_internal.h"
    k.write_text("int f(int x) { return x + 1; }  // one\n/* two */\n")
    h.write_text("struct S { int a; };\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_hash()
    k.write_text("int f(int x) {\n  return x + 1;  // another comment\n}\n")
    assert bench.kernel_source_hash() == base
    k.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != base
