"""Host-side parts of bench.py's output contract (no GPU needed)."""
import argparse
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_source_digest_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("int f(int x) {\n  return x + 1;\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    d0 = bench.kernel_source_digest()
    src.write_text("// note\nint f(int x) {   /* block\n comment */\n\n  return x + 1;  // why\n}\n")
    assert bench.kernel_source_digest() == d0
    src.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_source_digest() != d0


def test_traffic_record_is_used_only_for_matching_sources(tmp_path):
    args = argparse.Namespace(traffic_kib=None, split="pow2")
    rec = {"kernel_sources_sha256": bench.kernel_source_digest(), "split": "pow2",
           "fetch_kib_scaled": 1000.0, "write_kib_scaled": 24.0}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    assert bench._traffic_bytes(args, path=str(f), split="pow2") == 1024.0 * 1024.0
    assert bench._traffic_bytes(args, path=str(f), split="radix") is None   # another hierarchy
    assert bench._traffic_bytes(args, path=str(f)) == 1024.0 * 1024.0       # not keyed (range min)
    del rec["split"]
    f.write_text(json.dumps(rec))
    assert bench._traffic_bytes(args, path=str(f), split="pow2") is None    # unkeyed = radix
    rec["kernel_sources_sha256"] = "0" * 64
    f.write_text(json.dumps(rec))
    assert bench._traffic_bytes(args, path=str(f)) is None
    assert bench._traffic_bytes(args, path=str(tmp_path / "missing.json")) is None
    over = argparse.Namespace(traffic_kib=[3.0, 1.0], split="radix")
    assert bench._traffic_bytes(over, path=str(f)) == 4096.0
