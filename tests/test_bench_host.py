"""Host-side logic of bench.py (no GPU): the kernel-source hash that ties the
committed HBM counters to the sources they were taken from, the counters'
use, and the refusal of more than one GPU."""
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _copy_sources(tmp_path):
    dst = tmp_path / "paper_2405_02483_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_2405_02483_amd", "csrc"), dst,
                    ignore=shutil.ignore_patterns("__pycache__", "*.o", "*.so", "_build"))
    return dst


def test_source_hash_ignores_comments_but_not_code(tmp_path):
    dst = _copy_sources(tmp_path)
    base = bench.kernel_source_hash(str(tmp_path))
    assert base == bench.kernel_source_hash(ROOT)
    src = dst / "mhd_zmarch.hip"
    text = src.read_text()
    src.write_text(text + "\n// a note\n\n")
    assert bench.kernel_source_hash(str(tmp_path)) == base
    src.write_text(text + "\nstatic int unused_probe_value = 1;\n")
    assert bench.kernel_source_hash(str(tmp_path)) != base
    # the adjoint's own sources do not take part
    src.write_text(text)
    adj = dst / "mhd_adjoint.hip"
    adj.write_text(adj.read_text() + "\nstatic int another_value = 2;\n")
    assert bench.kernel_source_hash(str(tmp_path)) == base
    # nor do the div B cleaning's (not part of the stage)
    cln = dst / "mhd_clean.hip"
    cln.write_text(cln.read_text() + "\nstatic int a_third_value = 3;\n")
    assert bench.kernel_source_hash(str(tmp_path)) == base


def test_counters_are_dropped_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda root=None: "0" * 16)
    assert bench.measured_traffic("f32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
