"""Host-side logic of bench.py (no GPU): the kernel-source hash that ties the
committed HBM counters to the sources they were taken from, the counters'
use, the per-stage pass times, and the refusal of more than one GPU."""
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


def test_stage_times_are_per_stage_not_per_interval():
    # two steps (six stages); A2 timed in 4 intervals per step, as around the
    # Courant dt kernel in the first stage, one of them empty
    prof = {"A1": (12.0, 6), "A2": (4.2, 8), "Q": (24.0, 6), "P": (18.0, 6),
            "F": (45.0, 6), "ghost": (0.6, 8), "reduce": (0.02, 2), "unused": (0.0, 0)}
    passes, stage = bench.stage_times(prof, 2)
    assert set(passes) == {"A1", "A2", "Q", "P", "F", "ghost", "reduce"}
    assert abs(passes["A2"][0] - 0.7) < 1e-12 and passes["A2"][1] == 8
    assert abs(passes["A1"][0] - 2.0) < 1e-12
    assert abs(stage - (12.0 + 4.2 + 24.0 + 18.0 + 45.0) / 6) < 1e-12
    # the per-pass times of the stage passes add up to the stage time
    assert abs(sum(passes[p][0] for p in bench.STAGE_PASSES) - stage) < 1e-12
