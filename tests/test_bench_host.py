"""Host logic of bench.py (no GPU): the algorithmic-bytes model of the
tracing kernel, the two readouts gated on the hashes of the sources their
committed summaries were measured with, and the refusal of more than one
GPU."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_event():
    stats = {"collisions": 1000, "scat_gas": 10, "scat_cloud": 300, "surface": 50, "escape": 40}
    # 16 B per tentative collision, +4 B per real scattering, +4 B more per
    # cloud scattering, 20 B per surface hit, 8 B per escape
    assert bench.algorithmic_bytes(stats) == 16 * 1000 + 4 * 310 + 4 * 300 + 20 * 50 + 8 * 40


def test_committed_summaries_match_the_sources():
    """The committed profile summaries were taken on the current sources,
    so both readouts are live (this guards against committing a changed
    kernel without re-profiling)."""
    t = bench.measured_traffic((8, 8, 8), 1 << 26)
    assert t is not None and t > 1e10
    r = bench.time_to_5pct()
    assert r is not None and r["speedup"] > 1.0
    assert r["plain_time_to_5pct_s"] > r["denoised_time_to_5pct_s"] > 0.0


def test_readouts_are_gated(tmp_path, monkeypatch):
    """Another workload, or any change to a hashed source, turns the
    readouts off."""
    assert bench.measured_traffic((4, 4, 4), 1 << 26) is None
    assert bench.measured_traffic((8, 8, 8), 1 << 20) is None
    copy = tmp_path / "repo"
    for d in ("profiles", os.path.join("paper_2208_05247_amd", "csrc")):
        shutil.copytree(os.path.join(ROOT, d), copy / d)
    for f in ("denoise.py", "experiment.py"):
        shutil.copy(os.path.join(ROOT, "paper_2208_05247_amd", f), copy / "paper_2208_05247_amd" / f)
    monkeypatch.setattr(bench, "ROOT", str(copy))
    assert bench.measured_traffic((8, 8, 8), 1 << 26) is not None
    assert bench.time_to_5pct() is not None
    src = copy / "paper_2208_05247_amd" / "csrc" / "rt3d.hip"
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.measured_traffic((8, 8, 8), 1 << 26) is None
    assert bench.time_to_5pct() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
