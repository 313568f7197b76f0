"""Host logic of bench.py (no GPU): the algorithmic-bytes model of the
tracing kernel, the traffic readout gated on the hash of the kernel source
and the workload its committed summary was measured with, and the refusal of
more than one GPU."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_event():
    stats = {"collisions": 1000, "scat_gas": 10, "scat_cloud": 300, "surface": 50, "escape": 40}
    # 16 B per tentative collision, +4 B per real scattering, +4 B more per
    # cloud scattering, 20 B per surface hit, 8 B per escape
    assert bench.algorithmic_bytes(stats) == 16 * 1000 + 4 * 310 + 4 * 300 + 20 * 50 + 8 * 40


def test_roofline_fields():
    stats = {"collisions": 2000, "scat_gas": 0, "scat_cloud": 0, "surface": 0, "escape": 0}
    r = bench.tracer_roofline(stats, 2, 1e-3, 64e3)
    # 16 kB per launch in 1 microsecond = 16 GB/s
    assert abs(r["achieved"] - 16.0) < 1e-9 and abs(r["frac"] - 16.0 / 8000.0) < 1e-12
    assert abs(r["traffic_GBps"] - 64.0) < 1e-9
    assert bench.tracer_roofline(stats, 2, 1e-3, None)["traffic"] is None


def test_traffic_readout_is_gated(tmp_path, monkeypatch):
    """The readout is live only for the kernel source hash and workload the
    summary names; any change to the source, or another workload, turns it
    off."""
    copy = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_2208_05247_amd", "csrc"), copy / "paper_2208_05247_amd" / "csrc")
    (copy / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(copy))
    sha = bench.source_hash(bench.TRACER_SOURCES)
    (copy / "profiles" / "p.md").write_text(
        "# summary\n\n    source_sha256_16: %s\n    workload: wl_a\n    traffic_bytes_per_launch: 123456789\n" % sha)
    assert bench.measured_traffic("p.md", "wl_a") == 123456789.0
    assert bench.measured_traffic("p.md", "wl_b") is None
    assert bench.measured_traffic("missing.md", "wl_a") is None
    src = copy / "paper_2208_05247_amd" / "csrc" / "rt3d.hip"
    src.write_text(src.read_text() + "\n// changed\n")
    assert bench.measured_traffic("p.md", "wl_a") is None


def test_committed_traffic_summaries_name_their_workload():
    """Every committed tracing-kernel summary states the source hash and the
    workload its figures belong to."""
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("trace_kernel_"):
            f = bench.profile_fields(name)
            assert "source_sha256_16" in f and "workload" in f, name


def test_headline_workload_key_and_cell_argument():
    """The headline summary is keyed by workload, acceleration cell and
    schedule tile, so counters taken with another cell are not reported;
    --brick takes one edge or three."""
    key = bench.headline_key((8, 8, 8), (128, 128))
    assert key == bench.HEADLINE_NAME + ", brick 8x8x8, schedule tile 128x128"
    assert bench.headline_key((4, 4, 8), (128, 128)) != key
    assert bench.parse_brick("") == bench.HEADLINE_BRICK
    assert bench.parse_brick("4") == (4, 4, 4)
    assert bench.parse_brick("4,4,8") == (4, 4, 8)
    f = bench.profile_fields("trace_kernel_batched_cumulus_1024x1024x128.md")
    assert f["workload"] == bench.headline_key(bench.HEADLINE_BRICK, bench.HEADLINE_TILE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
