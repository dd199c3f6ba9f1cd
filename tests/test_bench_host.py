"""Host logic of bench.py (no GPU): the traffic figure is taken from a
profile summary only when it was measured on the sweep kernel's source as it
stands, and more than one GPU is refused with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_only_for_the_current_sweep_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "paper_1609_07936_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "sail.hip").write_bytes(open(os.path.join(ROOT, "paper_1609_07936_amd", "csrc", "sail.hip"), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    stem = bench.WORKLOADS["fp64"]
    path = tmp_path / "profiles" / f"{stem}_traffic.md"
    assert bench.measured_traffic("fp64") is None  # no summary
    path.write_text(f"# t\n\ntraffic_bytes_per_launch: 1.5e+11\nsweep_source_sha256_16: {bench.sweep_source_digest()}\n")
    assert bench.measured_traffic("fp64") == 1.5e11
    path.write_text("# t\n\ntraffic_bytes_per_launch: 1.5e+11\nsweep_source_sha256_16: 0000000000000000\n")
    assert bench.measured_traffic("fp64") is None  # measured on another source
    assert bench.measured_traffic("served") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_matched_final_chi2_and_cpu_model():
    """Final residues count as matched when the median residues agree within
    5%; the CPU baseline names the host's CPU model."""
    assert bench.matched(1.04, 1.0) and bench.matched(0.96, 1.0)
    assert not bench.matched(1.06, 1.0) and not bench.matched(0.9, 1.0)
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_lds_figures_from_the_committed_summary():
    """roofline.lds comes from the committed LDS counter summary only while
    its source digest matches the sweep kernel as built; its fraction is the
    achieved LDS bandwidth over the probe's measured ceiling."""
    import bench
    assert bench.measured_lds("batched", 1.0) is None
    for w, ms in (("fp64", 41.0), ("fp32", 17.0)):
        r = bench.measured_lds(w, ms)
        if r is None:
            continue
        assert r["bytes_per_launch"] > 0 and r["ceiling"] > 0
        assert abs(r["achieved"] - r["bytes_per_launch"] / (ms * 1e-3) / 1e12) < 1e-9
        assert abs(r["frac"] - r["achieved"] / r["ceiling"]) < 1e-12
