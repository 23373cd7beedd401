"""Host-side checks of the benchmark contract (no GPU): the single-GPU guard
and the rule that counter traffic is reported only for an unchanged kernel."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_unchanged_source(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "kernel.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha1(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.md").write_text("text\ntraffic: kernel=poisson_spmv workload=w1 bytes_per_launch=1234 "
                               f"source_sha1={sha}\n")
    assert bench.measured_traffic("poisson_spmv", "w1", str(prof), str(src)) == 1234.0
    assert bench.measured_traffic("poisson_spmv", "w2", str(prof), str(src)) is None
    assert bench.measured_traffic("stencil_orb", "w1", str(prof), str(src)) is None
    src.write_text("kernel v2\n")
    assert bench.measured_traffic("poisson_spmv", "w1", str(prof), str(src)) is None
