"""Host-side checks of the benchmark contract (no GPU): the single-GPU guard
and the rule that counter traffic is reported only for unchanged sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_unchanged_sources(tmp_path):
    """A stored traffic line counts only while every library source and
    workload generator is byte-for-byte the one it was measured on: a change
    to a kernel, to host code that lays out the data, or to a workload's mesh
    recipe each void it."""
    sys.path.insert(0, ROOT)
    import bench
    csrc = tmp_path / "paper_2301_02387_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "synth").mkdir()
    (csrc / "stencil.hip").write_text("kernel v1\n")
    (csrc / "host_mesh.cpp").write_text("numbering v1\n")
    (tmp_path / "synth" / "inputs.py").write_text("mesh recipe v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()

    def store():
        sha = bench.sources_sha1(str(tmp_path))
        (prof / "x.md").write_text("text\ntraffic: kernel=poisson_spmv workload=w1 schedule=53/8192 "
                                   f"bytes_per_launch=1234 sources_sha1={sha}\n")

    def traffic(kernel="poisson_spmv", workload="w1", schedule=None):
        return bench.measured_traffic(kernel, workload, str(prof), str(tmp_path), schedule)

    store()
    assert traffic() == 1234.0
    assert traffic(schedule="53/8192") == 1234.0
    assert traffic(schedule="52/8192") is None
    assert traffic(workload="w2") is None
    assert traffic(kernel="stencil_orb") is None
    for f, text in [(csrc / "stencil.hip", "kernel v2\n"), (csrc / "host_mesh.cpp", "numbering v2\n"),
                    (tmp_path / "synth" / "inputs.py", "mesh recipe v2\n")]:
        store()
        assert traffic() == 1234.0
        f.write_text(text)
        assert traffic() is None, f
    store()
    (csrc / "api.hip").write_text("a new source file\n")
    assert traffic() is None



def test_vector_potential_is_minus_the_field_integral():
    """The velocity-gauge field values of the triangular pulse: A(t) equals
    minus the running integral of E(t) (trapezoid rule on a fine grid), starts
    and ends at zero."""
    import numpy as np
    from scipy.integrate import cumulative_trapezoid
    from synth import vector_potential_triangular, pulse_triangular, OMEGA_400NM, E0_8E14
    T = 4 * np.pi / OMEGA_400NM
    t = np.linspace(-1.0, 1.1 * T, 200001)
    ref = -cumulative_trapezoid(pulse_triangular(t, E0_8E14), t, initial=0.0)
    A = vector_potential_triangular(t, E0_8E14)
    assert np.abs(A - ref).max() < 1e-8 * np.abs(ref).max()
    assert A[0] == 0.0 and abs(A[-1]) < 1e-12
