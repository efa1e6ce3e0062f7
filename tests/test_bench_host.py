"""Host-side contract of bench.py (no GPU needed): more than one GPU is
refused with a message and exit status 2, and the workload table names every
configuration the --config option accepts."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_workload_names(cfg):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1508_04596_amd import inputs
    text = bench.WORKLOADS[cfg].format(reps=10)
    p = inputs.config(cfg) if cfg == 2 else None
    assert f"C{cfg}:" in text and "10 Jv FP64" in text
    if p is not None:
        assert f"{p.nx}x{p.ny}x{p.nz}" in text and f"{p.n_dof:,}" in text


def test_host_cpu_record():
    sys.path.insert(0, ROOT)
    import bench
    info = bench.host_cpu()
    assert info["cpus_available"] >= 1
    assert "model" in info and "physical_cores" in info and "sockets" in info


def test_traffic_guard_tracks_the_element_source():
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.elem_source_sha256()
    assert len(sha) == 64 and len(bench.ELEM_TRAFFIC_SRC_SHA256) == 64


def test_traffic_per_workload():
    """Counter-based traffic exists for the 64^3 and 160x160x320 workloads (KiB
    per dispatch scaled by the copy calibration), and is null elsewhere."""
    sys.path.insert(0, ROOT)
    import bench
    t2, t3 = bench.elem_traffic_bytes(2), bench.elem_traffic_bytes(3)
    assert t2 == pytest.approx(1024 * (14235.56 * 1.951 + 17217.22))
    assert t3 > 30 * t2  # 32,000 tiles against 1,024
    assert bench.elem_traffic_bytes(4) is None
