"""bench.py host logic: the one-GPU contract and the algorithmic byte model (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1505_05341_amd import native  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_byte_model_matches_the_library_workspace():
    """The X and H sizes of the byte model equal the library's own buffers (the workspace
    difference between two grid sizes of the same catalogue)."""
    for N, dn, nbins in [(64, 1, 32), (128, 2, 31), (512, 2, 128)]:
        cfg = dict(N=N, box_min=(0.0, 0.0, 0.0), L=100.0, dn=dn, nbins=nbins, ell_max=4)
        b = bench.plan_bytes(cfg, 0, 10)
        X = b["fft_y"] - b["fft_z_bin"]        # X + H - H
        H = b["fft_z_bin"]
        full = native.workspace_size(cfg, 0, 10)
        nox = native.workspace_size(dict(cfg, x_planes=1), 0, 10)   # two 1-plane slots of X
        assert full - nox == X - 2 * X // N, (N, full - nox, X)
        assert H > 0 and X == 15 * N * N * (-(-nbins * dn // (16 if N <= 512 else 8)) * (16 if N <= 512 else 8)) * 8
    # slabs: the x and y transforms are timed as one stage
    s = bench.plan_bytes(dict(N=2048, box_min=(0, 0, 0), L=1.0, dn=2, nbins=512, ell_max=4), 10, 10, slabs=True)
    assert "fft_y" not in s and s["assign_x"] > s["fft_z_bin"]


def test_traffic_is_reported_only_for_the_workload_it_was_measured_on():
    """The calibrated HBM traffic in the bench line belongs to one (workload, kernel) pair:
    another workload with the same dominant kernel reports null, not that figure."""
    keys = list(bench.TRAFFIC)
    assert keys and all(isinstance(k, tuple) and len(k) == 2 for k in keys)
    for workload, kernel in keys:
        t = bench.TRAFFIC[(workload, kernel)]
        got = bench.measured_traffic(workload, kernel)
        if got is not None:  # sources unchanged since the counters were taken
            assert got == 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])
        for other in ("desi_1024", "survey", "tiny_32", "clustered_512"):
            if (other, kernel) not in bench.TRAFFIC:
                assert bench.measured_traffic(other, kernel) is None
