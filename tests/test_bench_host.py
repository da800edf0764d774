"""Host-side checks of bench.py: the multi-GPU refusal, the stored HBM-traffic
lookup (tied to the kernel sources' hash) and the roofline's per-unit figures."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single-GPU" in r.stderr


def test_roofline_unit_figures():
    K, N, P = 3, 288, 17
    # the fixed count of the method's steps: forward 10K + 8, adjoint 12K + 10
    assert bench.ALG_VALU_PER_PAIR == (10 * K + 8) + (12 * K + 10)
    # the implementation's algebra: forward 9K + 5, data term 2, adjoint 10K + 8
    assert bench.MIN_VALU_PER_PAIR == (9 * K + 5) + 2 + (10 * K + 8)
    assert bench.ALG_EXP_PER_PAIR == 2 * K
    # y, theta read, Adam moments read, theta and moments written
    assert (bench.N_MEAS, bench.P_VOX) == (N, P)
    assert bench.ALG_BYTES_PER_VOXEL == 4 * N + 4 * P + 8 * P + 12 * P
    assert bench.PEAK_SLOTS == pytest.approx(256 * 4 * 16 * 2.4e9)


def test_stored_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    from paper_2604_00250_amd import profile_summary as ps
    t = bench.stored_traffic("brain145x174x145_n288_k3_mse")
    if t is not None:            # the committed profile matches these sources
        assert 5e8 < t < 5e9
    assert bench.stored_traffic("no_such_workload") is None
    # a different source hash voids the stored figure
    monkeypatch.setattr(ps, "kernel_source_hash", lambda root=None: "000000000000")
    assert bench.stored_traffic("brain145x174x145_n288_k3_mse") is None
