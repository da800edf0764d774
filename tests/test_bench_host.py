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
    # the implementation's algebra: forward 7K + 3, data term 3, adjoint 8K + 7
    assert bench.MIN_VALU_PER_PAIR == (7 * K + 3) + 3 + (8 * K + 7)
    assert bench.B0_VALU_PER_PAIR == 5
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


def test_tuned_report_lists_bucket_choices_and_best_trial_times():
    import bench
    tuned = dict(launch=dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1), ms=7.5, cached=False,
                 trials=[dict(launch="a", ms=7.8), dict(launch="b", ms=9.0)],
                 buckets=[dict(n_meas=288, K=3, mode="mse", learn_diffusivity=False, vox_per_lane=1, n_split=1,
                               item_vox=512)],
                 bucket_trials=[dict(bucket="N288_K3_mse_fixedD", shape=dict(n_split=1, item_vox=512), ms=7.5),
                                dict(bucket="N288_K3_mse_fixedD", shape=dict(n_split=2, item_vox=256), ms=7.9),
                                dict(bucket="N33_K1_nll_fixedD", shape=dict(n_split=4, item_vox=64), ms=7.8)])
    r = bench.tuned_report(tuned)
    assert r["best_problem_wide_ms"] == 7.8 and r["ms"] == 7.5
    assert r["bucket_overrides"] == tuned["buckets"]
    b = r["bucket_search"]["N288_K3_mse_fixedD"]
    assert b["trials"] == 2 and b["best_ms"] == 7.5 and b["best_shape"] == dict(n_split=1, item_vox=512)
    assert r["bucket_search"]["N33_K1_nll_fixedD"]["trials"] == 1
