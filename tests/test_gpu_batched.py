"""The batched workload: many independent patches of uneven size with mixed
acquisitions (N = 33 / 96 / 288), K = 1..5 and MSE / NLL in one problem.
Parity of every group against the FP64 oracle, bitwise equality of the
per-variant and the persistent launch plans, and the autotuner."""
import numpy as np
import pytest

from paper_2604_00250_amd import inputs as I

from gpu_helpers import assert_parity, merged_grad, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def _workload(n=96, edges=(2, 12)):
    w = I.batched_patches(n_patches=n, edge_range=edges)
    for g in w.groups:  # a generic parameter point, not the symmetric init
        g.theta = I.perturb_theta(g.theta, np.random.default_rng(g.n_vox), scale=0.5)
    return w


@pytest.mark.parametrize("launch", [dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1),
                                    dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=0),
                                    dict(vox_per_lane=2, n_split=1, item_vox=512, persistent=0)])
def test_batched_groups_match_oracle(launch):
    w = _workload()
    r = run_gpu(w.groups, [g.theta for g in w.groups], launch=launch)
    assert r["status"] == 0
    say(f"[batched] {launch} groups={len(w.groups)} voxels={w.n_vox}")
    for i, g in enumerate(w.groups):
        out, grad, _ = run_oracle(g, g.theta)
        assert_parity(f"batched/{i} K={g.K} N={g.acq.n} {g.mode}", r["loss"][i],
                      merged_grad(r["gmicro"][i], r["gcal"][i]), out, grad)


def test_persistent_and_per_variant_plans_agree_bitwise():
    w = _workload(n=160, edges=(3, 16))
    a = run_gpu(w.groups, [g.theta for g in w.groups], launch=dict(vox_per_lane=1, n_split=0, persistent=1))
    b = run_gpu(w.groups, [g.theta for g in w.groups], launch=dict(vox_per_lane=1, n_split=0, persistent=0))
    assert np.array_equal(a["loss"], b["loss"])
    for x, y in zip(a["gmicro"], b["gmicro"]):
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    for x, y in zip(a["gcal"], b["gcal"]):
        for k in x:
            assert np.array_equal(x[k], y[k]), k


def test_autotuner_picks_a_valid_plan_and_caches_it(tmp_path):
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    from paper_2604_00250_amd.tune import autotune
    w = _workload(n=128, edges=(3, 14))
    prob = Problem(w.groups)
    st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups])
    st.loss_grad()
    torch.cuda.synchronize()
    ref = st.loss_host().copy()
    cache = str(tmp_path / "tune.json")
    res = autotune(st, cache=cache, reps=3)
    say(f"[tune] best {res['launch']} {res['ms']:.4f} ms; trials {[(t['launch'], round(t['ms'], 4)) for t in res['trials']]}")
    assert not res["cached"] and len(res["trials"]) >= 5
    st.loss_grad()
    torch.cuda.synchronize()
    assert np.allclose(st.loss_host(), ref, rtol=1e-6, atol=0)
    res2 = autotune(st, cache=cache)
    assert res2["cached"] and res2["launch"] == res["launch"]
