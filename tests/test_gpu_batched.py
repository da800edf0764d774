"""The batched workload: many independent patches of uneven size with mixed
acquisitions (N = 33 / 96 / 288), K = 1..5 and MSE / NLL in one problem.
Parity of every group against the FP64 oracle in several launch plans
(per-variant, persistent, persistent with several items per block, per-bucket
shapes), bitwise equality of the per-variant and the persistent plans, the
autotuner, and the full 4096-patch problem in its autotuned persistent plan
against the oracle on a seeded sample of whole groups."""
import multiprocessing as mp
import os

import numpy as np
import pytest

from paper_2604_00250_amd import inputs as I

from gpu_helpers import assert_parity, merged_grad, oracle_group, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def _workload(n=96, edges=(2, 12)):
    w = I.batched_patches(n_patches=n, edge_range=edges)
    for g in w.groups:  # a generic parameter point, not the symmetric init
        g.theta = I.perturb_theta(g.theta, np.random.default_rng(g.n_vox), scale=0.5)
    return w


def _all_groups_match(w, r, label):
    assert r["status"] == 0
    for i, g in enumerate(w.groups):
        out, grad, _ = run_oracle(g, g.theta)
        assert_parity(f"{label}/{i} K={g.K} N={g.acq.n} {g.mode}", r["loss"][i],
                      merged_grad(r["gmicro"][i], r["gcal"][i]), out, grad)


@pytest.mark.parametrize("launch", [dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1),
                                    dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=0),
                                    dict(vox_per_lane=2, n_split=1, item_vox=512, persistent=0)])
def test_batched_groups_match_oracle(launch):
    w = _workload()
    r = run_gpu(w.groups, [g.theta for g in w.groups], launch=launch)
    say(f"[batched] {launch} groups={len(w.groups)} voxels={w.n_vox} plan {r['prob'].plan_info()}")
    _all_groups_match(w, r, "batched")


def test_concurrent_variant_launches_are_bitwise_the_serial_ones():
    """A per-variant plan with several variants runs them on up to four
    streams (forked from and joined back into the caller's); each item writes
    its own record and the reductions follow the join, so the results equal
    those of the same plan launched one variant after another, bit for bit,
    and stay so over several fused Adam iterations."""
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    w = _workload()
    shape = dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=0)
    states = []
    for conc in (1, 0):
        prob = Problem(w.groups, launch=dict(shape, concurrent=conc))
        st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups])
        for _ in range(3):
            st.iteration(1e-2)
        st.loss_grad()
        torch.cuda.synchronize()
        states.append(st)
        say(f"[concurrent={conc}] launch {prob.launch()} plan {prob.plan_info()} buckets {len(prob.buckets())}")
    a, b = states
    assert a.prob.plan_info()["launches"] >= 4
    for k in ("params", "m", "v", "grad", "loss", "step", "status"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def test_persistent_blocks_run_several_items_each():
    """max_blocks caps the persistent grid far below the item count, so every
    block pops and runs many items in turn (LDS reuse across items of different
    variants, the counter loop's exit)."""
    w = _workload()
    r = run_gpu(w.groups, [g.theta for g in w.groups],
                launch=dict(vox_per_lane=1, n_split=0, item_vox=64, persistent=1, max_blocks=8))
    info = r["prob"].plan_info()
    ratio = info["items"] / info["persistent_blocks"]
    say(f"[persistent x several] plan {info}: {ratio:.1f} items per block")
    assert info["persistent_blocks"] == 8 and ratio >= 10
    _all_groups_match(w, r, "persistent-8-blocks")


def _mixed_buckets(w, persistent):
    """Per-bucket shapes that differ from the problem-wide one."""
    out = []
    seen = set()
    for g in w.groups:
        key = (g.acq.n, g.K, g.mode, bool(g.learn_diffusivity))
        if key in seen:
            continue
        seen.add(key)
        if g.acq.n == 288:
            shape = dict(vox_per_lane=1 if persistent else 2, n_split=1, item_vox=512 if persistent else 1024)
        elif g.acq.n == 96:
            shape = dict(vox_per_lane=1, n_split=2, item_vox=256)
        else:
            shape = dict(vox_per_lane=1, n_split=4, item_vox=64)
        out.append(dict(n_meas=g.acq.n, K=g.K, mode=g.mode, learn_diffusivity=g.learn_diffusivity, **shape))
    return out


@pytest.mark.parametrize("persistent", [0, 1])
def test_per_bucket_shapes_match_oracle(persistent):
    from paper_2604_00250_amd.problem import DeviceState, Problem
    import torch
    w = _workload()
    prob = Problem(w.groups)
    prob.tune(vox_per_lane=1, n_split=0, item_vox=0, persistent=persistent, buckets=_mixed_buckets(w, persistent))
    got = {(b["n_meas"], b["K"], b["mode"]): (b["vox_per_lane"], b["n_split"], b["item_vox"]) for b in prob.buckets()}
    say(f"[per-bucket persistent={persistent}] plan {prob.plan_info()} shapes {sorted(got.items())[:4]} ...")
    assert all(v[2] > 0 for v in got.values())
    st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups])
    st.loss_grad()
    torch.cuda.synchronize()
    gm, gc = st.grads_host()
    r = dict(loss=st.loss_host(), gmicro=gm, gcal=gc, status=int(st.status.item()))
    _all_groups_match(w, r, f"per-bucket-{persistent}")


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


def test_autotuner_picks_valid_shapes_per_bucket_and_caches_them(tmp_path):
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    from paper_2604_00250_amd.tune import autotune
    w = _workload(n=128, edges=(3, 14))
    prob = Problem(w.groups)
    st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups])
    st.loss_grad()
    torch.cuda.synchronize()
    ref = st.loss_host().copy()
    p0 = st.params.clone()
    cache = str(tmp_path / "tune.json")
    res = autotune(st, cache=cache, reps=3)
    say(f"[tune] best {res['launch']} {res['ms']:.4f} ms; {len(res['buckets'])} bucket shapes; "
        f"trials {[(t['launch'], round(t['ms'], 4)) for t in res['trials']]}")
    assert not res["cached"] and len(res["trials"]) >= 5 and len(res["bucket_trials"]) > 0
    # the tuner leaves the parameters as they were and the new plan computes the same loss
    assert torch.equal(st.params, p0) and int(st.step[0].item()) == 0
    st.loss_grad()
    torch.cuda.synchronize()
    # a different plan sums the same terms in a different order: equal to rounding
    # of the summed parts.  An NLL data term is a float32-summed positive part plus
    # the constant 2 sigma_log N |M|, which nearly cancel on some small patches, so
    # the tolerance scales with the parts, not with their sum.
    got = st.loss_host()
    scale = np.abs(ref).copy()
    for i, g in enumerate(w.groups):
        if g.mode == "nll":
            c = abs(2.0 * float(g.theta["sigma_log"]) * g.acq.n * g.n_vox)
            scale[i, 0] += c
            scale[i, 9] += c
    rel = np.abs(got - ref) / np.maximum(scale, 1e-30)
    worst = np.unravel_index(np.argmax(rel), rel.shape)
    say(f"[tune] loss after re-planning: worst relative change {rel.max():.2e} at group {worst[0]} term {worst[1]}")
    assert rel.max() <= 1e-6
    res2 = autotune(st, cache=cache)
    assert res2["cached"] and res2["launch"] == res["launch"]
    key = lambda b: (b["n_meas"], b["K"], b["mode"])  # noqa: E731
    assert sorted(map(key, res2["buckets"])) == sorted(map(key, res["buckets"]))


def _pool_size(limit=16):
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(limit, cores))


@pytest.mark.timeout(900)
def test_full_batched_problem_in_its_tuned_persistent_plan():
    """4096 patches (10.5M voxels) in one persistent launch with autotuned
    per-bucket shapes; whole groups compared with the oracle: one seeded pick
    from every (N, K, mode) bucket, the largest patch, and seeded others up
    to 64 groups."""
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    from paper_2604_00250_amd.tune import autotune
    w = I.batched_patches()
    say(f"[full batched] {len(w.groups)} patches, {w.n_vox} voxels")
    rng = np.random.default_rng(4096)
    for g in w.groups:
        g.theta = I.perturb_theta(g.theta, rng, scale=0.5)
    prob = Problem(w.groups)
    st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups])
    res = autotune(st, cache=None, reps=3, cands=[dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1)])
    info = prob.plan_info()
    say(f"[full batched] tuned: {res['launch']} {res['ms']:.3f} ms per iteration; "
        f"{len(res['buckets'])} bucket overrides; plan {info} "
        f"({info['items'] / max(info['persistent_blocks'], 1):.1f} items per block)")
    st.loss_grad()
    torch.cuda.synchronize()
    assert int(st.status.item()) == 0
    loss = st.loss_host()
    gm, gc = st.grads_host()
    # the sample
    buckets = {}
    for i, g in enumerate(w.groups):
        buckets.setdefault((g.acq.n, g.K, g.mode), []).append(i)
    pick = {int(rng.choice(v)) for v in buckets.values()}
    pick.add(int(np.argmax([g.n_vox for g in w.groups])))
    rest = [i for i in range(len(w.groups)) if i not in pick]
    pick |= {int(i) for i in rng.choice(rest, size=64 - len(pick), replace=False)}
    pick = sorted(pick)
    say(f"[full batched] {len(buckets)} buckets, {len(pick)} groups sampled "
        f"(largest {max(w.groups[i].n_vox for i in pick)} voxels)")
    with mp.get_context("spawn").Pool(_pool_size(16)) as pool:
        refs = pool.map(oracle_group, [(w.groups[i], w.groups[i].theta) for i in pick], chunksize=1)
    for i, (out, grad) in zip(pick, refs):
        g = w.groups[i]
        assert_parity(f"full-batched/{i} V={g.n_vox} K={g.K} N={g.acq.n} {g.mode}", loss[i],
                      merged_grad(gm[i], gc[i]), out, grad)
