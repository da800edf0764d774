"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 kernels vs FP64 oracle, same float32 inputs): total loss
relative error <= 1e-5; gradient error <= 1e-4 normwise per parameter class
(max |g - g_ref| / max |g_ref| over the class).
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

from gpu_helpers import (assert_parity, masked_group, merged_grad, run_gpu, run_oracle, say,
                         theta32, with_theta)

pytestmark = pytest.mark.gpu


def _check_groups(name, groups, launch=None, loss_rtol=1e-5, grad_rtol=1e-4):
    say(f"[{name}] groups={len(groups)} V={[g.n_vox for g in groups]} launch={launch}")
    r = run_gpu(groups, [g.theta for g in groups], launch=launch)
    assert r["status"] == 0, r["status"]
    for i, g in enumerate(groups):
        out, grad, _ = run_oracle(g, g.theta)
        assert_parity(f"{name}/{i}", r["loss"][i], merged_grad(r["gmicro"][i], r["gcal"][i]), out, grad,
                      loss_rtol, grad_rtol)
    return r


@pytest.mark.parametrize("priors", [("rep",), I.PRIOR_NAMES])
@pytest.mark.parametrize("perturb", [False, True])
def test_patch8_n33_mse(priors, perturb):
    w = I.patch8_crossings(priors=priors)
    g = w.groups[0]
    if perturb:
        g = with_theta(g, I.perturb_theta(g.theta, np.random.default_rng(5)))
    _check_groups(f"patch8 priors={len(priors)} perturb={perturb}", [g])


@pytest.mark.parametrize("perturb", [False, True])
def test_patch16_n288_nll_calibrated(perturb):
    g = I.patch16_hcp().groups[0]
    if perturb:
        g = with_theta(g, I.perturb_theta(g.theta, np.random.default_rng(6)))
    _check_groups(f"patch16 nll perturb={perturb}", [g])


def test_phantom_crossing_subpatch_learned_diffusivities():
    w = I.tube_phantom()
    corner = I.crossing_subpatch(w, 4)
    g = I.sub_box(w.groups[0], corner, 4)
    g = with_theta(g, I.perturb_theta(g.theta, np.random.default_rng(7)))
    _check_groups("phantom 4^3 K=4 nll learned-D", [g])


RAGGED = [
    dict(shape=(7, 5, 9), K=2, mode="mse", seed=1, acq_kind="two96", bias="poly2"),
    dict(shape=(6, 6, 6), K=4, mode="nll", seed=2, acq_kind="single33", bias="trilinear8"),
    dict(shape=(9, 4, 11), K=3, mode="mse", seed=3, acq_kind="three288", bias="none", nbh=26),
    dict(shape=(5, 7, 5), K=1, mode="nll", seed=4, acq_kind="two96", bias="poly2", learn=True),
    dict(shape=(3, 3, 3), K=5, mode="mse", seed=5, acq_kind="single33", bias="poly2"),
    dict(shape=(10, 10, 3), K=6, mode="nll", seed=6, acq_kind="two96", bias="none", fill=0.5),
]


@pytest.mark.parametrize("launch", [None, dict(vox_per_lane=1, n_split=1, item_vox=256),
                                    dict(vox_per_lane=1, n_split=4, item_vox=64),
                                    dict(vox_per_lane=2, n_split=1, item_vox=512),
                                    dict(vox_per_lane=2, n_split=2, item_vox=256)])
def test_ragged_masked_mixed_groups(launch):
    groups = [masked_group(**kw) for kw in RAGGED]
    _check_groups("ragged", groups, launch=launch)


@pytest.mark.parametrize("order", ["shells", "interleaved"])
@pytest.mark.parametrize("launch", [None, dict(vox_per_lane=1, n_split=2, item_vox=128)])
def test_mse_acquisition_order(order, launch):
    """The same measurements shell by shell (the b = 0 ones first, which the
    pass takes as whole b = 0 tiles) and in a random order (b = 0 measurements
    scattered through the acquisition, every tile mixing shells), with the
    range also split over two waves."""
    g = masked_group(shape=(11, 9, 7), K=3, mode="mse", seed=21, acq_kind="three288", bias="poly2", fill=0.9)
    if order == "interleaved":
        perm = np.random.default_rng(3).permutation(g.acq.n)
        acq = I.Acquisition(bval=g.acq.bval[perm], bvec=g.acq.bvec[perm], name="three288-interleaved")
        th = dict(g.theta)
        th["alpha"], th["beta"] = th["alpha"][perm], th["beta"][perm]
        g = dataclasses.replace(g, acq=acq, y=np.ascontiguousarray(g.y[perm]), theta=th)
    _check_groups(f"order={order}", [g], launch=launch)


def test_many_items_per_group_and_ragged_tail():
    g = masked_group(shape=(23, 19, 17), K=3, mode="mse", seed=11, acq_kind="three288", bias="poly2", fill=0.8)
    _check_groups("multi-item", [g], launch=dict(vox_per_lane=1, n_split=2, item_vox=128))


def test_empty_group_contributes_only_calibration_prior():
    g0 = masked_group(shape=(4, 4, 4), K=2, mode="mse", seed=8, acq_kind="single33")
    empty = dataclasses.replace(g0, mask=np.zeros((4, 4, 4), dtype=bool), y=np.zeros((33, 0), np.float32),
                                theta={k: (v[..., :0] if k not in ("bias", "alpha", "beta", "sigma_log") else v)
                                       for k, v in g0.theta.items()})
    r = run_gpu([g0, empty], [g0.theta, empty.theta])
    assert r["status"] == 0
    out, _, _ = O.objective(O.Problem(coords=np.zeros((0, 3), dtype=int), shape=(4, 4, 4), bval=g0.acq.bval,
                                      bvec=g0.acq.bvec, K=2, mode="mse", bias="poly2"),
                            theta32(empty.theta), np.zeros((33, 0))), None, None
    assert r["loss"][1][9] == pytest.approx(out["total"], rel=1e-6, abs=1e-12)
    assert r["loss"][1][0] == 0.0
    cal = theta32(empty.theta)
    assert np.allclose(r["gcal"][1]["alpha"], 0.02 * cal["alpha"], rtol=1e-5, atol=1e-9)
    out0, grad0, _ = run_oracle(g0, g0.theta)
    assert_parity("nonempty-beside-empty", r["loss"][0], merged_grad(r["gmicro"][0], r["gcal"][0]), out0, grad0)


def test_synthesize_matches_oracle_forward():
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    groups = [masked_group(**kw) for kw in RAGGED[:4]]
    prob = Problem(groups)
    st = DeviceState(prob, ys=[g.y for g in groups], thetas=[g.theta for g in groups])
    out = st.synthesize()
    torch.cuda.synchronize()
    yh = prob.unpack_y(out.cpu().numpy())
    for g, a in zip(groups, yh):
        ref = O.synthesize(O.Problem(coords=g.coords, shape=g.shape, bval=g.acq.bval, bvec=g.acq.bvec, K=g.K,
                                     mode=g.mode, bias=g.bias, learn_diffusivity=g.learn_diffusivity),
                           theta32(g.theta))
        err = np.abs(a - ref).max() / np.abs(ref).max()
        say(f"[synth] K={g.K} max rel err {err:.2e}")
        assert err < 2e-6


def test_adam_and_rprop_match_oracle_elementwise():
    import torch
    from paper_2604_00250_amd.problem import adam_step_ptr, rprop_step_ptr
    rng = np.random.default_rng(0)
    n = 100_003
    p0 = rng.normal(0, 1, n).astype(np.float32)
    dev = torch.device("cuda:0")
    p = torch.from_numpy(p0.copy()).to(dev)
    m = torch.zeros(n, device=dev)
    v = torch.zeros(n, device=dev)
    step = torch.zeros(2, dtype=torch.int32, device=dev)
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    s = torch.cuda.current_stream().cuda_stream
    for t in range(1, 6):
        g = rng.normal(0, 1, n).astype(np.float32)
        gt = torch.from_numpy(g).to(dev)
        adam_step_ptr(p.data_ptr(), gt.data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-2, 0.9, 0.999, 1e-8,
                      step.data_ptr(), s)
        pr, mr, vr = O.adam_step(pr, g.astype(np.float64), mr, vr, t)
    torch.cuda.synchronize()
    assert step.cpu().tolist() == [5, 0]
    assert np.abs(p.cpu().numpy() - pr).max() < 1e-5
    # Rprop
    p = torch.from_numpy(p0.copy()).to(dev)
    prev = torch.zeros(n, device=dev)
    st = torch.full((n,), 0.01, device=dev)
    pr, prevr, str_ = p0.astype(np.float64), np.zeros(n), np.full(n, 0.01)
    for t in range(6):
        g = rng.normal(0, 1, n).astype(np.float32)
        g[::7] = 0.0
        gt = torch.from_numpy(g).to(dev)
        rprop_step_ptr(p.data_ptr(), gt.data_ptr(), prev.data_ptr(), st.data_ptr(), n, 0.5, 1.2, 1e-6, 50.0, s)
        pr, prevr, str_ = O.rprop_step(pr, g, prevr, str_)
    torch.cuda.synchronize()
    assert np.abs(st.cpu().numpy() - str_).max() < 1e-7
    assert np.abs(p.cpu().numpy() - pr).max() < 1e-6


def test_bitwise_determinism_and_direction_sign_invariance():
    groups = [masked_group(**kw) for kw in RAGGED[:3]]
    r1 = run_gpu(groups, [g.theta for g in groups])
    r2 = run_gpu(groups, [g.theta for g in groups], repeat=2)
    assert np.array_equal(r1["loss"], r2["loss"])
    for a, b in zip(r1["gmicro"], r2["gmicro"]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    flipped = []
    for g in groups:
        th = dict(g.theta)
        th["v"] = -th["v"]
        flipped.append(th)
    r3 = run_gpu(groups, flipped)
    assert np.array_equal(r1["loss"], r3["loss"])
    for a, b in zip(r1["gmicro"], r3["gmicro"]):
        assert np.array_equal(a["v"], -b["v"])


def test_status_bits_for_zero_direction_and_nonfinite_data():
    g = masked_group(shape=(4, 4, 4), K=2, mode="mse", seed=9, acq_kind="single33")
    th = {k: v.copy() for k, v in g.theta.items()}
    th["v"][1, :, 5] = 0.0
    r = run_gpu([g], [th])
    assert r["status"] & 4
    y = g.y.copy()
    y[3, 7] = np.nan
    r = run_gpu([dataclasses.replace(g, y=y)], [g.theta])
    assert r["status"] & 1 and r["status"] & 2
    # NLL with an infinite noise level: the loss is not finite
    gn = masked_group(shape=(4, 4, 4), K=2, mode="nll", seed=10, acq_kind="single33")
    th = {k: v.copy() for k, v in gn.theta.items()}
    th["sigma_log"] = np.array(np.inf, dtype=np.float32)
    r = run_gpu([gn], [th])
    assert r["status"] & 1
    th["sigma_log"] = np.array(-np.inf, dtype=np.float32)
    r = run_gpu([gn], [th])
    assert r["status"] & 1


def test_workspace_smaller_than_required_is_rejected():
    import ctypes
    import torch
    from paper_2604_00250_amd import _lib as L
    g = masked_group(shape=(5, 4, 3), K=2, mode="mse", seed=12, acq_kind="single33")
    r = run_gpu([g], [g.theta])
    st = r["state"]
    need = st.prob.workspace_bytes()
    assert need > 0
    pm, pc, gm, gc = st.ptrs()
    rc = L.lib().prism_loss_grad(st.prob.handle, st.y.data_ptr(), pm, pc, st.loss.data_ptr(), gm, gc,
                                 st.ws.data_ptr(), need - 1, st.status.data_ptr(), None)
    assert rc == L.PRISM_E_WORKSPACE
    assert "workspace" in L.lib().prism_last_error().decode()
    rc = L.lib().prism_loss_grad(st.prob.handle, st.y.data_ptr(), pm, pc, st.loss.data_ptr(), gm, gc,
                                 None, need, st.status.data_ptr(), None)
    assert rc == L.PRISM_E_INVALID
    torch.cuda.synchronize()
