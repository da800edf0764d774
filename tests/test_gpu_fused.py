"""The fused Adam iteration (prism_iteration_adam) gives bitwise the results
of prism_loss_grad followed by prism_adam_step, with and without the
calibration update, in the per-variant and the persistent launch, and when a
group's continuity prior makes the call run the two steps one after the
other."""
import numpy as np
import pytest

from gpu_helpers import masked_group, say

pytestmark = pytest.mark.gpu

BASE = [
    dict(shape=(9, 7, 8), K=3, mode="mse", seed=81, acq_kind="two96", bias="poly2"),
    dict(shape=(6, 6, 6), K=2, mode="nll", seed=82, acq_kind="single33", bias="trilinear8"),
    dict(shape=(8, 5, 7), K=4, mode="mse", seed=83, acq_kind="three288", bias="none", nbh=26),
]


def _states(groups, launch):
    from paper_2604_00250_amd.problem import DeviceState, Problem
    prob = Problem(groups, launch=launch)
    mk = lambda: DeviceState(prob, ys=[g.y for g in groups], thetas=[g.theta for g in groups])  # noqa: E731
    return prob, mk(), mk()


def _same(a, b):
    import torch
    return (torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
            and torch.equal(a.step, b.step) and torch.equal(a.loss, b.loss))


@pytest.mark.parametrize("priors", [("spatial", "rep", "sparse", "cal"),
                                    ("spatial", "rep", "sparse", "orphan", "ordering", "cal", "tv"),
                                    ("spatial", "rep", "continuity", "cal")])
@pytest.mark.parametrize("launch", [None, dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1),
                                    dict(vox_per_lane=2, n_split=1, item_vox=512)])
def test_fused_iteration_is_bitwise_loss_grad_plus_adam(priors, launch):
    import torch
    groups = [masked_group(priors=priors, **kw) for kw in BASE]
    prob, a, b = _states(groups, launch)
    for it in range(3):
        a.iteration(1e-2)
        b.iteration_unfused(1e-2)
        torch.cuda.synchronize()
        say(f"[fused {priors} {launch}] it {it} loss {a.loss[:, -1].tolist()}")
        assert _same(a, b), it
    assert int(a.status.item()) == 0 and a.step.tolist() == [3, 0]


def test_fused_iteration_can_hold_the_calibration():
    import torch
    groups = [masked_group(**kw) for kw in BASE[:2]]
    prob, a, b = _states(groups, None)
    cal0 = a.params[a.n_micro:].clone()
    for _ in range(2):
        a.iteration(1e-2, update_cal=False)
        b.loss_grad()
        b.adam(1e-2, n=b.n_micro)
    torch.cuda.synchronize()
    assert torch.equal(a.params[a.n_micro:], cal0)
    assert _same(a, b)
