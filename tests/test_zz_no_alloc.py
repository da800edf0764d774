"""prism_loss_grad_noalloc (the entry point whose workspace is the library's
static device array) against prism_loss_grad (caller workspace): bit for bit
on two calls in a row, the second on a smaller problem, so the second call
runs on what the first left in the shared array; and a problem whose
workspace exceeds the static array is refused before anything is queued."""
import ctypes

import numpy as np
import pytest

from paper_2604_00250_amd import _lib as L
from paper_2604_00250_amd import inputs as I

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _compare(group, theta):
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    prob = Problem([group])
    st = DeviceState(prob, ys=[group.y], thetas=[theta])
    st.loss_grad()
    torch.cuda.synchronize()
    loss_ref, grad_ref, status_ref = st.loss.clone(), st.grad.clone(), st.status.clone()
    loss = torch.full_like(st.loss, float("nan"))
    grad = torch.full_like(st.grad, float("nan"))
    status = torch.zeros_like(st.status)
    pm, pc, _, _ = st.ptrs()
    gm = grad.data_ptr()
    prob.loss_grad_noalloc_ptr(st.y.data_ptr(), pm, pc, loss.data_ptr(), gm, gm + 4 * st.n_micro,
                               status.data_ptr(), st._s())
    torch.cuda.synchronize()
    say(f"[noalloc] V={group.n_vox} N={group.acq.n} workspace {prob.workspace_bytes()} B "
        f"loss {loss[0, -1].item():.10g} ref {loss_ref[0, -1].item():.10g}")
    assert int(status_ref.item()) == 0
    assert torch.equal(loss, loss_ref)
    assert torch.equal(grad, grad_ref)
    assert torch.equal(status, status_ref)


def test_noalloc_is_bitwise_loss_grad_on_two_calls_in_a_row():
    large = I.patch16_hcp().groups[0]            # 4096 voxels, N = 288, NLL, calibration
    small = I.patch8_crossings(priors=I.PRIOR_NAMES).groups[0]   # 512 voxels, N = 33
    _compare(large, I.perturb_theta(large.theta, np.random.default_rng(5), scale=0.5))
    _compare(small, I.perturb_theta(small.theta, np.random.default_rng(6), scale=0.5))


def test_noalloc_refuses_a_problem_beyond_the_static_workspace():
    import torch
    from paper_2604_00250_amd.problem import Problem
    acq = I.Acquisition(bval=np.zeros(1), bvec=np.array([[1.0, 0.0, 0.0]]))
    shape = (200, 200, 100)   # 4M voxels with the Eq. 7 prior: ~128 MB of [V][cs] rows
    g = I.Group(shape=shape, mask=np.ones(shape, dtype=bool), acq=acq, K=1, mode="mse",
                priors=("spatial",))
    prob = Problem([g])
    need = prob.workspace_bytes()
    assert need > L.NOALLOC_WORKSPACE_BYTES
    buf = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    p = buf.data_ptr()
    rc = L.lib().prism_loss_grad_noalloc(prob.handle, p, p, p, p, p, p, p, None)
    msg = L.lib().prism_last_error().decode()
    say(f"[noalloc] workspace {need} B: rc {rc}: {msg}")
    assert rc == L.PRISM_E_WORKSPACE and "static workspace" in msg
    torch.cuda.synchronize()
    assert not torch.any(buf)  # nothing was queued
