"""torch.autograd.Function over the fused pass.

`PrismLoss.apply(params, problem_state)` returns the total objective (sum of
the groups' totals, float64) of the flat parameter vector `params`
([theta_micro | theta_cal], float32, on the GPU).  The forward call runs the
fused forward + adjoint kernel once (prism_loss_grad): the compartment
exponentials are recomputed inside the kernel's adjoint and never stored, so
the only saved tensor is the gradient itself (P floats per voxel plus the
calibration vector).  backward() scales that gradient by the incoming one.
"""
from __future__ import annotations

import torch

from . import _lib as L


class PrismLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, state):
        if params.device != state.params.device or params.dtype != torch.float32 or not params.is_contiguous():
            raise ValueError("params must be a contiguous float32 tensor on the problem's device")
        if params.numel() != state.params.numel():
            raise ValueError("params has the wrong size for this problem")
        grad = torch.empty_like(params)
        pm = params.data_ptr()
        gm = grad.data_ptr()
        st = state
        st.prob.loss_grad_ptr(st.y.data_ptr(), pm, pm + 4 * st.n_micro, st.loss.data_ptr(), gm,
                              gm + 4 * st.n_micro, st.ws.data_ptr(), st.ws_bytes, st.status.data_ptr(),
                              st._s())
        ctx.save_for_backward(grad)
        return st.loss[:, L.LOSS_TOTAL].sum()

    @staticmethod
    def backward(ctx, g_out):
        (grad,) = ctx.saved_tensors
        return grad * g_out.to(grad.dtype), None


def prism_loss(params, state):
    return PrismLoss.apply(params, state)
