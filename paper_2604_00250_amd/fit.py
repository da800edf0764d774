"""The fit loop: one iteration (fused pass + optimiser step) captured as a HIP
graph and replayed, with the step counter and the per-iteration loss history
on the device; checkpoint / resume of the optimiser state.

    state = DeviceState(problem, ys, thetas)
    hist = fit(state, iterations=1000, lr=1e-2)          # graph-captured
    hist = fit(state, iterations=100, graph=False)       # eager

The host synchronises once, at the end.  `history` is a float64 device tensor
[iterations][n_groups][10] (data, spatial, rep, sparse, orphan, continuity,
ordering, cal, tv, total; the layout of the library's loss rows) of the
loss evaluated at the start of each iteration.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .problem import DeviceState, rprop_step_ptr


class Loop:
    """One optimiser iteration on a DeviceState, optionally captured as a graph."""

    def __init__(self, state: DeviceState, lr: float = 1e-2, optimizer: str = "adam",
                 betas=(0.9, 0.999), eps: float = 1e-8, history: int = 0,
                 rprop=(0.5, 1.2, 1e-6, 50.0), calibrate: bool = True):
        self.st = state
        # calibrate=False keeps theta_cal fixed: the optimiser sees theta_micro only
        self.calibrate = calibrate
        self.n_opt = state.n_micro + (state.n_cal if calibrate else 0)
        self.lr = lr
        self.optimizer = optimizer
        self.betas = betas
        self.eps = eps
        self.rprop = rprop
        dev = state.device
        self.hist = torch.zeros((max(history, 1), state.prob.n_groups, len(L.LOSS_TERMS)), dtype=torch.float64, device=dev)
        self.hist_len = max(history, 1)
        self.graph = None
        if optimizer == "rprop":
            n = state.n_micro + state.n_cal
            self.prev = torch.zeros(n, dtype=torch.float32, device=dev)
            self.rstep = torch.full((n,), lr, dtype=torch.float32, device=dev)
            self.it = torch.zeros(1, dtype=torch.int64, device=dev)

    def _record(self):
        # Rprop: history slot = the iteration's index (device counter), modulo the ring length
        idx = torch.remainder(self.it, self.hist_len)
        self.hist.index_copy_(0, idx, self.st.loss.unsqueeze(0))

    def step_eager(self):
        st = self.st
        if self.optimizer == "adam":
            # one call: loss at the current parameters (also written by the library to
            # the history row of this iteration), then the Adam step
            st.iteration(self.lr, self.betas[0], self.betas[1], self.eps, update_cal=self.calibrate,
                         history=self.hist)
            return
        st.loss_grad()
        self._record()
        em, ep, smin, smax = self.rprop
        rprop_step_ptr(st.params.data_ptr(), st.grad.data_ptr(), self.prev.data_ptr(),
                       self.rstep.data_ptr(), self.n_opt, em, ep, smin, smax, st._s())
        self.it.add_(1)

    def capture(self):
        """Capture one iteration; the library calls allocate nothing and never
        synchronise, so they record into the graph as plain kernel nodes."""
        st = self.st
        side = torch.cuda.Stream(device=st.device)
        side.wait_stream(torch.cuda.current_stream(st.device))
        old = st.stream
        with torch.cuda.stream(side):
            st.stream = side
            self.step_eager()  # warm-up on the capture stream (allocates torch temporaries)
        torch.cuda.current_stream(st.device).wait_stream(side)
        torch.cuda.synchronize(st.device)
        # undo the warm-up iteration's effect on the state by capturing from a copy point
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            self.step_eager()
        st.stream = old
        self.graph = g
        return g

    def replay(self, n: int):
        for _ in range(n):
            self.graph.replay()


def fit(state: DeviceState, iterations: int, lr: float = 1e-2, graph: bool = True,
        optimizer: str = "adam", calibrate: bool = True) -> torch.Tensor:
    """Run `iterations` optimiser iterations; returns the device loss history.
    calibrate=False holds the calibration parameters at their current values."""
    if graph:
        snap = snapshot(state)
        loop = Loop(state, lr=lr, optimizer=optimizer, history=iterations, calibrate=calibrate)
        loop.capture()                      # the warm-up ran one iteration: restore, then replay
        restore(state, snap)
        if optimizer == "rprop":
            loop.prev.zero_()
            loop.rstep.fill_(lr)
            loop.it.zero_()
        loop.hist.zero_()
        loop.replay(iterations)
    else:
        loop = Loop(state, lr=lr, optimizer=optimizer, history=iterations, calibrate=calibrate)
        for _ in range(iterations):
            loop.step_eager()
    torch.cuda.synchronize(state.device)
    return loop.hist


# ----------------------------------------------------------------------------
# checkpoint / resume
# ----------------------------------------------------------------------------

def snapshot(state: DeviceState) -> dict:
    return {k: getattr(state, k).clone() for k in ("params", "m", "v", "step", "status")}


def restore(state: DeviceState, snap: dict):
    for k, t in snap.items():
        getattr(state, k).copy_(t)


def save_checkpoint(state: DeviceState, path: str, **meta):
    arrays = {k: v.cpu().numpy() for k, v in snapshot(state).items()}
    arrays.update({f"meta_{k}": np.asarray(v) for k, v in meta.items()})
    np.savez(path, **arrays)


def load_checkpoint(state: DeviceState, path: str) -> dict:
    z = np.load(path, allow_pickle=False)
    for k in ("params", "m", "v", "step", "status"):
        t = getattr(state, k)
        a = z[k]
        if a.shape != tuple(t.shape):
            raise ValueError(f"checkpoint {k} has shape {a.shape}, state has {tuple(t.shape)}")
        t.copy_(torch.from_numpy(a))
    return {k[5:]: z[k] for k in z.files if k.startswith("meta_")}
