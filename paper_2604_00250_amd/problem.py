"""Problem handle and device buffers over the libprism C ABI.

`Problem` wraps a `prism_problem` handle built from `inputs.Group`
descriptions; `pack_*` / `unpack_*` convert between per-group parameter
dictionaries and the library's flat layouts (documented in include/prism.h);
`DeviceState` keeps y, parameters, gradients, optimiser moments, workspace,
loss and status resident on the GPU (torch tensors, used only as device
memory) and drives the per-iteration calls on a torch stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

MICRO_ROWS = ("s0", "logits", "v", "fin", "dpar", "dperp")


def n_params_vox(K: int, learn_d: bool) -> int:
    return 4 * K + 5 + (2 if learn_d else 0)


class Problem:
    """A set of independent groups (each one calibration group of PRISM)."""

    def __init__(self, groups: Sequence, model: Optional[L.Model] = None, launch: Optional[dict] = None):
        lib = L.lib()
        self.groups = list(groups)
        acq_index = {}
        acqs = []
        self._keep = []
        for g in self.groups:
            key = id(g.acq)
            if key not in acq_index:
                acq_index[key] = len(acqs)
                bval = np.ascontiguousarray(g.acq.bval, dtype=np.float32)
                bvec = np.ascontiguousarray(g.acq.bvec, dtype=np.float32)
                self._keep += [bval, bvec]
                acqs.append(L.Acq(bval.shape[0], bval.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  bvec.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        descs = (L.GroupDesc * len(self.groups))()
        for i, g in enumerate(self.groups):
            mask = np.ascontiguousarray(g.mask, dtype=np.uint8)
            self._keep.append(mask)
            pri = 0
            for p in g.priors:
                pri |= L.PRIOR_BITS[p]
            nx, ny, nz = g.shape
            descs[i] = L.GroupDesc(nx, ny, nz, g.K, L.RICIAN if g.mode == "nll" else L.MSE,
                                   L.BIAS[g.bias], acq_index[id(g.acq)], int(g.neighbourhood),
                                   int(bool(g.learn_diffusivity)), pri,
                                   mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        acq_arr = (L.Acq * len(acqs))(*acqs)
        self.model = model if model is not None else L.model_defaults()
        h = ctypes.c_void_p()
        L.check(lib.prism_problem_create(ctypes.byref(h), descs, len(self.groups), acq_arr,
                                         len(acqs), ctypes.byref(self.model)))
        self.handle = h
        self._keep = None
        info = L.ProblemInfo()
        L.check(lib.prism_problem_info(h, ctypes.byref(info)))
        self.info = info
        self.ginfo = []
        for i in range(len(self.groups)):
            gi = L.GroupInfo()
            L.check(lib.prism_group_info(h, i, ctypes.byref(gi)))
            self.ginfo.append(gi)
        if launch:
            self.tune(**launch)

    # -- handle management -------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().prism_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, vox_per_lane=1, n_split=1, item_vox=0, persistent=0, max_blocks=0, stagger=1, concurrent=1,
             buckets=()):
        """Set the launch shape; `buckets` holds per-bucket overrides, dicts with
        n_meas, K, mode ("mse"/"nll" or 0/1), learn_diffusivity, vox_per_lane,
        n_split and item_vox."""
        base = L.Launch(vox_per_lane, n_split, item_vox, int(persistent), int(max_blocks), int(stagger),
                        int(concurrent))
        arr = (L.BucketLaunch * max(len(buckets), 1))()
        for i, b in enumerate(buckets):
            mode = b["mode"]
            mode = L.RICIAN if mode in ("nll", L.RICIAN) else L.MSE
            arr[i] = L.BucketLaunch(int(b["n_meas"]), int(b["K"]), mode, int(bool(b["learn_diffusivity"])),
                                    int(b.get("vox_per_lane", 1)), int(b["n_split"]), int(b["item_vox"]))
        L.check(L.lib().prism_problem_tune_buckets(self.handle, ctypes.byref(base), arr, len(buckets)))

    def launch(self) -> dict:
        ln = L.Launch()
        L.check(L.lib().prism_problem_launch(self.handle, ctypes.byref(ln)))
        return dict(vox_per_lane=ln.vox_per_lane, n_split=ln.n_split, item_vox=ln.item_vox,
                    persistent=ln.persistent, max_blocks=ln.max_blocks, stagger=ln.stagger,
                    concurrent=ln.concurrent)

    def buckets(self) -> list:
        """The problem's (N, K, mode, learned D) buckets with the shape each runs with."""
        n = ctypes.c_int32()
        L.check(L.lib().prism_problem_buckets(self.handle, None, 0, ctypes.byref(n)))
        arr = (L.BucketLaunch * max(n.value, 1))()
        L.check(L.lib().prism_problem_buckets(self.handle, arr, n.value, ctypes.byref(n)))
        return [dict(n_meas=b.n_meas, K=b.K, mode="nll" if b.mode == L.RICIAN else "mse",
                     learn_diffusivity=bool(b.learn_diffusivity), vox_per_lane=b.vox_per_lane,
                     n_split=b.n_split, item_vox=b.item_vox) for b in arr[:n.value]]

    def plan_info(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().prism_problem_plan_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(items=a.value, launches=b.value, persistent_blocks=c.value)

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        L.check(L.lib().prism_workspace_bytes(self.handle, ctypes.byref(n)))
        return int(n.value)

    @property
    def n_groups(self):
        return len(self.groups)

    # -- host-side layout conversion ----------------------------------------
    def pack_micro(self, thetas: Sequence[dict]) -> np.ndarray:
        out = np.zeros(self.info.n_micro, dtype=np.float32)
        for g, gi, th in zip(self.groups, self.ginfo, thetas):
            V, C = int(gi.n_vox), g.K + 3
            rows = [np.asarray(th["s0"]).reshape(1, V), np.asarray(th["logits"]).reshape(C, V),
                    np.asarray(th["v"]).reshape(3 * g.K, V), np.asarray(th["fin"]).reshape(1, V)]
            if g.learn_diffusivity:
                rows += [np.asarray(th["dpar"]).reshape(1, V), np.asarray(th["dperp"]).reshape(1, V)]
            blk = np.concatenate(rows, 0).astype(np.float32)
            assert blk.shape[0] == gi.n_params_vox
            out[gi.micro_offset:gi.micro_offset + blk.size] = blk.reshape(-1)
        return out

    def pack_cal(self, thetas: Sequence[dict]) -> np.ndarray:
        out = np.zeros(self.info.n_cal, dtype=np.float32)
        for gi, th in zip(self.ginfo, thetas):
            vec = np.concatenate([np.asarray(th["bias"], dtype=np.float32).reshape(-1),
                                  np.asarray(th["alpha"], dtype=np.float32).reshape(-1),
                                  np.asarray(th["beta"], dtype=np.float32).reshape(-1),
                                  np.asarray(th["sigma_log"], dtype=np.float32).reshape(1)])
            assert vec.size == gi.n_cal, (vec.size, gi.n_cal)
            out[gi.cal_offset:gi.cal_offset + vec.size] = vec
        return out

    def pack_y(self, ys: Sequence[np.ndarray]) -> np.ndarray:
        out = np.empty(self.info.n_y, dtype=np.float32)
        for gi, y in zip(self.ginfo, ys):
            out[gi.y_offset:gi.y_offset + y.size] = np.asarray(y, dtype=np.float32).reshape(-1)
        return out

    def unpack_micro(self, flat: np.ndarray) -> list:
        res = []
        for g, gi in zip(self.groups, self.ginfo):
            V, K = int(gi.n_vox), g.K
            blk = np.asarray(flat[gi.micro_offset:gi.micro_offset + gi.n_params_vox * V]).reshape(gi.n_params_vox, V)
            C = K + 3
            d = dict(s0=blk[0], logits=blk[1:1 + C], v=blk[1 + C:1 + C + 3 * K].reshape(K, 3, V),
                     fin=blk[1 + C + 3 * K])
            if g.learn_diffusivity:
                d["dpar"] = blk[2 + C + 3 * K]
                d["dperp"] = blk[3 + C + 3 * K]
            res.append(d)
        return res

    def unpack_cal(self, flat: np.ndarray) -> list:
        res = []
        for gi in self.ginfo:
            vec = np.asarray(flat[gi.cal_offset:gi.cal_offset + gi.n_cal])
            nb, N = gi.n_bias, gi.n_meas
            res.append(dict(bias=vec[:nb], alpha=vec[nb:nb + N], beta=vec[nb + N:nb + 2 * N],
                            sigma_log=vec[nb + 2 * N]))
        return res

    def unpack_y(self, flat: np.ndarray) -> list:
        return [np.asarray(flat[gi.y_offset:gi.y_offset + gi.n_meas * gi.n_vox]).reshape(gi.n_meas, int(gi.n_vox))
                for gi in self.ginfo]

    # -- raw calls on device pointers ----------------------------------------
    def loss_grad_ptr(self, y, th_micro, th_cal, loss, g_micro, g_cal, ws, ws_bytes, status, stream):
        L.check(L.lib().prism_loss_grad(self.handle, y, th_micro, th_cal, loss, g_micro, g_cal, ws,
                                        ws_bytes, status, stream))

    def loss_grad_noalloc_ptr(self, y, th_micro, th_cal, loss, g_micro, g_cal, status, stream):
        L.check(L.lib().prism_loss_grad_noalloc(self.handle, y, th_micro, th_cal, loss, g_micro, g_cal,
                                                status, stream))

    def iteration_adam_ptr(self, y, th_micro, th_cal, m_micro, v_micro, m_cal, v_cal, step, lr, b1, b2, eps,
                           update_cal, loss, g_micro, g_cal, ws, ws_bytes, status, stream, hist=None,
                           hist_len=0):
        L.check(L.lib().prism_iteration_adam(self.handle, y, th_micro, th_cal, m_micro, v_micro, m_cal, v_cal,
                                             step, float(lr), float(b1), float(b2), float(eps),
                                             int(bool(update_cal)), loss, hist, int(hist_len), g_micro, g_cal,
                                             ws, ws_bytes, status, stream))

    def synthesize_ptr(self, th_micro, th_cal, yhat, stream):
        L.check(L.lib().prism_synthesize(self.handle, th_micro, th_cal, yhat, stream))

    def stitch_plan(self, shape, z0) -> int:
        """Declare the groups to be z-slabs of a volume `shape` starting at
        slices `z0`; returns the number of stitched output voxels."""
        z = np.ascontiguousarray(z0, dtype=np.int32)
        if z.shape != (self.n_groups,):
            raise ValueError("one slab start per group")
        n = ctypes.c_int64()
        nx, ny, nz = (int(s) for s in shape)
        L.check(L.lib().prism_stitch_plan(self.handle, nx, ny, nz,
                                          z.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(n)))
        self.n_stitch = int(n.value)
        return self.n_stitch

    def stitch_maps_ptr(self, th_micro, maps, stream):
        L.check(L.lib().prism_stitch_maps(self.handle, th_micro, maps, stream))

    def profile(self, enable: bool, max_launches: int = 4096):
        L.check(L.lib().prism_profile_enable(self.handle, int(enable), int(max_launches)))

    def profile_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        L.check(L.lib().prism_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


def adam_step_ptr(p, g, m, v, n, lr, beta1, beta2, eps, step, stream):
    L.check(L.lib().prism_adam_step(p, g, m, v, int(n), float(lr), float(beta1), float(beta2),
                                    float(eps), step, stream))


def rprop_step_ptr(p, g, prev, step, n, eta_minus, eta_plus, step_min, step_max, stream):
    L.check(L.lib().prism_rprop_step(p, g, prev, step, int(n), float(eta_minus), float(eta_plus),
                                     float(step_min), float(step_max), stream))


class DeviceState:
    """Everything one fit needs, resident in HBM.

    The parameters live in ONE flat buffer `params` = [theta_micro | theta_cal]
    (and the gradient likewise), so one optimiser call updates both.
    """

    def __init__(self, prob: Problem, ys=None, thetas=None, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.device = torch.device(device)
        info = prob.info
        self.n_micro, self.n_cal, self.n_y = int(info.n_micro), int(info.n_cal), int(info.n_y)
        n = self.n_micro + self.n_cal
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.zeros(n, **f32)
        self.grad = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.y = torch.zeros(max(self.n_y, 1), **f32)
        self.loss = torch.zeros((prob.n_groups, len(L.LOSS_TERMS)), dtype=torch.float64, device=self.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.step = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.ws_bytes = prob.workspace_bytes()
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.stream = stream
        if ys is not None:
            self.set_y(ys)
        if thetas is not None:
            self.set_params(thetas)

    def resize_workspace(self):
        """Re-size the workspace after the problem's launch plan changed."""
        need = self.prob.workspace_bytes()
        if need > self.ws.numel():
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        self.ws_bytes = need

    def _s(self):
        st = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(st.cuda_stream)

    def set_y(self, ys):
        flat = self.prob.pack_y(ys) if isinstance(ys, (list, tuple)) else np.asarray(ys, dtype=np.float32)
        self.y[: flat.size].copy_(self.torch.from_numpy(flat))

    def set_params(self, thetas):
        self.params[: self.n_micro].copy_(self.torch.from_numpy(self.prob.pack_micro(thetas)))
        self.params[self.n_micro:].copy_(self.torch.from_numpy(self.prob.pack_cal(thetas)))

    def reset_optimizer(self):
        self.m.zero_()
        self.v.zero_()
        self.step.zero_()

    def ptrs(self):
        p = self.params.data_ptr()
        g = self.grad.data_ptr()
        return p, p + 4 * self.n_micro, g, g + 4 * self.n_micro

    def loss_grad(self):
        pm, pc, gm, gc = self.ptrs()
        self.prob.loss_grad_ptr(self.y.data_ptr(), pm, pc, self.loss.data_ptr(), gm, gc,
                                self.ws.data_ptr(), self.ws_bytes, self.status.data_ptr(), self._s())

    def adam(self, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, n=None):
        n = self.n_micro + self.n_cal if n is None else int(n)
        adam_step_ptr(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                      n, lr, beta1, beta2, eps, self.step.data_ptr(), self._s())

    def iteration(self, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, update_cal=True, history=None):
        """One Adam iteration through prism_iteration_adam (the per-voxel update
        runs inside the fused pass); self.loss holds the loss before the step.
        history: optional float64 device tensor [L][n_groups][10]; the loss rows
        also go to row (iteration index mod L), written by the library."""
        pm, pc, gm, gc = self.ptrs()
        m, v = self.m.data_ptr(), self.v.data_ptr()
        hp, hl = (history.data_ptr(), history.shape[0]) if history is not None else (None, 0)
        if history is not None:
            if (history.dtype != self.torch.float64 or history.device != self.device or not history.is_contiguous()
                    or tuple(history.shape[1:]) != (self.prob.n_groups, len(L.LOSS_TERMS))):
                raise ValueError("history must be a contiguous float64 device tensor [L][n_groups][10]")
        self.prob.iteration_adam_ptr(self.y.data_ptr(), pm, pc, m, v, m + 4 * self.n_micro, v + 4 * self.n_micro,
                                     self.step.data_ptr(), lr, beta1, beta2, eps, update_cal,
                                     self.loss.data_ptr(), gm, gc, self.ws.data_ptr(), self.ws_bytes,
                                     self.status.data_ptr(), self._s(), hist=hp, hist_len=hl)

    def iteration_unfused(self, lr=1e-2):
        """The same iteration as prism_loss_grad followed by prism_adam_step."""
        self.loss_grad()
        self.adam(lr)

    def synthesize(self, out=None):
        if out is None:
            out = self.torch.empty(max(self.n_y, 1), dtype=self.torch.float32, device=self.device)
        pm, pc, _, _ = self.ptrs()
        self.prob.synthesize_ptr(pm, pc, out.data_ptr(), self._s())
        return out

    def stitch_maps(self, out=None):
        """Whole-volume maps [P][n_out] of the current parameters (after
        Problem.stitch_plan), on the device."""
        g0 = self.prob.groups[0]
        P = n_params_vox(g0.K, bool(g0.learn_diffusivity))
        n = self.prob.n_stitch
        if out is None:
            out = self.torch.empty((P, max(n, 1)), dtype=self.torch.float32, device=self.device)
        self.prob.stitch_maps_ptr(self.params.data_ptr(), out.data_ptr(), self._s())
        return out[:, :n]

    # host views
    def grads_host(self):
        g = self.grad.cpu().numpy()
        return self.prob.unpack_micro(g[: self.n_micro]), self.prob.unpack_cal(g[self.n_micro:])

    def params_host(self):
        p = self.params.cpu().numpy()
        return self.prob.unpack_micro(p[: self.n_micro]), self.prob.unpack_cal(p[self.n_micro:])

    def loss_host(self):
        return self.loss.cpu().numpy()
