"""Parity at the benchmark's full size and launch shape: the brain-shaped
volume (145x174x145 grid, ~743k voxels, N=288, K=3, MSE, all priors, the
default launch plan that bench.py times).

* loss terms and the calibration gradient (alpha, beta, quadratic bias) over
  the whole volume: the FP64 oracle in voxel chunks on a spawned pool;
* per-voxel gradients at 64 sampled voxels: the oracle on the union of their
  2-rings (exact at the centres: Eq. 7 couples voxels two steps apart) with
  the global |M| and box.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

import gpu_helpers as H

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("perturb_seed", [None, 123])
def test_brain_volume_full_size(perturb_seed):
    import torch
    from paper_2604_00250_amd.problem import DeviceState, Problem
    g = H._full_workload(perturb_seed)
    V = g.n_vox
    H.say(f"[full] V={V} perturb={perturb_seed}")
    # oracle over the whole volume, chunked, on spawned workers
    chunk = 16384
    jobs = [(perturb_seed, lo, min(V, lo + chunk)) for lo in range(0, V, chunk)]
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    with mp.get_context("spawn").Pool(max(1, min(16, cores))) as pool:
        parts = pool.map(H.oracle_chunk_cal, jobs, chunksize=1)
    data = sum(p[0] for p in parts)
    g_alpha = sum(p[1] for p in parts)
    g_beta = sum(p[2] for p in parts)
    g_bias = sum(p[3] for p in parts)
    th = H.theta32(g.theta)
    oprob = H.oracle_problem(g)
    tr = O.transforms(oprob, th)
    ref = dict(data=data)
    ref["spatial"] = O.spatial_prior(oprob, tr["f"], O.Constants(), with_grad=False)[0]
    ref["rep"] = O.repulsion_prior(oprob, tr["f"], tr["d"], O.Constants())[0]
    ref["sparse"] = O.sparsity_prior(oprob, tr["f"], O.Constants())[0]
    cl, ga, gb, gw = O.calibration_prior(th, O.Constants())
    ref["cal"] = cl
    ref["total"] = sum(ref[k] for k in ("data", "spatial", "rep", "sparse", "cal"))
    for k in O.TERMS:
        ref.setdefault(k, 0.0)
    # GPU, the benchmark's launch plan
    prob = Problem([g])
    st = DeviceState(prob, ys=[g.y], thetas=[g.theta])
    st.loss_grad()
    torch.cuda.synchronize()
    loss = st.loss_host()[0]
    gm, gc = st.grads_host()
    assert int(st.status.item()) == 0
    H.say(f"[full] launch {prob.launch()} loss gpu {loss[9]:.10g} ref {ref['total']:.10g}")
    for i, t in enumerate(O.TERMS[:-1]):
        assert abs(loss[i] - ref[t]) <= 1e-5 * abs(ref["total"]) + 1e-12, (t, loss[i], ref[t])
    assert abs(loss[9] - ref["total"]) <= 1e-5 * abs(ref["total"])
    errs = H.class_errors(gc[0], dict(alpha=g_alpha + ga, beta=g_beta + gb, bias=g_bias + gw))
    H.say(f"[full] calibration gradient errors {errs}")
    assert max(errs.values()) <= 1e-4
    # sampled per-voxel gradients
    rng = np.random.default_rng(7 if perturb_seed is None else perturb_seed)
    centres = rng.choice(V, size=64, replace=False)
    ring = H.two_ring(g.coords, g.shape, centres)
    sub = O.Problem(coords=g.coords[ring], shape=g.shape, bval=g.acq.bval, bvec=g.acq.bvec, K=g.K,
                    mode=g.mode, bias=g.bias, priors=tuple(g.priors), norm_count=V)
    ths = {k: (v[..., ring] if k not in ("bias", "alpha", "beta", "sigma_log") else v) for k, v in th.items()}
    _, gs, _ = O.loss_grad(sub, ths, np.asarray(g.y[:, ring], np.float64))
    pos = np.searchsorted(ring, centres)
    sample_ref = {k: gs[k][..., pos] for k in ("s0", "logits", "v", "fin")}
    sample_gpu = {k: np.asarray(gm[0][k])[..., centres] for k in ("s0", "logits", "v", "fin")}
    errs = H.class_errors(sample_gpu, sample_ref)
    H.say(f"[full] sampled per-voxel gradient errors {errs}")
    assert max(errs.values()) <= 1e-4
