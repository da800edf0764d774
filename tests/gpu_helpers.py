"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs, and compare them."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

import oracle as O
from paper_2604_00250_amd import inputs as I

LOSS_RTOL = 1e-5      # relative error of the total loss (FP32 kernels vs FP64 oracle)
GRAD_RTOL = 1e-4      # normwise per parameter class: max|g - g_ref| / max|g_ref|

CLASSES = {
    "s0": ("s0",), "fractions": ("logits",), "directions": ("v",), "f_intra": ("fin",),
    "diffusivities": ("dpar", "dperp"), "bias": ("bias",), "alpha": ("alpha",), "beta": ("beta",),
    "sigma": ("sigma_log",),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_problem(g: I.Group, norm_count=None, coords=None) -> O.Problem:
    return O.Problem(coords=g.coords if coords is None else coords, shape=tuple(g.shape),
                     bval=np.asarray(g.acq.bval, dtype=np.float64),
                     bvec=np.asarray(g.acq.bvec, dtype=np.float64), K=g.K, mode=g.mode, bias=g.bias,
                     learn_diffusivity=g.learn_diffusivity, neighbourhood=g.neighbourhood,
                     priors=tuple(g.priors), norm_count=norm_count)


def theta64(th):
    return {k: np.asarray(v, dtype=np.float64) for k, v in th.items()}


def theta32(th):
    """The float32 parameters both sides evaluate (the oracle gets them exactly)."""
    return {k: np.asarray(np.asarray(v, dtype=np.float32), dtype=np.float64) for k, v in th.items()}


def run_oracle(g: I.Group, th: dict, consts: O.Constants = O.Constants()):
    prob = oracle_problem(g)
    y = np.asarray(g.y, dtype=np.float64)
    out, grad, yhat = O.loss_grad(prob, theta32(th), y, consts)
    return out, grad, yhat


def model_of(consts: O.Constants):
    """The library's model constants with the oracle's values."""
    from paper_2604_00250_amd import _lib as L
    m = L.model_defaults()
    for name, _ in L.Model._fields_:
        setattr(m, name, float(getattr(consts, name)))
    return m


def run_gpu(groups, thetas, launch=None, repeat=1, consts: O.Constants = None):
    from paper_2604_00250_amd.problem import DeviceState, Problem
    import torch
    prob = Problem(groups, launch=launch, model=None if consts is None else model_of(consts))
    st = DeviceState(prob, ys=[g.y for g in groups], thetas=thetas)
    for _ in range(repeat):
        st.loss_grad()
    torch.cuda.synchronize()
    gm, gc = st.grads_host()
    loss = st.loss_host()
    status = int(st.status.cpu().item())
    return dict(prob=prob, state=st, loss=loss, gmicro=gm, gcal=gc, status=status)


def merged_grad(gm, gc):
    d = dict(gm)
    d.update(gc)
    return d


def class_errors(g_gpu: dict, g_ref: dict):
    errs = {}
    for cls, keys in CLASSES.items():
        a = [np.asarray(g_gpu[k], dtype=np.float64).ravel() for k in keys if k in g_ref and k in g_gpu]
        b = [np.asarray(g_ref[k], dtype=np.float64).ravel() for k in keys if k in g_ref and k in g_gpu]
        if not a:
            continue
        a, b = np.concatenate(a), np.concatenate(b)
        if b.size == 0:
            continue
        scale = np.abs(b).max()
        errs[cls] = float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a).max())
    return errs


# Loss terms checked against their own oracle value: relative to the term
# itself (TV: 1e-4, since each face pair is the float32 difference of two
# nearby bias values), with an absolute floor far below any term's size for
# terms whose reference is zero.
TERM_RTOL = {"tv": 1e-4}
TERM_ATOL = 1e-12


def assert_parity(name, loss_gpu_row, g_gpu, out_ref, g_ref, loss_rtol=LOSS_RTOL, grad_rtol=GRAD_RTOL):
    terms = O.TERMS
    it = terms.index("total")
    tot_ref = out_ref["total"]
    rel = abs(loss_gpu_row[it] - tot_ref) / max(abs(tot_ref), 1e-300)
    errs = class_errors(g_gpu, g_ref)
    term_rel = {t: abs(loss_gpu_row[i] - out_ref[t]) / abs(out_ref[t])
                for i, t in enumerate(terms[:-1]) if out_ref[t] != 0.0}
    say(f"[{name}] loss gpu={loss_gpu_row[it]:.10g} ref={tot_ref:.10g} rel={rel:.2e} "
        + " ".join(f"{k}={v:.1e}" for k, v in errs.items())
        + " | terms " + " ".join(f"{k}={v:.1e}" for k, v in term_rel.items()))
    for i, t in enumerate(terms[:-1]):
        ref = out_ref[t]
        tol = max(loss_rtol, TERM_RTOL.get(t, 0.0)) * abs(ref) + TERM_ATOL * max(1.0, abs(tot_ref))
        assert abs(loss_gpu_row[i] - ref) <= tol, (name, t, loss_gpu_row[i], ref)
    assert rel <= loss_rtol, (name, rel)
    for cls, e in errs.items():
        assert e <= grad_rtol, (name, cls, e)
    return rel, errs


def masked_group(shape, K, mode, seed, acq_kind="two96", bias="poly2", fill=0.7, learn=False,
                 nbh=6, priors=I.PRIOR_NAMES, snr=25.0):
    """A group with a random mask and a ragged voxel count, truth from the generator."""
    rng = np.random.default_rng(seed)
    acq = I.make_acquisition(acq_kind, rng)
    mask = rng.random(shape) < fill
    mask.reshape(-1)[0] = True
    V = int(mask.sum())
    truth = I.tissue_truth(V, rng, max_fib=min(K, 3))
    S = I.truth_signal(acq, truth)
    sigma = 1.0 / snr
    y = I.rician(S, sigma, rng)
    nb = {"none": 0, "poly2": 10, "trilinear8": 512}[bias]
    th = I.init_theta(V, K, acq.n, nb, rng, sigma_init=2 * sigma if mode == "nll" else 0.0,
                      learn_diffusivity=learn)
    th = I.perturb_theta(th, rng, scale=0.7)
    return I.Group(shape=shape, mask=mask, acq=acq, K=K, mode=mode, bias=bias, learn_diffusivity=learn,
                   neighbourhood=nbh, priors=tuple(priors), y=y, theta=th, sigma_true=sigma)


def with_theta(g: I.Group, th: dict) -> I.Group:
    return dataclasses.replace(g, theta=th)


# ----------------------------------------------------------------------------
# full-size checks: the oracle in chunks on a spawned process pool
# ----------------------------------------------------------------------------

_FULL = {}


def _full_workload(perturb_seed):
    key = ("brain_volume", perturb_seed)
    if key not in _FULL:
        w = I.brain_volume()
        g = w.groups[0]
        if perturb_seed is not None:
            g = with_theta(g, I.perturb_theta(g.theta, np.random.default_rng(perturb_seed), scale=0.5))
        _FULL.clear()
        _FULL[key] = g
    return _FULL[key]


def oracle_chunk_cal(args):
    """Data term and calibration gradient of one voxel chunk of the brain-shaped
    volume (priors off; the calibration prior is added once by the caller)."""
    perturb_seed, lo, hi = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    g = _full_workload(perturb_seed)
    prob = oracle_problem(g, norm_count=g.n_vox, coords=g.coords[lo:hi])
    prob.priors = ()
    th = theta32(g.theta)
    th = {k: (v[..., lo:hi] if k not in ("bias", "alpha", "beta", "sigma_log") else v) for k, v in th.items()}
    out, grad, _ = O.loss_grad(prob, th, np.asarray(g.y[:, lo:hi], np.float64))
    return out["data"], grad["alpha"], grad["beta"], grad["bias"], float(grad["sigma_log"])


def oracle_planes_grad(args):
    """Per-voxel gradient of the brain-shaped volume's voxels with x in [i0, i1):
    the oracle on those voxels and every voxel within two x-planes of them,
    with the global |M| and box (exact on [i0, i1): the Eq. 7 prior couples
    voxels at most two steps apart, and no other term couples voxels)."""
    perturb_seed, i0, i1 = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    g = _full_workload(perturb_seed)
    x = g.coords[:, 0]
    lo, hi = np.searchsorted(x, i0 - 2), np.searchsorted(x, i1 + 2)
    c0, c1 = np.searchsorted(x, i0), np.searchsorted(x, i1)
    prob = oracle_problem(g, norm_count=g.n_vox, coords=g.coords[lo:hi])
    th = theta32(g.theta)
    th = {k: (v[..., lo:hi] if k not in ("bias", "alpha", "beta", "sigma_log") else v) for k, v in th.items()}
    _, grad, _ = O.loss_grad(prob, th, np.asarray(g.y[:, lo:hi], np.float64))
    return int(c0), int(c1), {k: grad[k][..., c0 - lo:c1 - lo] for k in ("s0", "logits", "v", "fin")}


def oracle_group(args):
    """Loss terms and gradient of one independent group (for a spawned pool)."""
    g, th = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    out, grad, _ = run_oracle(g, th)
    return out, grad


def two_ring(coords, shape, centres):
    """Indices of the voxels within two 6-neighbour steps of the centres."""
    grid = -np.ones(shape, dtype=np.int64)
    grid[tuple(coords.T)] = np.arange(coords.shape[0])
    keep = set()
    for c in centres:
        for dx in range(-2, 3):
            for dy in range(-2, 3):
                for dz in range(-2, 3):
                    if abs(dx) + abs(dy) + abs(dz) > 2:
                        continue
                    p = coords[c] + np.array([dx, dy, dz])
                    if np.all(p >= 0) and np.all(p < np.array(shape)):
                        v = grid[tuple(p)]
                        if v >= 0:
                            keep.add(int(v))
    return np.array(sorted(keep))
