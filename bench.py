"""Benchmark of the PRISM fused analysis-by-synthesis iteration on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload: the whole-brain-shaped volume (145x174x145 grid, ~741k masked
voxels, N = 288 three-shell measurements, K = 3, MSE mode, calibration on at
identity, all priors), synthetic data from paper_2604_00250_amd.inputs.
A step is one full iteration through prism_iteration_adam: the Eq. 7
kernels, the fused forward + adjoint pass with the Adam update of every
per-voxel parameter in its epilogue, the calibration reductions and the
calibration vector's Adam update, with y, parameters, moments and workspace
resident in HBM.  Prints one JSON line.

Before the timed region (untimed): the roofline microbenchmark, --warmup
iterations, then iterations for --warmup-seconds of wall time (the GPU's
clocks ramp up over the first second or so of work).

Extra legs (on by default, rank 0 only):
  roofline       fused-kernel time from HIP events recorded by the library
                 around each launch on the timed stream, against the VALU
                 issue roofline built from the microbenchmarked exp cost;
  graph          the same iteration captured as a HIP graph and replayed;
  fit            a whole fit of --fit-iterations graph-replayed iterations
                 from the initial parameters (loss history, final MSE);
  cpu_baseline   the FP64 oracle on a bounded sample of the same volume, on
                 one host core and on the host cores (a process pool, one
                 thread each), with the CPU model and core counts;
  torch_autograd the same objective written as plain per-op PyTorch FP32
                 autograd (+ torch.optim.Adam) on the same GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s (fwd+adjoint, 288 meas, K=3) fused HIP vs PyTorch autograd; %VALU"

# Algorithmic work of one (voxel, measurement) pair of the fused pass at K = 3,
# MSE, fixed diffusivities, as the roofline counts it: the figure derived from
# the method's steps before any kernel was written (forward 10K + 8 VALU, adjoint
# 12K + 10, 2K exps) and kept fixed as the implementation changes, so that
# roofline fractions stay comparable across versions.
ALG_VALU_PER_PAIR = 84
# The fewest operations the implementation's algebra needs for the same pair
# (every operation of Eq. 3-6, the data term and the adjoint counted once, an
# FMA as one, fused wherever the algebra allows, per-voxel factors such as the
# bias field, each fibre's fraction and f_intra applied once per voxel; a fibre's
# attenuation taken as f_in e1 + (1 - f_in) e12 with e1 and e12 = e1 e2 one exp
# each, so that e2 is never formed and the f_intra and log-bias adjoints follow
# per voxel from the per-fibre sums of dS e1 and dS e12; with fixed
# diffusivities the staged gradient direction carries sqrt(b Dpar log2 e), so
# that e1 = exp2(-cs^2) with cs the scaled cosine, and the adjoint's constant
# -2 ln 2 / Dpar sits in the per-voxel direction factors):
#   forward: mixture start 3; per fibre scaled cosine 3, its square 1, the e12
#     exponent 1, two weighted adds into S 2 (7K)                     -> 7K + 3
#   data term: beta - y 1, residual (gain S + (beta - y)) 1, squared-residual
#     accumulate 1                                                      -> 3
#   adjoint: seed S 1 (the alpha_n sum's input), dS 1, the two direction
#     factors times dS 2, isotropic 3; per fibre the sums of dS e1 and dS e12 2,
#     a2 e12 1, a1 e1 + a2 e12 1, times cs 1, direction 3 (8K)          -> 8K + 7
#   total 15K + 13 = 58 VALU and 2K = 6 exps at K = 3; reported as frac_min_count.
MIN_VALU_PER_PAIR = 58
ALG_EXP_PER_PAIR = 6
# At b = 0 every attenuation is exactly 1 and the kernel runs whole 16-measurement
# tiles of an acquisition's leading b = 0 measurements with the data term and the
# calibration adjoints only: beta - y, residual, squared-residual accumulate,
# seed x S (the alpha_n sum's input), the compartments' adjoint accumulate -> 5
# VALU, no exp.  The frozen count above prices every pair alike; frac_b0_aware
# prices these pairs at this count instead.
B0_VALU_PER_PAIR = 5
B0_TILE = 16
# Algorithmic HBM bytes of one voxel of the fused pass as the timed iteration runs
# it (prism_iteration_adam: Adam inside the pass): y (4N) + theta read (4P) + Adam
# moments read (8P) + theta and moments written (12P)
N_MEAS, P_VOX = 288, 17
ALG_BYTES_PER_VOXEL = 4 * N_MEAS + 24 * P_VOX
# MI355X issue capacity: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz lane-instruction slots / s
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------
# plain PyTorch autograd baseline of the same objective (FP32, per-op)
# ----------------------------------------------------------------------------

def torch_objective(T, th, y, G, b, Phi, nbr, cnt, M, K, consts):
    """Eq. 3-8 + priors of Sec. 2.4 with torch ops; th holds leaf tensors."""
    torch = T
    S0 = torch.nn.functional.softplus(th["s0"])
    f = torch.softmax(th["logits"], dim=0)
    d = th["v"] / th["v"].norm(dim=1, keepdim=True)
    fin = torch.sigmoid(th["fin"])
    logB = Phi.t() @ th["bias"]
    S = (f[0][None] * torch.exp(-b * consts["d_csf"]) + f[1][None] * torch.exp(-b * consts["d_gm"])
         + f[K + 2][None] * torch.exp(-b * consts["d_res"]))
    for k in range(K):
        c = G @ d[k]
        c2 = c * c
        e1 = torch.exp(-b * consts["d_par"] * c2)
        e2 = torch.exp(-b * consts["d_perp"] * (1.0 - c2))
        S = S + f[2 + k][None] * (fin[None] * e1 + (1.0 - fin[None]) * e1 * e2)
    yhat = torch.exp(th["alpha"])[:, None] * torch.exp(logB)[None] * S0[None] * S + th["beta"][:, None]
    data = ((yhat - y) ** 2).sum() / M
    fpad = torch.cat([f, torch.zeros_like(f[:, :1])], 1)
    mean = fpad[:, nbr].sum(-1) / cnt.clamp(min=1)[None]
    r = torch.where(cnt[None] > 0, f - mean, torch.zeros_like(f))
    a = r.abs()
    dl = consts["huber_delta"]
    spatial = torch.where(a <= dl, 0.5 * r * r, dl * (a - 0.5 * dl)).sum() * consts["lam_sp"] / M
    rep = 0.0
    fw = f[2:2 + K]
    for i in range(K):
        for j in range(i + 1, K):
            rep = rep + (fw[i] * fw[j] * (d[i] * d[j]).sum(0).abs()).sum()
    rep = rep * consts["lam_rep"] / M
    sparse = (fw * (fw < consts["tau_sparse"]).to(fw.dtype)).sum() * consts["lam_sparse"] / M
    cal = (consts["lam_alpha"] * (th["alpha"] ** 2).sum() + consts["lam_beta"] * (th["beta"] ** 2).sum()
           + consts["lam_bias"] * (th["bias"] ** 2).sum())
    return data + spatial + rep + sparse + cal


def torch_baseline(g, y_dev, steps=5, warmup=2):
    import numpy as np
    import torch
    dev = y_dev.device
    consts = dict(d_csf=3.0, d_gm=0.9, d_res=0.2, d_par=1.7, d_perp=0.4, lam_sp=0.01, huber_delta=0.05,
                  lam_rep=0.01, lam_sparse=0.02, tau_sparse=0.15, lam_alpha=0.01, lam_beta=0.01, lam_bias=0.01)
    V = g.n_vox
    coords = g.coords
    shape = g.shape
    xi = np.zeros((V, 3))
    for a in range(3):
        xi[:, a] = (2.0 * coords[:, a] - (shape[a] - 1)) / (shape[a] - 1)
    x_, y_, z_ = xi.T
    Phi = np.stack([np.ones(V), x_, y_, z_, x_ * x_, y_ * y_, z_ * z_, x_ * y_, x_ * z_, y_ * z_])
    grid = -np.ones(shape, dtype=np.int64)
    grid[tuple(coords.T)] = np.arange(V)
    nbr = np.full((V, 6), V, dtype=np.int64)
    for j, (dx, dy, dz) in enumerate([(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]):
        c = coords + np.array([dx, dy, dz])
        ok = np.all((c >= 0) & (c < np.array(shape)), 1)
        idx = np.full(V, -1)
        idx[ok] = grid[tuple(c[ok].T)]
        nbr[:, j] = np.where(idx >= 0, idx, V)
    cnt = (nbr < V).sum(1)
    f32 = dict(dtype=torch.float32, device=dev)
    th = {k: torch.tensor(np.asarray(v, dtype=np.float32), **f32).requires_grad_(True)
          for k, v in g.theta.items() if k != "sigma_log"}
    G = torch.tensor(g.acq.bvec, **f32)
    bb = torch.tensor(g.acq.bval, **f32)[:, None]
    Phi_t = torch.tensor(Phi, **f32)
    nbr_t = torch.tensor(nbr, device=dev)
    cnt_t = torch.tensor(cnt, **f32)
    opt = torch.optim.Adam(list(th.values()), lr=1e-2)

    def fwd_bwd():
        for p in th.values():
            p.grad = None
        loss = torch_objective(torch, th, y_dev, G, bb, Phi_t, nbr_t, cnt_t, float(V), g.K, consts)
        loss.backward()
        return loss

    res = {}
    for label, with_opt in (("fwd_adjoint", False), ("iteration", True)):
        for _ in range(warmup):
            fwd_bwd()
            if with_opt:
                opt.step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fwd_bwd()
            if with_opt:
                opt.step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[label] = dict(ms=ms, value=V / (ms * 1e-3))
    res["peak_mem_GB"] = torch.cuda.max_memory_allocated(dev) / 1e9
    del th, opt
    torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------------------------
# FP64 oracle on the host cores (bounded sample)
# ----------------------------------------------------------------------------

_CPU_JOB = {}


def _oracle_chunk(args):
    lo, hi = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    threadpool_limits(1)
    g = _CPU_JOB["g"]
    prob = O.Problem(coords=g.coords[lo:hi], shape=g.shape, bval=g.acq.bval, bvec=g.acq.bvec, K=g.K,
                     mode=g.mode, bias=g.bias, priors=tuple(g.priors), norm_count=g.n_vox)
    th = {k: (np.asarray(v, np.float64)[..., lo:hi] if k not in ("bias", "alpha", "beta", "sigma_log")
              else np.asarray(v, np.float64)) for k, v in g.theta.items()}
    t = time.perf_counter()
    O.loss_grad(prob, th, np.asarray(g.y[:, lo:hi], np.float64))
    return hi - lo, time.perf_counter() - t


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


# Worker processes of the all-core leg: the host cores this process may run on,
# but at most one GPU's share of a shared host (16 cores per GPU on the boxes
# this runs on), stated in the record as cpu_share.
CPU_SHARE = 16


def cpu_baseline(g, one_core_s=4.0, all_core_s=12.0, chunk=4096):
    """The oracle's loss_grad over chunks of the volume's voxels, timed twice:
    one process with one thread (1-core figure, about `one_core_s` seconds),
    then one single-threaded process per core (all-core figure, about
    `all_core_s` seconds of wall time, chunks cycling over the volume)."""
    import multiprocessing as mp
    visible = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = visible
    cores = max(1, min(allowed, CPU_SHARE))
    _CPU_JOB["g"] = g
    n_avail = max(1, g.n_vox // chunk)
    # 1 core: chunks in this process, in order, until the time budget is spent
    t = time.perf_counter()
    vox1 = 0
    i = 0
    while time.perf_counter() - t < one_core_s or i == 0:
        n, _ = _oracle_chunk(((i % n_avail) * chunk, (i % n_avail + 1) * chunk))
        vox1 += n
        i += 1
    wall1 = time.perf_counter() - t
    per_chunk = wall1 / i
    # all cores: enough chunks for about all_core_s of wall time
    n_chunks = max(cores, int(all_core_s * cores / per_chunk))
    jobs = [((k % n_avail) * chunk, (k % n_avail + 1) * chunk) for k in range(n_chunks)]
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(cores) as pool:
        done = pool.map(_oracle_chunk, jobs, chunksize=1)
    wall = time.perf_counter() - t
    vox = sum(d[0] for d in done)
    return dict(value=vox / wall, unit="voxel-iters/s", cores=cores, kind="oracle",
                sample=f"{n_chunks} chunks x {chunk} voxels of the volume, cycling over its "
                       f"{n_avail} chunks ({vox} voxel-iterations of loss+gradient, N=288, K=3, FP64 "
                       f"NumPy, one single-threaded process per core), {wall:.1f} s wall",
                one_core=dict(value=vox1 / wall1, cores=1, chunks=i, seconds=wall1,
                              sample=f"{i} chunks x {chunk} voxels in one single-threaded process"),
                cpu_model=_cpu_model(), nproc=visible, cores_allowed=allowed, cpu_share=CPU_SHARE,
                seconds_per_chunk_single_core=per_chunk)


# ----------------------------------------------------------------------------
# main
# ----------------------------------------------------------------------------

def stored_traffic(workload: str):
    """HBM bytes per k_pass dispatch from the committed counter summary, if it
    was taken with the current kernel sources (else None)."""
    import re
    from paper_2604_00250_amd.profile_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"k_pass_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_dispatch: ([0-9.e+]+)", text)
    h = re.search(r"kernel_source_sha1: ([0-9a-f]+)", text)
    if not m or not h or h.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


def parse_launch(text):
    if not text:
        return None
    vals = [int(x) for x in text.split(",")]
    keys = ("vox_per_lane", "n_split", "item_vox", "persistent", "max_blocks", "stagger", "concurrent")
    return dict(zip(keys, vals))


def _oracle_fit(g, iterations, lr, budget_s):
    """The oracle's own fit (its loss_grad and Adam in FP64, one process, one
    thread) from the workload's initial parameters, for at most `budget_s`
    seconds; returns (iterations done, seconds, loss after the last one)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    prob = O.Problem(coords=g.coords, shape=tuple(g.shape), bval=np.asarray(g.acq.bval, np.float64),
                     bvec=np.asarray(g.acq.bvec, np.float64), K=g.K, mode=g.mode, bias=g.bias,
                     learn_diffusivity=g.learn_diffusivity, neighbourhood=g.neighbourhood,
                     priors=tuple(g.priors))
    th = {k: np.asarray(np.asarray(v, np.float32), np.float64) for k, v in g.theta.items()}
    m = {k: np.zeros_like(v) for k, v in th.items()}
    v2 = {k: np.zeros_like(v) for k, v in th.items()}
    y = np.asarray(g.y, np.float64)
    t0 = time.perf_counter()
    done, loss = 0, None
    with threadpool_limits(1):
        while done < iterations and (done == 0 or time.perf_counter() - t0 < budget_s):
            out, grad, _ = O.loss_grad(prob, th, y)
            loss = out["total"]
            for k in th:
                th[k], m[k], v2[k] = O.adam_step(th[k], grad[k], m[k], v2[k], done + 1, lr=lr)
            done += 1
    return done, time.perf_counter() - t0, loss


def bench_patches(args):
    """Whole fits of the two single-patch workloads on the GPU (the iteration
    captured as a HIP graph and replayed), beside the oracle's own fit on one
    host core: one 8^3 patch (N = 33, K = 3, MSE, 100 Adam steps) and one 16^3
    patch (N = 288, K = 3, Rician NLL with calibration, 500 iterations; the
    oracle runs a bounded number of its iterations and the rate is scaled)."""
    import torch
    from paper_2604_00250_amd import _lib as L
    from paper_2604_00250_amd import inputs as I
    from paper_2604_00250_amd.fit import fit
    from paper_2604_00250_amd.problem import DeviceState, Problem
    res = []
    for w, budget in ((I.patch8_crossings(priors=I.PRIOR_NAMES), 30.0), (I.patch16_hcp(), 20.0)):
        g = w.groups[0]
        prob = Problem([g])
        st = DeviceState(prob, ys=[g.y], thetas=[g.theta], device="cuda:0")
        fit(st, 20, lr=w.lr)                          # warm-up fit (captures, replays, restores nothing)
        st.set_params([g.theta])
        st.reset_optimizer()
        torch.cuda.synchronize()
        t = time.perf_counter()
        hist = fit(st, w.iterations, lr=w.lr)
        wall = time.perf_counter() - t
        h = hist[:, 0].cpu().numpy()
        n_done, cpu_s, cpu_loss = _oracle_fit(g, w.iterations, w.lr, budget)
        res.append(dict(workload=w.name, voxels=g.n_vox, measurements=g.acq.n, iterations=w.iterations,
                        gpu_fit_s=wall, gpu_ms_per_iteration=wall / w.iterations * 1e3,
                        gpu_voxel_iters_per_s=g.n_vox * w.iterations / wall,
                        loss_first=float(h[0, L.LOSS_TOTAL]), loss_last=float(h[-1, L.LOSS_TOTAL]),
                        status=int(st.status.item()),
                        oracle_iterations_timed=n_done, oracle_s=cpu_s,
                        oracle_fit_s=cpu_s / n_done * w.iterations,
                        oracle_fit_s_note="measured" if n_done == w.iterations else
                        f"scaled from {n_done} of {w.iterations} iterations",
                        oracle_voxel_iters_per_s=g.n_vox * n_done / cpu_s,
                        oracle_loss_at_last_timed_iteration=float(cpu_loss),
                        gpu_loss_at_same_iteration=float(h[n_done - 1, L.LOSS_TOTAL])))
        log(f"{w.name}: GPU {wall * 1e3:.1f} ms for {w.iterations} iterations; oracle {cpu_s:.1f} s for {n_done}")
        del st
    out = {"metric": METRIC, "value": None, "unit": "s per fit", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f32", "config": {"workload": "patch fits"}, "fits": res}
    print(json.dumps(out), flush=True)


def tuned_report(tuned):
    """The autotuner's choices: the problem-wide shape with its time and the
    runners-up, then each bucket's shape (an override where one beat the
    problem-wide shape by more than 1%) with the best iteration time of its trials."""
    out = {k: tuned[k] for k in ("launch", "cached", "ms", "build") if k in tuned}
    if tuned.get("trials"):
        out["problem_wide_trials"] = tuned["trials"]
        out["best_problem_wide_ms"] = tuned["trials"][0]["ms"]
    out["bucket_overrides"] = tuned.get("buckets", [])
    per = {}
    for t in tuned.get("bucket_trials", []):
        b = per.setdefault(t["bucket"], dict(trials=0, best_ms=float("inf"), best_shape=None))
        b["trials"] += 1
        if t["ms"] < b["best_ms"]:
            b["best_ms"], b["best_shape"] = t["ms"], t["shape"]
    out["bucket_search"] = per
    return out


def bench_batched(args):
    """4096 independent patches of uneven size (edge log-uniform 4-24), N in
    {33, 96, 288}, K in 1..5, MSE or NLL, in one problem; the launch shape comes
    from the autotuner (persistent or per-variant launches)."""
    import numpy as np
    import torch
    from paper_2604_00250_amd import inputs as I
    from paper_2604_00250_amd.problem import DeviceState, Problem
    from paper_2604_00250_amd.tune import autotune
    t0 = time.time()
    w = I.batched_patches()
    log(f"workload {w.name}: {len(w.groups)} patches, {w.n_vox} voxels, generated in {time.time() - t0:.1f} s")
    prob = Problem(w.groups)
    st = DeviceState(prob, ys=[g.y for g in w.groups], thetas=[g.theta for g in w.groups], device="cuda:0")
    launch = parse_launch(args.launch)
    if launch:
        prob.tune(**launch)
        st.resize_workspace()
        tuned = dict(launch=launch, cached=False)
    else:
        tuned = autotune(st, cache=None, reps=3)
        log(f"autotuner: {tuned['launch']} ({tuned['ms']:.3f} ms with {len(tuned['buckets'])} bucket overrides); "
            + "; ".join(f"{t['launch']}: {t['ms']:.3f}" for t in tuned["trials"]))
    for _ in range(args.warmup):
        st.iteration(lr=w.lr)
    warm = gpu_warmup(st, w.lr, args.warmup_seconds) if args.warmup_seconds > 0 else None
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        st.iteration(lr=w.lr)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    V = w.n_vox
    pairs = sum(g.n_vox * g.acq.n for g in w.groups)
    out = {
        "metric": METRIC, "value": V / (ms * 1e-3), "unit": "voxel-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "patches": len(w.groups), "voxels": V, "pairs": pairs,
                   "launch": prob.launch(), "step": "prism_iteration_adam (fused pass with the per-voxel Adam update, then Adam on the calibration)"},
        "pairs_per_s": pairs / (ms * 1e-3),
        "autotune": tuned_report(tuned),
        "gpu_warmup": warm,
        "status": int(st.status.cpu().item()),
    }
    print(json.dumps(out), flush=True)


def gpu_warmup(st, lr, seconds):
    """Untimed iterations for a fixed wall time, whatever --warmup asks: the
    GPU's clocks ramp up over the first second or so of sustained work."""
    import torch
    n = 0
    t = time.perf_counter()
    while True:
        for _ in range(50):
            st.iteration(lr=lr)
        n += 50
        torch.cuda.synchronize()
        if time.perf_counter() - t >= seconds:
            return dict(seconds=time.perf_counter() - t, iterations=n)


def graph_leg(st, lr, steps):
    """The same iteration captured once as a HIP graph and replayed `steps`
    times (after a few untimed replays)."""
    import torch
    from paper_2604_00250_amd.fit import Loop, restore, snapshot
    snap = snapshot(st)
    loop = Loop(st, lr=lr)
    loop.capture()
    loop.replay(10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    loop.replay(steps)
    e1.record()
    torch.cuda.synchronize()
    restore(st, snap)
    return e0.elapsed_time(e1) / steps


def fit_leg(st, lr, iterations, N):
    """A whole fit from the initial parameters with the iteration captured as a
    HIP graph and replayed `iterations` times; the loss history stays on the
    device until the end."""
    import numpy as np
    import torch
    from paper_2604_00250_amd import _lib as L
    from paper_2604_00250_amd.fit import Loop, restore, snapshot
    snap = snapshot(st)
    loop = Loop(st, lr=lr, history=iterations)
    loop.capture()                    # runs one iteration on the way: start again from the snapshot
    restore(st, snap)
    loop.hist.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    loop.replay(iterations)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    hist = loop.hist[:, 0].cpu().numpy()             # [iterations][terms]
    st.loss_grad()                                   # the loss at the final parameters
    torch.cuda.synchronize()
    final = st.loss_host()[0]
    status = int(st.status.cpu().item())
    marks = sorted({0, 1, 10, 100, 250, 500, iterations - 1} & set(range(iterations)))
    data_i = L.LOSS_TERMS.index("data")
    total = hist[:, L.LOSS_TOTAL]
    best = float(total.min())
    within = np.nonzero(total <= 1.01 * best)[0]
    restore(st, snap)
    return dict(iterations=iterations, ms_total=ms, ms_per_iteration=ms / iterations,
                voxel_iters_per_s=None, loss_total={int(k): float(total[k]) for k in marks},
                data_mse_per_measurement={int(k): float(hist[k, data_i] / N) for k in marks},
                final_loss_total=float(final[L.LOSS_TOTAL]),
                final_data_mse_per_measurement=float(final[data_i] / N),
                first_iteration_within_1pct_of_best=int(within[0]) if within.size else None,
                status=status)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--warmup-seconds", type=float, default=2.0,
                    help="untimed iterations for this long before the timed region, whatever --warmup is")
    ap.add_argument("--fit-iterations", type=int, default=1000,
                    help="graph-captured fit from the initial parameters (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-torch-baseline", action="store_true")
    ap.add_argument("--no-microbench", action="store_true")
    ap.add_argument("--no-fwd-adjoint", action="store_true",
                    help="skip the prism_loss_grad-only leg (counter runs see the timed kernel only)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay leg")
    ap.add_argument("--launch", type=str, default="",
                    help="vox_per_lane,n_split,item_vox[,persistent[,max_blocks[,stagger[,concurrent]]]]")
    ap.add_argument("--workload", choices=("brain", "batched", "patches"), default="brain",
                    help="brain: the 743k-voxel volume (the metric's configuration); batched: 4096 "
                         "independent uneven patches in one problem, autotuned launch; patches: whole "
                         "fits of the 8^3 and 16^3 patch workloads beside the oracle's")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures the single-GPU path only: the fused pass runs on one MI355X "
              "and sharding over several GPUs is not implemented. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2604_00250_amd import inputs as I

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "patches":
        return bench_patches(args)
    t0 = time.time()
    w = I.brain_volume()
    g = w.groups[0]
    log(f"workload {w.name}: {g.n_vox} voxels, N={g.acq.n}, K={g.K}, generated in {time.time() - t0:.1f} s")
    # the CPU leg runs first, in worker processes forked before this process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(g)
    if cpu:
        log(f"cpu baseline: {cpu['value']:.4g} voxel-iters/s on {cpu['cores']} cores "
            f"({cpu['one_core']['value']:.4g} on one)")

    import torch
    from paper_2604_00250_amd import _lib as L
    from paper_2604_00250_amd.fit import restore, snapshot
    from paper_2604_00250_amd.problem import DeviceState, Problem
    launch = parse_launch(args.launch)
    prob = Problem([g], launch=launch)
    st = DeviceState(prob, ys=[g.y], thetas=[g.theta], device="cuda:0")
    initial = snapshot(st)
    V = g.n_vox

    # untimed GPU legs first: the roofline microbenchmark, then the fixed-duration warm-up
    mb = None
    if not args.no_microbench:
        try:
            from paper_2604_00250_amd import microbench
            mb = microbench.run()
        except Exception as ex:  # the roofline still reports with q = 1
            log(f"microbenchmark failed: {ex}")
    for _ in range(args.warmup):
        st.iteration(lr=w.lr)
    warm = gpu_warmup(st, w.lr, args.warmup_seconds) if args.warmup_seconds > 0 else None
    torch.cuda.synchronize()
    prob.profile(True, max_launches=args.steps + 4)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        st.iteration(lr=w.lr)
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    k_ms_total, k_launches = prob.profile_read()
    prob.profile(False)
    k_ms = k_ms_total / max(k_launches, 1)
    status = int(st.status.cpu().item())
    loss = st.loss_host()[0]
    if status != 0 or not np.isfinite(loss[L.LOSS_TOTAL]):
        log(f"WARNING: status {status}, loss {loss}")

    # fwd+adjoint only (prism_loss_grad), same state
    ms_fa = None
    if not args.no_fwd_adjoint:
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            st.loss_grad()
        e1.record()
        torch.cuda.synchronize()
        ms_fa = e0.elapsed_time(e1) / args.steps
    ms_graph = None if args.no_graph else graph_leg(st, w.lr, args.steps)
    fit = None
    if args.fit_iterations > 0:
        restore(st, initial)
        fit = fit_leg(st, w.lr, args.fit_iterations, g.acq.n)
        fit["voxel_iters_per_s"] = V / (fit["ms_per_iteration"] * 1e-3)
        log(f"fit: {fit['iterations']} graph-replayed iterations, {fit['ms_per_iteration']:.4f} ms each; "
            f"loss {fit['loss_total']}")

    pairs = V * g.acq.n
    q = mb["q_exp"] if mb else 1.0
    slots = pairs * (ALG_VALU_PER_PAIR + q * ALG_EXP_PER_PAIR)
    achieved = slots / (k_ms * 1e-3)
    nb0 = 0
    while nb0 < g.acq.n and g.acq.bval[nb0] == 0.0:
        nb0 += 1
    b0_short = (nb0 // B0_TILE) * B0_TILE if prob.launch()["n_split"] == 1 else 0
    slots_b0 = V * (b0_short * B0_VALU_PER_PAIR
                    + (g.acq.n - b0_short) * (ALG_VALU_PER_PAIR + q * ALG_EXP_PER_PAIR))
    traffic = stored_traffic(w.name)
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                    frac=achieved / PEAK_SLOTS, traffic=traffic,
                    traffic_vs_algorithmic=(traffic / (ALG_BYTES_PER_VOXEL * V)) if traffic else None,
                    kernel="k_pass<3,MSE,fixedD>", kernel_ms=k_ms, launches=k_launches,
                    alg_slots_per_pair=ALG_VALU_PER_PAIR + q * ALG_EXP_PER_PAIR, q_exp=q,
                    frac_min_count=pairs * (MIN_VALU_PER_PAIR + q * ALG_EXP_PER_PAIR) / (k_ms * 1e-3)
                    / PEAK_SLOTS,
                    min_slots_per_pair=MIN_VALU_PER_PAIR + q * ALG_EXP_PER_PAIR,
                    frac_b0_aware=slots_b0 / (k_ms * 1e-3) / PEAK_SLOTS,
                    b0_pairs_per_voxel_short=b0_short,
                    hbm_GBps=ALG_BYTES_PER_VOXEL * V / (k_ms * 1e-3) / 1e9,
                    hbm_frac=ALG_BYTES_PER_VOXEL * V / (k_ms * 1e-3) / PEAK_HBM)
    out = {
        "metric": METRIC,
        "value": V / (ms * 1e-3),
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "voxels": V, "grid": list(g.shape), "measurements": g.acq.n,
                   "K": g.K, "mode": "mse", "priors": list(g.priors), "bias": g.bias,
                   "launch": prob.launch(), "step": "prism_iteration_adam (fused pass with the per-voxel Adam update, then Adam on the calibration)"},
        "gpu_warmup": dict(warm or {}, microbench_first=mb is not None,
                           note="untimed: the microbenchmark, then --warmup iterations, then iterations "
                                "for --warmup-seconds of wall time, before the timed region"),
        "fwd_adjoint": {"value": V / (ms_fa * 1e-3), "ms": ms_fa} if ms_fa else None,
        "graph": {"value": V / (ms_graph * 1e-3), "ms": ms_graph,
                  "note": "the same iteration captured once as a HIP graph, replayed --steps times"}
        if ms_graph else None,
        "roofline": roofline,
        "wall_s_timed": t_wall,
        "loss": float(loss[L.LOSS_TOTAL]),
        "status": status,
        "paper_context": "~741k voxels x 100 iterations per slab in ~12 min on one RTX A6000 "
                         "(about 1e5 voxel-iters/s, MSE; a different machine and workload)",
    }
    if fit:
        out["fit"] = fit
    if mb:
        out["microbench"] = mb
    if not args.no_torch_baseline:
        try:
            tb = torch_baseline(g, st.y[: g.acq.n * V].view(g.acq.n, V))
            out["torch_autograd"] = dict(value=tb["iteration"]["value"], ms=tb["iteration"]["ms"],
                                         fwd_adjoint_value=tb["fwd_adjoint"]["value"],
                                         fwd_adjoint_ms=tb["fwd_adjoint"]["ms"],
                                         peak_mem_GB=tb["peak_mem_GB"],
                                         speedup_iteration=out["value"] / tb["iteration"]["value"],
                                         speedup_fwd_adjoint=out["fwd_adjoint"]["value"] / tb["fwd_adjoint"]["value"])
        except Exception as ex:
            log(f"torch baseline failed: {ex}")
            out["torch_autograd"] = {"error": str(ex)[:200]}
    del st
    torch.cuda.empty_cache()
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
