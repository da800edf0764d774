"""Launch-shape autotuner for the fused pass.

For a problem resident on the GPU, every candidate launch shape
(voxels per lane, measurement split, voxels per work item, per-variant or
persistent launch) is planned with prism_problem_tune, timed with HIP events
over a few calls of prism_loss_grad, and the fastest is kept.  Results are
cached in a JSON file keyed by the problem's signature (group count, voxel
count and the histogram of (N, K, mode, learned-D) buckets) and the GPU name,
so a later run on the same shapes skips the search.

    best = autotune(state)                # state: problem.DeviceState
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "prism_mi355x_tune.json")


def signature(prob) -> str:
    hist = {}
    for g, gi in zip(prob.groups, prob.ginfo):
        key = (int(gi.n_meas), int(g.K), g.mode, bool(g.learn_diffusivity))
        a = hist.setdefault(key, [0, 0])
        a[0] += 1
        a[1] += int(gi.n_vox)
    items = sorted((f"{k}", v) for k, v in hist.items())
    raw = json.dumps([prob.n_groups, int(prob.info.n_vox), items])
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def candidates(prob) -> list:
    V = int(prob.info.n_vox)
    out = []
    for vpl in (1, 2):
        for split in (0, 1, 2, 4):
            for iv in (0,):
                out.append(dict(vox_per_lane=vpl, n_split=split, item_vox=iv, persistent=0))
    out.append(dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1))
    if prob.n_groups == 1 and V >= 262144:
        out += [dict(vox_per_lane=2, n_split=1, item_vox=1024, persistent=0),
                dict(vox_per_lane=1, n_split=1, item_vox=512, persistent=0)]
    return out


def _time(state, reps: int) -> float:
    import torch
    st = state
    for _ in range(2):
        st.loss_grad()
    torch.cuda.synchronize(st.device)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        st.loss_grad()
        e1.record()
        torch.cuda.synchronize(st.device)
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def autotune(state, reps: int = 5, cache: Optional[str] = DEFAULT_CACHE, cands: Optional[list] = None,
             verbose: bool = False) -> dict:
    """Pick the fastest launch shape for `state`'s problem and apply it."""
    import torch
    prob = state.prob
    dev_name = torch.cuda.get_device_name(state.device)
    sig = signature(prob)
    db = {}
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
        except (OSError, ValueError):
            db = {}
    key = f"{dev_name}|{sig}"
    if cands is None and key in db:
        best = db[key]["launch"]
        prob.tune(**best)
        state.resize_workspace()
        return dict(db[key], cached=True)
    results = []
    for c in cands or candidates(prob):
        try:
            prob.tune(**c)
        except Exception as ex:  # an invalid shape for this problem
            if verbose:
                print("skip", c, ex)
            continue
        state.resize_workspace()
        ms = _time(state, reps)
        results.append((ms, c))
        if verbose:
            print(f"{c} {ms:.4f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    prob.tune(**best)
    state.resize_workspace()
    entry = dict(launch=best, ms=best_ms, trials=[dict(launch=c, ms=m) for m, c in results])
    if cache:
        db[key] = entry
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return dict(entry, cached=False)
