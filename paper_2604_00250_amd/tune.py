"""Launch-shape autotuner for the fused pass, per (N, K, mode, learned-D) bucket.

For a problem resident on the GPU:

1. every candidate problem-wide shape (voxels per lane, measurement split,
   voxels per work item, per-variant or persistent launch) is planned with
   prism_problem_tune and timed with HIP events over a few whole fit
   iterations (prism_iteration_adam, the call a fit makes), and the fastest
   is kept;
2. when the problem has more than one bucket of groups, each bucket in turn
   (most expensive first) tries its own measurement split and item size (and
   voxels per lane outside the persistent launch) with every other bucket held
   at its current shape; a bucket keeps a new shape only if the whole
   iteration gets faster by more than `min_gain`.

The problem's parameters, Adam moments, step counter and status are restored
after timing.  Results are cached in a JSON file per bucket signature: the
device name, the library's build id and ABI version, whether the plan is
persistent, and the bucket's (N, K, mode, learned D), so a later problem with
the same buckets starts from the cached shapes instead of searching.

    best = autotune(state)                # state: problem.DeviceState
"""
from __future__ import annotations

import json
import os
from typing import Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "prism_mi355x_tune.json")


def bucket_key(b: dict) -> str:
    return f"N{b['n_meas']}_K{b['K']}_{b['mode']}_{'D' if b['learn_diffusivity'] else 'fixedD'}"


def candidates(prob) -> list:
    """Problem-wide shapes tried in the first phase."""
    V = int(prob.info.n_vox)
    out = []
    for vpl in (1, 2):
        for split in (0, 1, 2, 4):
            out.append(dict(vox_per_lane=vpl, n_split=split, item_vox=0, persistent=0))
    out.append(dict(vox_per_lane=1, n_split=0, item_vox=0, persistent=1))
    if prob.n_groups == 1 and V >= 262144:
        out += [dict(vox_per_lane=2, n_split=1, item_vox=1024, persistent=0),
                dict(vox_per_lane=1, n_split=1, item_vox=512, persistent=0)]
    return out


def bucket_candidates(persistent: bool) -> list:
    """Per-bucket shapes tried in the second phase (item sizes are whole block chunks)."""
    out = []
    for vpl in ((1,) if persistent else (1, 2)):
        for split in (0, 1, 2, 4):
            chunk = 64 * vpl * (4 // split) if split else 64 * vpl * 4
            for mult in ((0,) if split == 0 else (1, 2, 4)):
                out.append(dict(vox_per_lane=vpl, n_split=split, item_vox=mult * chunk))
    return out


def _time(state, reps: int) -> float:
    """Median milliseconds of one fused Adam iteration (state restored by the caller)."""
    import torch
    st = state
    for _ in range(2):
        st.iteration()
    torch.cuda.synchronize(st.device)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        st.iteration()
        e1.record()
        torch.cuda.synchronize(st.device)
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def _apply(state, launch: dict, buckets: list):
    state.prob.tune(**launch, buckets=buckets)
    state.resize_workspace()


def _load(cache):
    if cache and os.path.exists(cache):
        try:
            return json.load(open(cache))
        except (OSError, ValueError):
            return {}
    return {}


def _store(cache, db):
    if not cache:
        return
    os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, cache)


def autotune(state, reps: int = 5, cache: Optional[str] = DEFAULT_CACHE, cands: Optional[list] = None,
             per_bucket: bool = True, min_gain: float = 0.01, verbose: bool = False) -> dict:
    """Pick the fastest launch shape for `state`'s problem (problem-wide, then
    per bucket) and apply it.  Returns the chosen shapes, the timings and
    whether they came from the cache."""
    import torch
    from . import _lib as L
    from .fit import restore, snapshot
    prob = state.prob
    dev_name = torch.cuda.get_device_name(state.device)
    build = L.lib().prism_build_id().decode()
    prefix = f"{dev_name}|{build}|abi{L.lib().prism_abi_version()}"
    db = _load(cache)
    snap = snapshot(state)
    try:
        # phase 1: problem-wide shape (cached under the problem's bucket set)
        sigs = prob.buckets()
        whole_key = prefix + "|problem|" + ",".join(sorted(bucket_key(b) for b in sigs))
        if cands is None and whole_key in db:
            best, best_ms, trials, cached = db[whole_key]["launch"], db[whole_key]["ms"], [], True
        else:
            results = []
            for c in cands or candidates(prob):
                try:
                    _apply(state, c, [])
                except L.PrismError as ex:  # not a valid shape for this problem
                    if verbose:
                        print("skip", c, ex)
                    continue
                ms = _time(state, reps)
                restore(state, snap)
                results.append((ms, c))
                if verbose:
                    print(f"{c} {ms:.4f} ms", flush=True)
            if not results:
                raise RuntimeError("autotune: no candidate launch shape is valid for this problem")
            results.sort(key=lambda r: r[0])
            best_ms, best = results[0]
            trials = [dict(launch=c, ms=m) for m, c in results]
            cached = False
            db[whole_key] = dict(launch=best, ms=best_ms)
        _apply(state, best, [])
        chosen = []
        bucket_trials = []
        if per_bucket and len(sigs) > 1:
            persistent = bool(best.get("persistent", 0))
            shape_keys = ("vox_per_lane", "n_split", "item_vox")
            # each bucket's shape under the problem-wide one (no override)
            base = {bucket_key(b): {k: b[k] for k in shape_keys} for b in prob.buckets()}
            # cached per-bucket shapes first; only those that differ become overrides
            searched = set()
            for b in sigs:
                k = f"{prefix}|{'persistent' if persistent else 'variants'}|{bucket_key(b)}"
                if k in db:
                    searched.add(bucket_key(b))
                    if db[k]["shape"] != base[bucket_key(b)]:
                        chosen.append(dict(b, **db[k]["shape"]))
            if chosen:
                try:
                    _apply(state, best, chosen)
                except L.PrismError:
                    chosen = []
                    _apply(state, best, [])
            cur_ms = _time(state, reps)
            restore(state, snap)
            if len(searched) < len(sigs) or cands is not None:
                # coordinate descent over the buckets without a cached shape, most work first
                work = {}
                for g, gi in zip(prob.groups, prob.ginfo):
                    key = bucket_key(dict(n_meas=int(gi.n_meas), K=g.K, mode=g.mode,
                                          learn_diffusivity=bool(g.learn_diffusivity)))
                    work[key] = work.get(key, 0) + int(gi.n_vox) * int(gi.n_meas) * (g.K + 2)
                done = set() if cands is not None else searched
                todo = sorted((b for b in sigs if bucket_key(b) not in done), key=lambda b: -work[bucket_key(b)])
                for b in todo:
                    kb = bucket_key(b)
                    best_shape, best_b_ms = None, cur_ms
                    for shape in bucket_candidates(persistent):
                        if shape == base[kb]:
                            continue  # the problem-wide shape itself: already timed as cur_ms
                        trial = [c for c in chosen if bucket_key(c) != kb] + [dict(b, **shape)]
                        try:
                            _apply(state, best, trial)
                        except L.PrismError:
                            continue
                        ms = _time(state, reps)
                        restore(state, snap)
                        bucket_trials.append(dict(bucket=kb, shape=shape, ms=ms))
                        if ms < best_b_ms * (1.0 - min_gain):
                            best_shape, best_b_ms = shape, ms
                    if best_shape is not None:
                        chosen = [c for c in chosen if bucket_key(c) != kb] + [dict(b, **best_shape)]
                        cur_ms = best_b_ms
                    # the shape kept for this bucket (the problem-wide one when nothing beat it)
                    kept = best_shape or base[kb]
                    db[f"{prefix}|{'persistent' if persistent else 'variants'}|{kb}"] = dict(shape=kept)
                    if verbose:
                        print(f"bucket {kb}: {kept} -> {cur_ms:.4f} ms", flush=True)
                    _apply(state, best, chosen)
                cached = False
            _apply(state, best, chosen)
            best_ms = cur_ms
        _store(cache, db)
    finally:
        restore(state, snap)
    return dict(launch=best, buckets=chosen, ms=best_ms, trials=trials, bucket_trials=bucket_trials,
                cached=cached, build=build)
