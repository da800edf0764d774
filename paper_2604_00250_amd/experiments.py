"""Accuracy and convergence harnesses on synthetic data.

crossing    best-match angular error, recall, precision and F1 per crossing
            angle on the shape of the paper's crossing-fibre benchmark
            (Sec. 3 dataset i, Table 1), MSE or Rician NLL, several SNRs; with
            --gain, the gain-perturbation sweep of Sec. 4 with the
            calibration fitted or held at identity.
optimizers  final data MSE and the first iteration within 110% of the best
            final MSE for Rprop, Adam (lr 0.01) and Adam (lr 0.05) on a
            brain-shaped 20-slice volume with a single-shell HARDI-like
            acquisition (the protocol of Table 2 on synthetic data).

Detection and matching (readings; the paper names the metrics only): a
fitted fibre is detected when its share of the WM fraction is at least 0.15
(the sparsity threshold tau of Sec. 2.4); the best-match angular error of a
ground-truth fibre is its axial angle to the closest detected fibre; true
positives come from a one-to-one matching of ground-truth and detected
fibres taken in increasing order of angle and accepted up to 20 degrees;
recall = TP / ground-truth fibres, precision = TP / detected fibres, F1 their
harmonic mean.

    python -m paper_2604_00250_amd.experiments crossing --snr 10 30 50 --mode mse nll
    python -m paper_2604_00250_amd.experiments crossing --gain 0.02 0.05 0.1 0.2
    python -m paper_2604_00250_amd.experiments optimizers
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

DETECT_SHARE = 0.15
TP_DEGREES = 20.0


# ----------------------------------------------------------------------------
# metrics (host side, on fitted parameters)
# ----------------------------------------------------------------------------

def fibres(theta: dict, K: int):
    """Unit fibre directions [K, V, 3] and each fibre's share of the WM
    fraction [K, V] from raw micro-structure parameters."""
    lg = np.asarray(theta["logits"], dtype=np.float64)
    f = np.exp(lg - lg.max(0, keepdims=True))
    f /= f.sum(0, keepdims=True)
    fw = f[2:2 + K]
    share = fw / np.maximum(fw.sum(0, keepdims=True), 1e-30)
    v = np.asarray(theta["v"], dtype=np.float64)                  # [K, 3, V]
    d = v / np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-30)
    return np.transpose(d, (0, 2, 1)), share


def axial_angle(a, b):
    """Angle in degrees between the axes of unit vectors (0..90)."""
    c = np.abs((np.asarray(a) * np.asarray(b)).sum(-1))
    return np.rad2deg(np.arccos(np.clip(c, 0.0, 1.0)))


def voxel_metrics(d_pred, share, gt_dirs, n_fib, detect=DETECT_SHARE, tp_deg=TP_DEGREES):
    """Per voxel: sum of best-match errors over its ground-truth fibres, the
    number of ground-truth fibres, true positives and detected fibres.
    d_pred [K, V, 3], share [K, V], gt_dirs [G, V, 3], n_fib [V]."""
    K, V = share.shape
    err_sum = np.zeros(V)
    tp = np.zeros(V, dtype=np.int64)
    det = share >= detect
    n_det = det.sum(0)
    for x in range(V):
        pk = [k for k in range(K) if det[k, x]]
        if not pk:                               # nothing above threshold: take the largest
            pk = [int(np.argmax(share[:, x]))]
        ang = np.array([[float(axial_angle(gt_dirs[g, x], d_pred[k, x])) for k in pk]
                        for g in range(int(n_fib[x]))])
        err_sum[x] = ang.min(1).sum()
        pairs = sorted((ang[g, j], g, j) for g in range(ang.shape[0]) for j in range(ang.shape[1]))
        used_g, used_k = set(), set()
        for a, g, j in pairs:
            if a > tp_deg:
                break
            if g in used_g or j in used_k or not det[pk[j], x]:
                continue
            used_g.add(g)
            used_k.add(j)
        tp[x] = len(used_g)
    return dict(err_sum=err_sum, n_gt=np.asarray(n_fib, dtype=np.int64), tp=tp, n_det=n_det)


def summarise(m: dict, sel=None) -> dict:
    """Mean best-match error (degrees), recall, precision and F1 over voxels `sel`."""
    sel = np.ones(m["n_gt"].shape, dtype=bool) if sel is None else sel
    n_gt = int(m["n_gt"][sel].sum())
    n_det = int(m["n_det"][sel].sum())
    tp = int(m["tp"][sel].sum())
    rec = tp / max(n_gt, 1)
    prec = tp / max(n_det, 1)
    f1 = 2 * prec * rec / max(prec + rec, 1e-30)
    return dict(error_deg=float(m["err_sum"][sel].sum() / max(n_gt, 1)), recall=rec, precision=prec, f1=f1,
                voxels=int(sel.sum()))


# ----------------------------------------------------------------------------
# crossing-fibre benchmark
# ----------------------------------------------------------------------------

def run_crossing(snr=30.0, mode="mse", iterations=300, optimizer="rprop", lr=1e-2, gain_sigma=0.0,
                 calibrate=True, seed=None, per_angle=200, n_single=200, angles=None, device="cuda:0"):
    import torch
    from . import inputs as I
    from .fit import fit
    from .problem import DeviceState, Problem
    kw = {} if angles is None else dict(angles=tuple(angles))
    w = I.crossing_benchmark(snr=snr, seed=seed, per_angle=per_angle, n_single=n_single, mode=mode,
                             gain_sigma=gain_sigma, **kw)
    g = w.groups[0]
    prob = Problem([g])
    st = DeviceState(prob, ys=[g.y], thetas=[g.theta], device=device)
    t0 = time.perf_counter()
    hist = fit(st, iterations, lr=lr, optimizer=optimizer, calibrate=calibrate)
    torch.cuda.synchronize(st.device)
    secs = time.perf_counter() - t0
    pm, _ = st.params_host()
    d, share = fibres(pm[0], g.K)
    t = g.truth
    m = voxel_metrics(d, share, t["dirs"], t["n_fib"])     # truth dirs [2, V, 3]
    ang = t["angle"]
    rows = {}
    for a in sorted(set(ang.tolist())):
        key = "single" if a == 0 else f"{int(a)}"
        rows[key] = summarise(m, ang == a)
    out = dict(workload=w.name, snr=snr, mode=mode, optimizer=optimizer, lr=lr, iterations=iterations,
               gain_sigma=gain_sigma, calibrate=calibrate, fit_seconds=secs,
               loss_first=float(hist[0, 0, -1]), loss_last=float(hist[-1, 0, -1]),
               overall=summarise(m), per_angle=rows)
    return out


# ----------------------------------------------------------------------------
# optimiser comparison
# ----------------------------------------------------------------------------

def run_optimizers(iterations=200, shape=(81, 106, 20), target=60_000, seed=None, device="cuda:0",
                   runs=(("rprop", 1e-2), ("adam", 1e-2), ("adam", 5e-2))):
    """Final data MSE per measurement and the first iteration whose MSE is
    within 110% of the best final MSE of all runs (Table 2's threshold)."""
    import torch
    from . import _lib as L
    from . import inputs as I
    from .fit import fit
    from .problem import DeviceState, Problem
    w = I.brain_volume(seed=seed, shape=shape, target=target, acq_kind="hardi160")
    g = w.groups[0]
    prob = Problem([g])
    curves = {}
    for opt, lr in runs:
        st = DeviceState(prob, ys=[g.y], thetas=[g.theta], device=device)
        hist = fit(st, iterations, lr=lr, optimizer=opt)
        torch.cuda.synchronize(st.device)
        data = hist[:, 0, L.LOSS_TERMS.index("data")].cpu().numpy()
        curves[f"{opt}({lr:g})"] = data / g.acq.n        # mean squared residual per measurement
    best = min(c[-1] for c in curves.values())
    res = {}
    for k, c in curves.items():
        hit = np.nonzero(c <= 1.1 * best)[0]
        res[k] = dict(final_mse=float(c[-1]), iter_to_thr=int(hit[0]) if hit.size else None,
                      curve=[float(x) for x in c[:: max(1, iterations // 20)]])
    return dict(workload=f"brain{shape[0]}x{shape[1]}x{shape[2]}_n{g.acq.n}_k3_mse", voxels=g.n_vox,
                iterations=iterations, best_final_mse=float(best), runs=res)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("crossing")
    c.add_argument("--snr", type=float, nargs="+", default=[30.0])
    c.add_argument("--mode", nargs="+", default=["mse"])
    c.add_argument("--iterations", type=int, default=300)
    c.add_argument("--optimizer", default="rprop")
    c.add_argument("--lr", type=float, default=1e-2)
    c.add_argument("--gain", type=float, nargs="*", default=[])
    c.add_argument("--out", default=None)
    o = sub.add_parser("optimizers")
    o.add_argument("--iterations", type=int, default=200)
    o.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    results = []
    if a.cmd == "crossing":
        if a.gain:
            for gs in a.gain:
                for cal in (False, True):
                    r = run_crossing(snr=a.snr[0], mode=a.mode[0], iterations=a.iterations, optimizer=a.optimizer,
                                     lr=a.lr, gain_sigma=gs, calibrate=cal, angles=(30, 45, 60, 90), n_single=0)
                    print(json.dumps(dict(gain=gs, calibrate=cal, **r["overall"])), flush=True)
                    results.append(r)
        else:
            for mode in a.mode:
                for snr in a.snr:
                    r = run_crossing(snr=snr, mode=mode, iterations=a.iterations, optimizer=a.optimizer, lr=a.lr)
                    print(json.dumps(dict(mode=mode, snr=snr, **r["overall"])), flush=True)
                    results.append(r)
    else:
        r = run_optimizers(iterations=a.iterations)
        print(json.dumps({k: {kk: v[kk] for kk in ("final_mse", "iter_to_thr")} for k, v in r["runs"].items()}),
              flush=True)
        results.append(r)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(results, f, indent=1)
    return results


if __name__ == "__main__":
    main(sys.argv[1:])
