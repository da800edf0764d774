"""GPU tests of the slab pipeline (Sec. 2.5): the stitch kernel against the
oracle's stitching, on independent random slab parameters and on the
parameters a slab fit on the GPU reaches."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

from gpu_helpers import oracle_problem, say, theta32

pytestmark = pytest.mark.gpu

MARGIN = 1e-4     # matching decisions closer than this are not compared


def _decision_margins(z0, probs, thetas, shape):
    """Per output voxel, the smallest gap of the oracle's float32 matching
    decisions (best vs second-best |cos|, and |cos| of the chosen fibre from
    0 for its sign); inf where no matching happens."""
    nx, ny, nz = shape
    K = probs[0].K
    C = K + 3
    w = O.slab_weights(list(z0), [p.shape[2] for p in probs])
    maps = [O.constrained_maps(p, th) for p, th in zip(probs, thetas)]
    src = {}
    for g, p in enumerate(probs):
        for v, (i, j, k) in enumerate(p.coords):
            src.setdefault((int(i) * ny + int(j)) * nz + int(z0[g]) + int(k), []).append((g, v, w[g][int(k)]))
    out = []
    for r in sorted(src):
        s = src[r]
        if len(s) == 1:
            out.append(np.inf)
            continue
        (ga, va, wa), (gb, vb, wb) = s
        (gr, vr), (go, vo) = ((ga, va), (gb, vb)) if wa >= wb else ((gb, vb), (ga, va))
        dr = maps[gr][1 + C:1 + C + 3 * K, vr].reshape(K, 3).astype(np.float32)
        do = maps[go][1 + C:1 + C + 3 * K, vo].reshape(K, 3).astype(np.float32)
        dots = dr @ do.T
        used, m = [], np.inf
        for k in range(K):
            cand = sorted((abs(float(dots[k, j])), j) for j in range(K) if j not in used)[::-1]
            if len(cand) > 1:
                m = min(m, cand[0][0] - cand[1][0])
            used.append(cand[0][1])
            m = min(m, abs(float(dots[k, cand[0][1]])))
        out.append(m)
    return np.array(out)


def _compare(name, state, prob_slabs, thetas32, shape, z0):
    import torch
    gpu = state.stitch_maps()
    torch.cuda.synchronize()
    gpu = gpu.cpu().numpy().astype(np.float64)
    oprobs = [oracle_problem(g) for g in prob_slabs]
    coords, ref = O.stitch_slabs(shape, z0, oprobs, thetas32)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    m = _decision_margins(z0, oprobs, thetas32, shape)
    ok = m > MARGIN
    say(f"[{name}] out voxels {ref.shape[1]}, blended {int(np.isfinite(m).sum())}, "
        f"near-tie excluded {int((~ok).sum())}")
    assert (~ok).sum() <= max(3, 0.01 * np.isfinite(m).sum())
    err = np.abs(gpu[:, ok] - ref[:, ok]).max(axis=1)
    say(f"[{name}] max abs error per row {np.array2string(err, precision=1)}")
    assert err.max() < 2e-6
    return coords


def test_stitch_kernel_matches_oracle_on_independent_slab_parameters():
    """The phantom (40^3, K = 4, learned diffusivities) as two slabs whose
    parameters are drawn independently, so every overlap voxel needs the
    fibre matching."""
    from paper_2604_00250_amd.problem import DeviceState
    from paper_2604_00250_amd.slabs import SlabFit
    g = I.tube_phantom().groups[0]
    fit = SlabFit(g, thickness=30, overlap=5)
    rng = np.random.default_rng(71)
    ths = [I.perturb_theta(s.theta, rng, scale=1.0) for s in fit.slabs]
    st = DeviceState(fit.prob, ys=[s.y for s in fit.slabs], thetas=ths)
    coords = _compare("phantom slabs", st, fit.slabs, [theta32(t) for t in ths], g.shape,
                      [a for a, _ in fit.ranges])
    assert np.array_equal(coords, g.coords)


def test_slab_fit_on_a_brain_shaped_volume_then_stitch():
    """A smaller brain-shaped volume as three slabs (30 / 30 / 14 slices)
    fitted on the GPU in one batched problem; every slab's loss falls, and
    the stitched maps of the fitted parameters match the oracle's stitch."""
    from paper_2604_00250_amd.slabs import SlabFit
    w = I.brain_volume(shape=(40, 48, 64), target=30_000)
    g = w.groups[0]
    fit = SlabFit(g, thickness=30, overlap=5)
    assert [t for _, t in fit.ranges] == [30, 30, 14]
    hist = fit.run(40, lr=1e-2).cpu().numpy()
    tot = hist[:, :, O.TERMS.index("total")]
    say(f"[slab fit] loss first {tot[0]} last {tot[-1]}")
    assert np.all(tot[-1] < tot[0])
    pm, _ = fit.state.params_host()
    ths = []
    for s, p in zip(fit.slabs, pm):
        t = dict(p)
        t.update({k: s.theta[k] for k in ("bias", "alpha", "beta", "sigma_log")})
        ths.append(theta32(t))
    _compare("brain slabs", fit.state, fit.slabs, ths, g.shape, [a for a, _ in fit.ranges])
