"""GPU tests of the autograd wrapper, the graph-captured fit loop and
checkpoint/resume, all through the C ABI."""
import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

from gpu_helpers import assert_parity, masked_group, merged_grad, oracle_problem, say, theta32, with_theta

pytestmark = pytest.mark.gpu


def _state(groups, thetas=None, launch=None):
    from paper_2604_00250_amd.problem import DeviceState, Problem
    prob = Problem(groups, launch=launch)
    return DeviceState(prob, ys=[g.y for g in groups], thetas=thetas or [g.theta for g in groups])


def test_autograd_function_matches_oracle_and_fp64_finite_differences():
    """The phantom's 4^3 crossing sub-patch (K=4, NLL, learned sigma and
    diffusivities, quadratic bias): the autograd gradient against the FP64
    oracle gradient for every parameter class, and directional derivatives
    against central differences (h = 1e-6) of the FP64 oracle objective."""
    import torch
    from paper_2604_00250_amd.autograd import PrismLoss
    w = I.tube_phantom()
    g = I.sub_box(w.groups[0], I.crossing_subpatch(w, 4), 4)
    g = with_theta(g, I.perturb_theta(g.theta, np.random.default_rng(17)))
    st = _state([g])
    p = st.params.clone().requires_grad_(True)
    loss = PrismLoss.apply(p, st)
    loss.backward()
    torch.cuda.synchronize()
    gm = st.prob.unpack_micro(p.grad[: st.n_micro].cpu().numpy())[0]
    gc = st.prob.unpack_cal(p.grad[st.n_micro:].cpu().numpy())[0]
    prob = oracle_problem(g)
    th = theta32(g.theta)
    y = np.asarray(g.y, np.float64)
    out, ref, _ = O.loss_grad(prob, th, y)
    assert_parity("autograd phantom 4^3", st.loss_host()[0], merged_grad(gm, gc), out, ref)
    assert float(loss.item()) == pytest.approx(out["total"], rel=1e-5)
    # directional derivatives along random directions, one per class
    rng = np.random.default_rng(3)
    h = 1e-6
    for key in ("s0", "logits", "v", "fin", "dpar", "dperp", "bias", "alpha", "beta", "sigma_log"):
        u = rng.standard_normal(np.shape(th[key]))
        tp = dict(th)
        tm = dict(th)
        tp[key] = th[key] + h * u
        tm[key] = th[key] - h * u
        fd = (O.objective(prob, tp, y)["total"] - O.objective(prob, tm, y)["total"]) / (2 * h)
        gpu = float(np.sum(np.asarray(merged_grad(gm, gc)[key], np.float64) * u))
        say(f"[directional {key}] gpu={gpu:.6g} fd64={fd:.6g}")
        assert gpu == pytest.approx(fd, rel=2e-4, abs=1e-6 * max(1.0, abs(fd)))


def test_graph_replay_equals_eager_iterations_bitwise():
    import torch
    from paper_2604_00250_amd.fit import Loop, restore, snapshot
    groups = [masked_group(shape=(9, 7, 8), K=3, mode="mse", seed=31, acq_kind="two96", bias="poly2"),
              masked_group(shape=(6, 6, 6), K=2, mode="nll", seed=32, acq_kind="single33", bias="trilinear8")]
    st = _state(groups)
    snap = snapshot(st)
    eager = Loop(st, lr=1e-2, history=8)
    for _ in range(8):
        eager.step_eager()
    torch.cuda.synchronize()
    p_eager = st.params.clone()
    h_eager = eager.hist.clone()
    restore(st, snap)
    loop = Loop(st, lr=1e-2, history=8)
    loop.capture()
    restore(st, snap)
    loop.hist.zero_()
    for r in range(8):
        loop.replay(1)
        if r % 3 == 1:  # eager work and a synchronisation between replays
            torch.cuda.synchronize()
            _ = (st.params * 2).sum().item()
    torch.cuda.synchronize()
    assert int(st.step[0].item()) == 8
    assert torch.equal(st.params, p_eager)
    assert torch.equal(loop.hist, h_eager)
    # the loss history decreases over the first iterations
    tot = h_eager[:, :, 9].sum(1).cpu().numpy()
    say(f"[graph] loss history {tot}")
    assert tot[-1] < tot[0]


def test_library_loss_history_rows_are_each_iterations_loss():
    """prism_iteration_adam writes each iteration's loss rows into the history
    ring at (iteration index mod length): the fused path, the fused path with
    the calibration held fixed, and the unfused path that a continuity prior
    forces; seven iterations on a ring of three rows."""
    import torch
    base = dict(shape=(7, 6, 6), K=2, mode="mse", acq_kind="two96", bias="poly2")
    cases = [("fused", masked_group(seed=61, priors=("spatial", "rep", "cal"), **base), True),
             ("fused, calibration fixed", masked_group(seed=62, priors=("spatial", "rep", "cal"), **base), False),
             ("unfused (continuity)", masked_group(seed=63, priors=("spatial", "continuity", "cal"), **base), True)]
    for name, g, cal in cases:
        st = _state([g])
        hist = torch.full((3, 1, 10), float("nan"), dtype=torch.float64, device=st.device)
        rows = []
        for t in range(7):
            st.iteration(1e-2, update_cal=cal, history=hist)
            torch.cuda.synchronize()
            rows.append(st.loss.clone())
            assert torch.equal(hist[t % 3], rows[t]), f"{name}: iteration {t}"
        assert int(st.step[0].item()) == 7
        for t in (4, 5, 6):
            assert torch.equal(hist[t % 3], rows[t])
        say(f"[history {name}] totals {[float(r[0, 9]) for r in rows]}")
        assert float(rows[-1][0, 9]) < float(rows[0][0, 9])


def test_rprop_loop_graph_equals_eager():
    import torch
    from paper_2604_00250_amd.fit import Loop, restore, snapshot
    g = masked_group(shape=(8, 8, 5), K=3, mode="mse", seed=41, acq_kind="two96", bias="poly2")
    st = _state([g])
    snap = snapshot(st)
    ea = Loop(st, lr=1e-2, optimizer="rprop", history=6)
    for _ in range(6):
        ea.step_eager()
    torch.cuda.synchronize()
    p_eager = st.params.clone()
    restore(st, snap)
    lp = Loop(st, lr=1e-2, optimizer="rprop", history=6)
    lp.capture()
    restore(st, snap)
    lp.prev.zero_()
    lp.rstep.fill_(1e-2)
    lp.it.zero_()
    lp.replay(6)
    torch.cuda.synchronize()
    assert torch.equal(st.params, p_eager)


def test_checkpoint_resume_is_bitwise(tmp_path):
    import torch
    from paper_2604_00250_amd.fit import fit, load_checkpoint, save_checkpoint
    g = masked_group(shape=(7, 6, 5), K=2, mode="nll", seed=51, acq_kind="two96", bias="poly2")
    a = _state([g])
    fit(a, 10, lr=1e-2, graph=False)
    b = _state([g])
    fit(b, 5, lr=1e-2, graph=False)
    path = str(tmp_path / "ck.npz")
    save_checkpoint(b, path, iterations=5)
    c = _state([g])
    meta = load_checkpoint(c, path)
    assert int(meta["iterations"]) == 5
    fit(c, 5, lr=1e-2, graph=False)
    torch.cuda.synchronize()
    assert torch.equal(a.params, c.params) and torch.equal(a.m, c.m) and torch.equal(a.v, c.v)
    assert a.step.tolist() == c.step.tolist() == [10, 0]


def test_short_adam_trajectory_matches_oracle():
    """Five Adam steps on the 8^3 patch: the loss history and the parameters
    follow the FP64 oracle's trajectory (Adam on the oracle gradient)."""
    import torch
    from paper_2604_00250_amd.fit import fit
    g = I.patch8_crossings(priors=I.PRIOR_NAMES).groups[0]
    st = _state([g])
    hist = fit(st, 5, lr=1e-2, graph=True)
    torch.cuda.synchronize()
    prob = oracle_problem(g)
    th = theta32(g.theta)
    y = np.asarray(g.y, np.float64)
    keys = list(th.keys())
    m = {k: np.zeros_like(th[k]) for k in keys}
    v = {k: np.zeros_like(th[k]) for k in keys}
    ref_hist = []
    for t in range(1, 6):
        out, gr, _ = O.loss_grad(prob, th, y)
        ref_hist.append(out["total"])
        for k in keys:
            th[k], m[k], v[k] = O.adam_step(th[k], gr[k], m[k], v[k], t)
    gpu_hist = hist[:, 0, 9].cpu().numpy()
    say(f"[trajectory] gpu {gpu_hist} ref {np.array(ref_hist)}")
    assert np.allclose(gpu_hist, ref_hist, rtol=1e-5)
    pm, pc = st.params_host()
    got = merged_grad(pm[0], pc[0])
    for k in ("s0", "logits", "v", "fin"):
        d = np.abs(np.asarray(got[k], np.float64) - th[k])
        assert np.mean(d > 1e-4) < 1e-3, (k, float(d.max()))


def test_fit_reduces_loss_on_the_calibrated_patch():
    import torch
    from paper_2604_00250_amd.fit import fit
    g = I.patch16_hcp().groups[0]
    st = _state([g])
    hist = fit(st, 60, lr=1e-2, graph=True)
    torch.cuda.synchronize()
    tot = hist[:, 0, 9].cpu().numpy()
    say(f"[fit patch16] loss {tot[0]:.6g} -> {tot[-1]:.6g}")
    assert np.all(np.isfinite(tot)) and tot[-1] < tot[0]
    assert int(st.status.item()) == 0
