"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed
form, an independent formulation (diffusion tensors), an invariant, a special
case, quadrature / arbitrary-precision Bessel values, finite differences of
its own objective (which pins the hand-derived adjoint to the pinned forward
model), a stationary point, or brute-force recovery on a tiny input.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

C = O.Constants()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_prob(V=8, N=33, K=3, mode="mse", bias="none", learn=False, nb=6, shape=None,
              priors=("spatial", "rep", "sparse", "cal"), seed=0):
    rng = np.random.default_rng(seed)
    if shape is None:
        shape = (2, 2, 2) if V == 8 else (V, 1, 1)
    coords = np.argwhere(np.ones(shape, dtype=bool))
    assert coords.shape[0] == V
    bval = np.concatenate([[0.0], rng.choice([1.0, 2.0, 3.0], size=N - 1)])
    bvec = I.uniform_sphere(N, rng)
    return O.Problem(coords=coords, shape=shape, bval=bval, bvec=bvec, K=K, mode=mode,
                     bias=bias, learn_diffusivity=learn, neighbourhood=nb, priors=priors)


def rand_theta(prob, seed=1, scale=1.0):
    rng = np.random.default_rng(seed)
    V, K, N = prob.V, prob.K, prob.N
    nbias = {"none": 0, "poly2": 10, "trilinear8": 512}[prob.bias]
    th = dict(
        s0=rng.normal(0.5, 0.5, V),
        logits=rng.normal(0, scale, (K + 3, V)),
        v=rng.normal(0, 1, (K, 3, V)),
        fin=rng.normal(0, 1, V),
        bias=rng.normal(0, 0.1, nbias),
        alpha=rng.normal(0, 0.05, N),
        beta=rng.normal(0, 0.02, N),
        sigma_log=np.array(math.log(0.1)),
    )
    if prob.learn_diffusivity:
        th["dpar"] = rng.normal(0.8, 0.3, V)
        th["dperp"] = rng.normal(-0.5, 0.3, V)
    return th


# ----------------------------------------------------------------------------
# constants printed in the paper
# ----------------------------------------------------------------------------

def test_constants_match_paper_text():
    gold = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    for k in ("d_csf", "d_gm", "d_res", "d_par", "d_perp", "huber_delta", "lam_sp", "lam_rep",
              "lam_sparse", "tau_sparse"):
        assert getattr(C, k) == gold[k]["value"], k


# ----------------------------------------------------------------------------
# forward model: closed forms and special cases
# ----------------------------------------------------------------------------

def _tensor_signal(b, g, D):
    """exp(-b g^T D g) for a 3x3 diffusion tensor D: an independent formulation."""
    return np.exp(-b * np.einsum("ni,ij,nj->n", g, D, g))


@pytest.mark.parametrize("fin", [1.0, 0.0])
def test_single_fibre_is_a_cylindrical_tensor(fin):
    rng = np.random.default_rng(3)
    N = 50
    bval = rng.uniform(0, 3, N)
    bvec = I.uniform_sphere(N, rng)
    u = I.uniform_sphere(1, rng)[0]
    f = np.zeros((4, 1))
    f[2, 0] = 1.0  # K=1: (csf, gm, wm_1, res)
    yhat = O.forward_constrained(bval, bvec, np.ones(1), f, u.reshape(1, 3, 1), np.array([fin]),
                                 np.array([C.d_par]), np.array([C.d_perp]), np.zeros(1),
                                 np.zeros(N), np.zeros(N))[:, 0]
    # stick: D = Dpar u u^T ; zeppelin: D = Dperp I + (Dpar - Dperp) u u^T
    if fin == 1.0:
        D = C.d_par * np.outer(u, u)
        assert np.allclose(yhat, np.exp(-bval * C.d_par * (bvec @ u) ** 2), rtol=1e-14, atol=0)
    else:
        D = C.d_perp * np.eye(3) + (C.d_par - C.d_perp) * np.outer(u, u)
    assert np.allclose(yhat, _tensor_signal(bval, bvec, D), rtol=1e-13, atol=0)


def test_intra_fraction_mixes_stick_and_zeppelin_linearly():
    rng = np.random.default_rng(4)
    N = 20
    bval = rng.uniform(0, 3, N)
    bvec = I.uniform_sphere(N, rng)
    u = I.uniform_sphere(1, rng)[0]
    f = np.zeros((4, 1))
    f[2, 0] = 1.0
    stick = _tensor_signal(bval, bvec, C.d_par * np.outer(u, u))
    zep = _tensor_signal(bval, bvec, C.d_perp * np.eye(3) + (C.d_par - C.d_perp) * np.outer(u, u))
    for fin in (0.3, 0.8):
        yhat = O.forward_constrained(bval, bvec, np.ones(1), f, u.reshape(1, 3, 1), np.array([fin]),
                                     np.array([C.d_par]), np.array([C.d_perp]), np.zeros(1),
                                     np.zeros(N), np.zeros(N))[:, 0]
        assert np.allclose(yhat, fin * stick + (1 - fin) * zep, rtol=1e-13)


@pytest.mark.parametrize("slot,D", [(0, 3.0), (1, 0.9), ("res", 0.2)])
def test_isotropic_compartments_by_index(slot, D):
    """A one-hot fraction on one isotropic slot gives exp(-b D) with the paper's D
    (pins the slot order csf, gm, wm_1..K, res and the three constants)."""
    prob = make_prob(V=8, N=40, K=2)
    th = rand_theta(prob)
    j = prob.K + 2 if slot == "res" else slot
    th["logits"] = np.full((prob.C, prob.V), -60.0)
    th["logits"][j] = 60.0
    th["alpha"][:] = 0
    th["beta"][:] = 0
    S0 = O.softplus(th["s0"])
    yhat = O.synthesize(prob, th)
    expect = S0[None] * np.exp(-prob.bval[:, None] * D)
    assert np.allclose(yhat, expect, rtol=1e-12, atol=0)


def test_b0_gives_calibrated_S0():
    """At b = 0 every compartment attenuation is 1 and the fractions sum to one,
    so yhat = exp(alpha) B(x) S0 + beta (Eq. 3 and Eq. 6)."""
    prob = make_prob(V=8, N=12, K=3, bias="poly2")
    prob.bval[:] = 0.0
    th = rand_theta(prob)
    yhat = O.synthesize(prob, th)
    S0 = np.log1p(np.exp(th["s0"]))
    x = O.unit_box_coords(prob)
    c = th["bias"]
    # quadratic log-bias written as a symmetric form, independent of the basis order
    A = np.array([[c[4], c[7] / 2, c[8] / 2], [c[7] / 2, c[5], c[9] / 2], [c[8] / 2, c[9] / 2, c[6]]])
    logB = c[0] + x @ c[1:4] + np.einsum("vi,ij,vj->v", x, A, x)
    expect = np.exp(th["alpha"])[:, None] * np.exp(logB)[None] * S0[None] + th["beta"][:, None]
    assert np.allclose(yhat, expect, rtol=1e-13, atol=1e-15)


def test_poly2_basis_at_box_corners():
    prob = make_prob(V=27, N=3, K=1, bias="poly2", shape=(3, 3, 3))
    Phi = O.bias_basis(prob)
    for v, (i, j, k) in enumerate(prob.coords):
        sx, sy, sz = i - 1.0, j - 1.0, k - 1.0  # -1, 0, 1 across a size-3 box
        expect = [1, sx, sy, sz, sx * sx, sy * sy, sz * sz, sx * sy, sx * sz, sy * sz]
        assert np.allclose(Phi[:, v], expect)


def test_trilinear_basis_reproduces_linear_fields_and_partition_of_unity():
    prob = make_prob(V=13 * 5 * 9, N=3, K=1, bias="trilinear8", shape=(13, 5, 9))
    Phi = O.bias_basis(prob)
    assert np.allclose(Phi.sum(0), 1.0)
    grid = np.indices((8, 8, 8)).reshape(3, -1).astype(float)
    for a in range(3):
        n = prob.shape[a]
        field = Phi.T @ grid[a]  # control value = its own index along axis a
        assert np.allclose(field, prob.coords[:, a] * 7.0 / (n - 1))


def test_direction_sign_scale_and_slot_permutation_invariance():
    prob = make_prob(V=8, N=33, K=3, mode="nll", bias="poly2")
    th = rand_theta(prob)
    y = np.abs(O.synthesize(prob, th) + 0.02)
    base = O.objective(prob, th, y)["total"]
    th2 = dict(th, v=th["v"] * np.array([-1.0, 2.5, -0.3])[:, None, None])
    assert O.objective(prob, th2, y)["total"] == pytest.approx(base, rel=1e-13)
    perm = [2, 0, 1]
    lg = th["logits"].copy()
    lg[2:5] = th["logits"][2:5][perm]
    th3 = dict(th, logits=lg, v=th["v"][perm])
    assert O.objective(prob, th3, y)["total"] == pytest.approx(base, rel=1e-13)


def test_calibration_identity():
    prob = make_prob(V=8, N=20, K=2, bias="poly2")
    th = rand_theta(prob)
    th["alpha"][:] = 0
    th["beta"][:] = 0
    th["bias"][:] = 0
    tr = O.transforms(prob, th)
    S = O.forward_constrained(prob.bval, prob.bvec, tr["S0"], tr["f"], tr["d"], tr["fin"],
                              tr["dpar"], tr["dperp"], np.zeros(8), np.zeros(20), np.zeros(20))
    assert np.array_equal(O.synthesize(prob, th), S)


# ----------------------------------------------------------------------------
# data terms
# ----------------------------------------------------------------------------

def test_mse_normalisation_counts_masked_voxels():
    prob = make_prob(V=8, N=6, K=1, priors=())
    prob.bval[:] = 0.0
    th = rand_theta(prob)
    th["alpha"][:] = 0
    th["beta"][:] = 0
    y = np.random.default_rng(0).normal(1, 0.1, (6, 8))
    S0 = np.log1p(np.exp(th["s0"]))
    expect = sum((S0[v] - y[n, v]) ** 2 for n in range(6) for v in range(8)) / 8
    assert O.objective(prob, th, y)["data"] == pytest.approx(expect, rel=1e-13)
    prob.norm_count = 1000
    assert O.objective(prob, th, y)["data"] == pytest.approx(expect * 8 / 1000, rel=1e-13)


def test_nll_at_zero_measurement():
    """y = 0: I0(0) = 1, so each term is log s^2 + yhat^2 / (2 s^2)."""
    prob = make_prob(V=8, N=10, K=2, mode="nll", priors=())
    th = rand_theta(prob)
    yhat = O.synthesize(prob, th)
    s2 = math.exp(2 * float(th["sigma_log"]))
    expect = (math.log(s2) + yhat ** 2 / (2 * s2)).sum()
    assert O.objective(prob, th, np.zeros_like(yhat))["data"] == pytest.approx(expect, rel=1e-13)


def test_nll_approaches_gaussian_form_at_high_snr():
    """As sigma -> 0: NLL - [(y-yhat)^2/(2 s^2) + log s^2] - 0.5 log(2 pi y yhat / s^2)
    = -1/(8z) + O(z^-2) with z = y yhat / s^2 (large-argument expansion of I0)."""
    prob = make_prob(V=8, N=10, K=2, mode="nll", priors=())
    th = rand_theta(prob)
    yhat = O.synthesize(prob, th)
    y = yhat * (1.0 + 0.05 * np.random.default_rng(2).standard_normal(yhat.shape))
    for sigma in (0.1, 0.03, 0.01, 0.003):
        th["sigma_log"] = np.array(math.log(sigma))
        s2 = sigma * sigma
        z = y * yhat / s2
        nll = O.objective(prob, th, y)["data"]
        gauss = ((y - yhat) ** 2 / (2 * s2) + math.log(s2) + 0.5 * np.log(2 * math.pi * z)).sum()
        corr = (-1.0 / (8 * z)).sum()
        rem = abs(nll - gauss - corr)
        assert rem <= 2.0 * (1.0 / z ** 2).sum() * 0.1 + 1e-9 * abs(nll)


def test_log_i0_and_ratio_against_quadrature_and_mpmath():
    from scipy.integrate import quad
    import mpmath as mp
    mp.mp.dps = 40
    for z in (0.0, 1e-3, 0.5, 2.0, 3.75, 7.0, 19.0, 60.0, 430.0, 900.0, 3.0e4):
        # I0e(z) = (1/pi) int_0^pi exp(z (cos t - 1)) dt ; I1e: same weighted by cos t
        pts = [min(math.pi / 2, 8.0 / math.sqrt(z))] if z > 1 else None
        q = lambda fn: quad(fn, 0, math.pi, epsabs=0, epsrel=1e-13, limit=400, points=pts)[0] / math.pi  # noqa: E731
        i0 = q(lambda t: math.exp(z * (math.cos(t) - 1.0)))
        one_minus_r = q(lambda t: (1 - math.cos(t)) * math.exp(z * (math.cos(t) - 1.0))) / i0
        assert O.log_i0(z) == pytest.approx(z + math.log(i0), rel=1e-12, abs=1e-14)
        r = O.bessel_ratio(z)
        assert 1.0 - r == pytest.approx(one_minus_r, rel=1e-8, abs=1e-300)
        if z > 0:
            hp_r = mp.besseli(1, z) / mp.besseli(0, z)
            assert r == pytest.approx(float(hp_r), rel=1e-13)
            assert O.log_i0(z) == pytest.approx(float(mp.log(mp.besseli(0, z))), rel=1e-13)
    assert O.bessel_ratio(-2.0) == pytest.approx(-O.bessel_ratio(2.0), rel=1e-15)


# ----------------------------------------------------------------------------
# priors
# ----------------------------------------------------------------------------

def test_spatial_prior_constant_field_is_zero():
    prob = make_prob(V=27, N=3, K=2, shape=(3, 3, 3))
    f = np.tile(np.array([0.1, 0.2, 0.3, 0.15, 0.25])[:, None], (1, 27))
    loss, g = O.spatial_prior(prob, f, C)
    assert loss < 1e-30 and np.abs(g).max() < 1e-15   # zero up to the rounding of the mean


def test_spatial_prior_line_by_hand():
    """Three voxels on a line, one compartment value per voxel (a, b, c)."""
    prob = make_prob(V=3, N=3, K=1, shape=(3, 1, 1))
    a, b, c_ = 0.30, 0.32, 0.50
    f = np.zeros((4, 3))
    f[0] = [a, b, c_]
    loss, _ = O.spatial_prior(prob, f, C)
    d = C.huber_delta
    hub = lambda r: 0.5 * r * r if abs(r) <= d else d * (abs(r) - 0.5 * d)  # noqa: E731
    r = [a - b, b - 0.5 * (a + c_), c_ - b]
    assert loss == pytest.approx(C.lam_sp / 3 * sum(hub(x) for x in r), rel=1e-14)
    # both Huber branches are exercised: |r0| < delta < |r2|
    assert abs(r[0]) < d < abs(r[2])


def test_spatial_prior_26_neighbourhood_counts():
    prob = make_prob(V=27, N=3, K=1, shape=(3, 3, 3), nb=26)
    cnt = (O.neighbour_table(prob) >= 0).sum(1).reshape(3, 3, 3)
    assert cnt[1, 1, 1] == 26 and cnt[0, 0, 0] == 7 and cnt[0, 1, 1] == 17 and cnt[0, 0, 1] == 11
    prob6 = make_prob(V=27, N=3, K=1, shape=(3, 3, 3), nb=6)
    cnt6 = (O.neighbour_table(prob6) >= 0).sum(1).reshape(3, 3, 3)
    assert cnt6[1, 1, 1] == 6 and cnt6[0, 0, 0] == 3


def test_repulsion_two_fibres_closed_form():
    prob = make_prob(V=1, N=3, K=2, shape=(1, 1, 1))
    f = np.array([[0.1], [0.1], [0.5], [0.2], [0.1]])
    ang = math.radians(35.0)
    d = np.zeros((2, 3, 1))
    d[0, :, 0] = [1, 0, 0]
    d[1, :, 0] = [-math.cos(ang), math.sin(ang), 0]
    loss, _, _ = O.repulsion_prior(prob, f, d, C)
    assert loss == pytest.approx(C.lam_rep * 0.5 * 0.2 * math.cos(ang), rel=1e-14)
    d[1, :, 0] = [0, 0, 1]
    assert O.repulsion_prior(prob, f, d, C)[0] == 0.0


def test_repulsion_is_averaged_over_the_mask():
    """Three voxels, each with its own pair of fibres: the prior is the mean of
    the per-voxel sums lam_rep f_1 f_2 |cos| over |M| = 3 voxels (Sec. 2.4,
    topology priors), and its derivative with respect to f_1 at voxel x is
    lam_rep f_2(x) |cos(x)| / 3.  Values worked out by hand."""
    prob = make_prob(V=3, N=3, K=2, shape=(3, 1, 1))
    f = np.zeros((5, 3))
    f[2] = [0.5, 0.25, 0.4]     # fibre 1
    f[3] = [0.2, 0.5, 0.4]      # fibre 2
    cosines = [0.5, -0.8, 0.0]  # 60 deg, 143.13 deg (|cos| 0.8), 90 deg
    d = np.zeros((2, 3, 3))
    for x, c in enumerate(cosines):
        d[0, :, x] = [1.0, 0.0, 0.0]
        d[1, :, x] = [c, math.sqrt(1.0 - c * c), 0.0]
    loss, gf, _ = O.repulsion_prior(prob, f, d, C)
    # 0.5*0.2*0.5 + 0.25*0.5*0.8 + 0 = 0.05 + 0.1 = 0.15, times lam_rep / 3
    assert loss == pytest.approx(0.01 * 0.15 / 3, rel=1e-13)
    # d/df_1 = f_2 |cos| lam/3: (0.1, 0.4, 0) * 0.01/3
    assert np.allclose(gf[0], np.array([0.1, 0.4, 0.0]) * 0.01 / 3, rtol=1e-13, atol=0)
    # d/df_2 = f_1 |cos| lam/3: (0.25, 0.2, 0) * 0.01/3
    assert np.allclose(gf[1], np.array([0.25, 0.2, 0.0]) * 0.01 / 3, rtol=1e-13, atol=0)
    # |M| counts the problem's masked voxels even where a sub-region is evaluated
    sub = make_prob(V=3, N=3, K=2, shape=(3, 1, 1))
    sub.norm_count = 6
    assert O.repulsion_prior(sub, f, d, C)[0] == pytest.approx(0.01 * 0.15 / 6, rel=1e-13)


def test_calibration_penalty_by_hand():
    """Sec. 2.3 item 2 and Sec. 2.4 (calibration regularisers): an L2 penalty
    toward the identity calibration, lam_a |alpha|^2 + lam_b |beta|^2 +
    lam_bias |c|^2 with the 0.01 weights.  Worked by hand for
    alpha = (0.3, -0.2), beta = (0.1,), c = (0.5, -0.5):
    0.01 (0.09 + 0.04) + 0.01 (0.01) + 0.01 (0.25 + 0.25) = 0.0064
    (an L1 penalty would give 0.01 (0.5 + 0.1 + 1.0) = 0.016)."""
    th = dict(alpha=np.array([0.3, -0.2]), beta=np.array([0.1]), bias=np.array([0.5, -0.5]))
    loss, ga, gb, gw = O.calibration_prior(th, C)
    assert loss == pytest.approx(0.0064, rel=1e-13)
    assert np.allclose(ga, [0.006, -0.004], rtol=1e-13, atol=0)
    assert np.allclose(gb, [0.002], rtol=1e-13, atol=0)
    assert np.allclose(gw, [0.01, -0.01], rtol=1e-13, atol=0)
    # quadratic: doubling every parameter quadruples the penalty
    th2 = {k: 2.0 * v for k, v in th.items()}
    assert O.calibration_prior(th2, C)[0] == pytest.approx(4.0 * 0.0064, rel=1e-13)
    # at the identity calibration the penalty and its gradient vanish
    z = {k: np.zeros_like(v) for k, v in th.items()}
    out = O.calibration_prior(z, C)
    assert out[0] == 0.0 and all(not np.any(g) for g in out[1:])


def test_calibration_penalty_enters_the_objective_once():
    """The total objective with the calibration prior on exceeds the one
    without it by exactly the hand-computed penalty of test above, on a
    problem whose calibration vector is set to those values."""
    prob = make_prob(V=2, N=2, K=1, shape=(2, 1, 1), bias="none", priors=("cal",))
    th = rand_theta(prob, seed=3)
    th["alpha"] = np.array([0.3, -0.2])
    th["beta"] = np.array([0.1, 0.0])
    y = np.full((2, 2), 0.5)
    on, _, _ = O.loss_grad(prob, th, y)
    prob.priors = ()
    off, _, _ = O.loss_grad(prob, th, y)
    # 0.01 (0.09 + 0.04) + 0.01 (0.01) = 0.0014
    assert on["total"] - off["total"] == pytest.approx(0.0014, rel=1e-10)
    assert on["cal"] == pytest.approx(0.0014, rel=1e-13)


def test_sparsity_threshold():
    prob = make_prob(V=2, N=3, K=3, shape=(2, 1, 1))
    f = np.array([[0.1, 0.1], [0.1, 0.1], [0.5, 0.14], [0.16, 0.3], [0.04, 0.2], [0.1, 0.16]])
    loss, g = O.sparsity_prior(prob, f, C)
    assert loss == pytest.approx(C.lam_sparse / 2 * (0.04 + 0.14), rel=1e-14)
    assert np.array_equal(g > 0, np.array([[0, 1], [0, 0], [1, 0]], dtype=bool))


# ----------------------------------------------------------------------------
# gradient: finite differences, invariants, stationary point
# ----------------------------------------------------------------------------

def _fd_check(prob, th, y, h=1e-6, rtol=2e-6):
    _, grad, _ = O.loss_grad(prob, th, y)
    for key, g in grad.items():
        a = np.asarray(th[key], dtype=np.float64)
        if a.size == 0:
            continue
        fd = np.zeros(a.shape)
        it = np.nditer(a, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            tp = {k: np.array(v, dtype=np.float64, copy=True) for k, v in th.items()}
            tm = {k: np.array(v, dtype=np.float64, copy=True) for k, v in th.items()}
            tp[key][idx] += h
            tm[key][idx] -= h
            fd[idx] = (O.objective(prob, tp, y)["total"] - O.objective(prob, tm, y)["total"]) / (2 * h)
        scale = max(np.abs(fd).max(), 1e-8)
        err = np.abs(np.asarray(g) - fd).max() / scale
        assert err < rtol, (key, err, g, fd)


@pytest.mark.parametrize("mode,bias,learn,nb", [
    ("mse", "none", False, 6),
    ("mse", "poly2", False, 26),
    ("nll", "poly2", True, 6),
    ("nll", "trilinear8", False, 6),
])
def test_gradient_matches_central_differences(mode, bias, learn, nb):
    prob = make_prob(V=8, N=33, K=3, mode=mode, bias=bias, learn=learn, nb=nb)
    th = rand_theta(prob, seed=5)
    rng = np.random.default_rng(7)
    y = np.abs(O.synthesize(prob, th) * (1 + 0.1 * rng.standard_normal((prob.N, prob.V)))) + 0.01
    _fd_check(prob, th, y)


def test_gradient_on_a_line_patch_with_masked_hole():
    shape = (5, 2, 1)
    mask = np.ones(shape, dtype=bool)
    mask[2, 0, 0] = False
    coords = np.argwhere(mask)
    rng = np.random.default_rng(11)
    N = 17
    prob = O.Problem(coords=coords, shape=shape, bval=np.concatenate([[0], rng.uniform(0.5, 3, N - 1)]),
                     bvec=I.uniform_sphere(N, rng), K=2, mode="mse", bias="poly2")
    th = rand_theta(prob, seed=3, scale=2.0)
    y = np.abs(O.synthesize(prob, th) + 0.05 * rng.standard_normal((N, prob.V)))
    _fd_check(prob, th, y)


def test_adjoint_invariants():
    prob = make_prob(V=8, N=33, K=3, mode="nll", bias="poly2", learn=True)
    th = rand_theta(prob)
    y = np.abs(O.synthesize(prob, th) + 0.03)
    _, g, _ = O.loss_grad(prob, th, y)
    assert np.abs(g["logits"].sum(0)).max() < 1e-12 * np.abs(g["logits"]).max()
    dots = (g["v"] * th["v"]).sum(1)
    assert np.abs(dots).max() < 1e-12 * np.abs(g["v"]).max()


def test_gradient_vanishes_at_matched_data():
    """Noise-free data synthesised at theta* makes theta* a stationary point of the
    MSE data term: every gradient class must vanish (priors off)."""
    prob = make_prob(V=8, N=40, K=3, mode="mse", bias="poly2", learn=True, priors=())
    th = rand_theta(prob)
    y = O.synthesize(prob, th)
    out, g, _ = O.loss_grad(prob, th, y)
    assert out["total"] == 0.0
    for k, a in g.items():
        assert np.abs(a).max() < 1e-14, k


def test_beta_gradient_is_sum_of_yhat_gradients_and_alpha_scales():
    """d/dbeta_n = sum_v dL/dyhat and d/dalpha_n = sum_v dL/dyhat (yhat - beta):
    checked against a finite difference of the data term in yhat."""
    prob = make_prob(V=8, N=9, K=2, mode="nll", priors=())
    th = rand_theta(prob)
    y = np.abs(O.synthesize(prob, th) + 0.05)
    _, g, yhat = O.loss_grad(prob, th, y)
    h = 1e-6
    gy = np.zeros_like(yhat)
    for n in range(prob.N):
        for v in range(prob.V):
            yp = yhat.copy(); yp[n, v] += h
            ym = yhat.copy(); ym[n, v] -= h
            gy[n, v] = (O.data_term(prob, yp, y, th["sigma_log"]) - O.data_term(prob, ym, y, th["sigma_log"])) / (2 * h)
    assert np.allclose(g["beta"], gy.sum(1), rtol=1e-6, atol=1e-6)
    assert np.allclose(g["alpha"], (gy * (yhat - th["beta"][:, None])).sum(1), rtol=1e-6, atol=1e-6)


# ----------------------------------------------------------------------------
# brute-force recovery of one known crossing (identifiability of the model)
# ----------------------------------------------------------------------------

def _hemisphere_grid(step_deg):
    pts = []
    for th in np.arange(0, 90.0 + 1e-9, step_deg):
        nphi = max(1, int(round(360.0 * math.sin(math.radians(th)) / step_deg)))
        for ph in np.arange(nphi) * 360.0 / nphi:
            t, p = math.radians(th), math.radians(ph)
            pts.append([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])
    return np.array(pts)


@pytest.mark.slow
@pytest.mark.parametrize("angle", [45.0])
def test_brute_force_recovers_a_known_crossing(angle):
    from scipy.optimize import nnls
    rng = np.random.default_rng(21)
    acq = I.make_acquisition("three288", rng)
    u1 = np.array([0.0, 0.0, 1.0])
    u2 = np.array([math.sin(math.radians(angle)), 0.0, math.cos(math.radians(angle))])
    rot = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    u1, u2 = rot @ u1, rot @ u2
    fin = 0.5
    f_true = np.array([0.1, 0.15, 0.35, 0.3, 0.1])
    prob = O.Problem(coords=np.zeros((1, 3), dtype=int), shape=(1, 1, 1), bval=acq.bval, bvec=acq.bvec,
                     K=2, mode="mse", priors=())
    d_true = np.stack([u1, u2])[:, :, None]
    y = O.forward_constrained(acq.bval, acq.bvec, np.ones(1), f_true[:, None], d_true, np.array([fin]),
                              np.array([C.d_par]), np.array([C.d_perp]), np.zeros(1),
                              np.zeros(acq.n), np.zeros(acq.n))
    grid = _hemisphere_grid(6.0)
    b = acq.bval[:, None]
    iso = np.concatenate([np.exp(-b * C.d_csf), np.exp(-b * C.d_gm), np.exp(-b * C.d_res)], 1)
    cols = []
    for u in grid:
        cols.append(O.forward_constrained(acq.bval, acq.bvec, np.ones(1), np.array([[0], [0], [1.0], [0]]),
                                          u.reshape(1, 3, 1), np.array([fin]), np.array([C.d_par]),
                                          np.array([C.d_perp]), np.zeros(1), np.zeros(acq.n),
                                          np.zeros(acq.n))[:, 0])
    cols = np.stack(cols, 1)
    best = (np.inf, None)
    for i in range(len(grid)):
        ci = cols[:, i:i + 1]
        for j in range(i + 1, len(grid)):
            A = np.concatenate([iso, ci, cols[:, j:j + 1]], 1)
            _, res = nnls(A, y[:, 0])
            if res < best[0]:
                best = (res, (i, j))
    i, j = best[1]
    ang = lambda a, b: math.degrees(math.acos(min(1.0, abs(float(a @ b)))))  # noqa: E731
    e1 = min(ang(grid[i], u1) + ang(grid[j], u2), ang(grid[i], u2) + ang(grid[j], u1))
    assert e1 <= 2 * 6.0
    # refine with Adam on the oracle gradient from the grid argmin
    th = dict(s0=np.array([math.log(math.e - 1)]), logits=np.zeros((5, 1)),
              v=np.stack([grid[i], grid[j]])[:, :, None].copy(), fin=np.zeros(1),
              bias=np.zeros(0), alpha=np.zeros(acq.n), beta=np.zeros(acq.n), sigma_log=np.array(0.0))
    keys = ("s0", "logits", "v")
    m = {k: np.zeros_like(th[k]) for k in keys}
    vv = {k: np.zeros_like(th[k]) for k in keys}
    lr = 1e-2
    for t in range(1, 4001):
        out, g, _ = O.loss_grad(prob, th, y)
        if t == 2000:
            lr = 2e-3
        for k in keys:
            th[k], m[k], vv[k] = O.adam_step(th[k], g[k], m[k], vv[k], t, lr=lr)
    d = th["v"][:, :, 0] / np.linalg.norm(th["v"][:, :, 0], axis=1, keepdims=True)
    err = max(min(ang(d[0], u1), ang(d[0], u2)), min(ang(d[1], u1), ang(d[1], u2)))
    assert err < 0.1
    assert out["data"] < 1e-10


# ----------------------------------------------------------------------------
# optimisers
# ----------------------------------------------------------------------------

def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -1e-3, 0.0, 250.0])
    p, m, v = O.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-2)
    # m_hat = g, v_hat = g^2: the update is lr * g / (|g| + eps)
    assert np.allclose(p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_two_steps_by_hand():
    b1, b2, lr, eps = 0.9, 0.999, 0.1, 1e-8
    g1, g2 = 2.0, -1.0
    p, m, v = O.adam_step(1.0, g1, 0.0, 0.0, 1, lr, b1, b2, eps)
    p, m, v = O.adam_step(p, g2, m, v, 2, lr, b1, b2, eps)
    m_ = 0.9 * 0.2 + 0.1 * g2          # m1 = 0.2
    v_ = 0.999 * 0.004 + 0.001 * 1.0   # v1 = 0.004
    # p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps), after step 1 and step 2
    p1 = 1.0 - (lr / 0.1) * 0.2 / (math.sqrt(0.004) / math.sqrt(0.001) + eps)
    p_expect = p1 - lr / (1 - 0.81) * m_ / (math.sqrt(v_) / math.sqrt(1 - 0.999 ** 2) + eps)
    assert float(p) == pytest.approx(p_expect, rel=1e-14)
    assert float(m) == pytest.approx(m_, rel=1e-15) and float(v) == pytest.approx(v_, rel=1e-15)


def test_rprop_sequence_by_hand():
    p, prev, step = 0.0, 0.0, 0.01
    seq = []
    for g in (1.0, 2.0, -1.0, -1.0, 0.5):
        p, prev, step = O.rprop_step(p, g, prev, step)
        seq.append((float(p), float(step)))
    # steps: 0.01 (no history) -> 0.012 (same sign) -> 0.006 (flip: no move, history
    #        erased) -> 0.006 (no history: move) -> 0.003 (flip: no move)
    expect_steps = [0.01, 0.012, 0.006, 0.006, 0.003]
    expect_p = [-0.01, -0.022, -0.022, -0.016, -0.016]
    assert np.allclose([s for _, s in seq], expect_steps)
    assert np.allclose([q for q, _ in seq], expect_p)
