"""Pins of the oracle's stabilisation priors (orphan-WM suppression,
directional continuity, fibre ordering) and of the bias-field total
variation (Sec. 2.4).

The paper prints their weights but not their forms; the forms are readings
(stated in the oracle's header).  Each reading is pinned here by values
worked out by hand, by closed forms (a telescoping sum for TV), by
invariances, and by finite differences of the total objective with every
prior switched on.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2604_00250_amd import inputs as I

from test_oracle_pins import _fd_check, make_prob, rand_theta

C = O.Constants()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL = ("spatial", "rep", "sparse", "orphan", "continuity", "ordering", "cal", "tv")


def test_stabilisation_weights_match_paper_text():
    gold = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert C.lam_orphan == gold["lam_orphan"]["value"]
    assert C.lam_cont == gold["lam_continuity"]["value"]
    assert C.lam_order == gold["lam_ordering"]["value"]


def _fractions(wm, K):
    """A fraction matrix [K+3, V] with the given WM fractions and the rest
    spread over csf, gm and res."""
    wm = np.asarray(wm, dtype=np.float64).reshape(K, -1)
    rest = (1.0 - wm.sum(0)) / 3.0
    return np.vstack([rest, rest, wm, rest])


def test_orphan_by_hand():
    prob = make_prob(V=3, N=3, K=2, shape=(3, 1, 1))
    S0 = np.array([0.05, 0.5, 0.0])
    f = _fractions([[0.3, 0.4, 0.2], [0.2, 0.1, 0.6]], 2)
    loss, g_s0, g_f = O.orphan_prior(prob, S0, f, C)
    # voxel 0: h = 1 - 0.05/0.1 = 0.5, WM sum 0.5; voxel 1: h = 0; voxel 2: h = 1, WM sum 0.8
    assert loss == pytest.approx(C.lam_orphan / 3 * (0.5 * 0.5 + 1.0 * 0.8), rel=1e-14)
    assert g_s0[1] == 0.0 and g_s0[0] < 0 and g_s0[2] < 0
    assert np.all(g_f[:, 1] == 0.0)
    # at the threshold the hinge and its derivative are zero
    l2, gs2, _ = O.orphan_prior(prob, np.full(3, C.s0_orphan), f, C)
    assert l2 == 0.0 and np.all(gs2 == 0.0)


def test_ordering_by_hand():
    prob = make_prob(V=2, N=3, K=3, shape=(2, 1, 1))
    f = _fractions([[0.1, 0.5], [0.3, 0.2], [0.2, 0.1]], 3)
    loss, g = O.ordering_prior(prob, f, C)
    # voxel 0: (0.3 - 0.1) + 0 ; voxel 1 sorted: 0
    assert loss == pytest.approx(C.lam_order / 2 * 0.2, rel=1e-13)
    assert np.array_equal(np.sign(g[:, 0]), [-1.0, 1.0, 0.0]) and np.all(g[:, 1] == 0)
    prob1 = make_prob(V=2, N=3, K=1, shape=(2, 1, 1))
    assert O.ordering_prior(prob1, _fractions([[0.7, 0.2]], 1), C)[0] == 0.0


@pytest.mark.parametrize("theta_deg", [0.0, 30.0, 90.0])
def test_continuity_on_a_line_closed_form(theta_deg):
    """Three voxels on a line, directions (x, rotated x, x): every voxel's
    average over its neighbours is sin^2 theta, so the prior is lam sin^2."""
    prob = make_prob(V=3, N=3, K=1, shape=(3, 1, 1), nb=6)
    t = math.radians(theta_deg)
    d = np.zeros((1, 3, 3))
    d[0, :, 0] = [1, 0, 0]
    d[0, :, 1] = [math.cos(t), math.sin(t), 0]
    d[0, :, 2] = [1, 0, 0]
    loss, gd = O.continuity_prior(prob, d, C)
    assert loss == pytest.approx(C.lam_cont * math.sin(t) ** 2, rel=1e-13, abs=1e-18)
    # sign-free: flipping any voxel's direction changes nothing
    d2 = d.copy()
    d2[0, :, 1] *= -1
    assert O.continuity_prior(prob, d2, C)[0] == pytest.approx(loss, rel=1e-14, abs=1e-18)
    # without a neighbourhood the prior is off
    prob0 = make_prob(V=3, N=3, K=1, shape=(3, 1, 1), nb=0)
    assert O.continuity_prior(prob0, d, C)[0] == 0.0


def test_continuity_is_slotwise():
    """Fibre slots are compared slot by slot: swapping the two slots of one
    voxel of an aligned pair turns a zero prior into a positive one."""
    prob = make_prob(V=2, N=3, K=2, shape=(2, 1, 1), nb=6)
    d = np.zeros((2, 3, 2))
    d[0, :, :] = np.array([1.0, 0, 0])[:, None]
    d[1, :, :] = np.array([0, 1.0, 0])[:, None]
    assert O.continuity_prior(prob, d, C)[0] == 0.0
    d[:, :, 1] = d[::-1, :, 1]
    # each voxel: 1/|N| = 1, two slots each with 1 - 0 = 1 -> 2 per voxel
    assert O.continuity_prior(prob, d, C)[0] == pytest.approx(C.lam_cont / 2 * 4, rel=1e-14)


def test_tv_telescopes_on_a_monotone_line():
    """logB = c1 x on a line spanning x in [-1, 1]: B is monotone, so the sum
    of |B(x+1) - B(x)| telescopes to e^c1 - e^-c1."""
    n = 9
    prob = make_prob(V=n, N=3, K=1, shape=(n, 1, 1), bias="poly2")
    c1 = 0.3
    bias = np.zeros(10)
    bias[1] = c1
    logB = O.bias_basis(prob).T @ bias
    loss, g = O.tv_prior(prob, logB, C)
    assert loss == pytest.approx(C.lam_tv / n * (math.exp(c1) - math.exp(-c1)), rel=1e-13)
    # interior voxels have one pair on each side with the same sign: their
    # derivative cancels; only the two ends carry a gradient
    assert np.abs(g[1:-1]).max() < 1e-15
    assert g[0] == pytest.approx(-C.lam_tv / n * math.exp(-c1), rel=1e-13)
    assert g[-1] == pytest.approx(C.lam_tv / n * math.exp(c1), rel=1e-13)


def test_tv_masked_hole_and_axis_separation():
    """A field varying along y only: pairs along x and z contribute nothing,
    and a masked voxel removes the two pairs that touch it."""
    shape = (2, 5, 3)
    mask = np.ones(shape, dtype=bool)
    mask[1, 2, 1] = False
    coords = np.argwhere(mask)
    prob = O.Problem(coords=coords, shape=shape, bval=np.zeros(3), bvec=np.eye(3), K=1,
                     bias="poly2", neighbourhood=6)
    bias = np.zeros(10)
    bias[2] = -0.2
    logB = O.bias_basis(prob).T @ bias
    loss, _ = O.tv_prior(prob, logB, C)
    ys = np.linspace(-1, 1, 5)
    B = np.exp(-0.2 * ys)
    full_line = abs(B[-1] - B[0])
    # 6 full y-lines, except the line (1, :, 1) which loses pairs (1,2) and (2,3)
    hole_line = full_line - abs(B[2] - B[1]) - abs(B[3] - B[2])
    expect = 5 * full_line + hole_line
    assert loss == pytest.approx(C.lam_tv / prob.V * expect, rel=1e-13)


def test_tv_is_zero_for_a_constant_trilinear_grid():
    prob = make_prob(V=8, N=3, K=1, bias="trilinear8")
    logB = O.bias_basis(prob).T @ np.full(512, 0.37)
    loss, g = O.tv_prior(prob, logB, C)
    assert loss < 1e-15 and np.abs(g).max() < 1e-12


def _orphan_theta(prob, seed):
    th = rand_theta(prob, seed=seed, scale=1.5)
    # a few voxels with S0 well below the orphan level, none near the kink
    th["s0"][::3] = -3.5
    return th


@pytest.mark.parametrize("mode,bias,nb", [
    ("mse", "poly2", 6),
    ("mse", "poly2", 26),
    ("nll", "trilinear8", 6),
    ("mse", "none", 26),
])
def test_gradient_with_every_prior_matches_central_differences(mode, bias, nb):
    prob = make_prob(V=8, N=33, K=3, mode=mode, bias=bias, nb=nb, priors=ALL)
    th = _orphan_theta(prob, seed=9)
    if bias == "poly2":
        th["bias"] = np.random.default_rng(4).normal(0, 0.3, 10)
    rng = np.random.default_rng(8)
    y = np.abs(O.synthesize(prob, th) * (1 + 0.1 * rng.standard_normal((prob.N, prob.V)))) + 0.01
    out = O.objective(prob, th, y)
    for t in ("orphan", "continuity", "ordering"):
        assert out[t] > 0, t
    if bias != "none":
        assert out["tv"] > 0
    _fd_check(prob, th, y)


def test_gradient_with_every_prior_on_a_masked_box():
    shape = (4, 3, 2)
    rng = np.random.default_rng(21)
    mask = rng.random(shape) < 0.75
    mask[0, 0, 0] = True
    coords = np.argwhere(mask)
    N = 15
    prob = O.Problem(coords=coords, shape=shape, bval=np.concatenate([[0], rng.uniform(0.5, 3, N - 1)]),
                     bvec=I.uniform_sphere(N, rng), K=2, mode="mse", bias="poly2", neighbourhood=6,
                     priors=ALL)
    th = _orphan_theta(prob, seed=12)
    th["bias"] = rng.normal(0, 0.3, 10)
    y = np.abs(O.synthesize(prob, th) + 0.05 * rng.standard_normal((N, prob.V)))
    _fd_check(prob, th, y)


def test_adjoint_invariants_with_every_prior():
    prob = make_prob(V=8, N=33, K=3, mode="nll", bias="poly2", nb=26, priors=ALL)
    th = _orphan_theta(prob, seed=2)
    y = np.abs(O.synthesize(prob, th) + 0.03)
    _, g, _ = O.loss_grad(prob, th, y)
    assert np.abs(g["logits"].sum(0)).max() < 1e-12 * np.abs(g["logits"]).max()
    dots = (g["v"] * th["v"]).sum(1)
    assert np.abs(dots).max() < 1e-12 * np.abs(g["v"]).max()


def test_total_is_the_sum_of_the_terms():
    prob = make_prob(V=8, N=33, K=3, mode="mse", bias="poly2", nb=6, priors=ALL)
    th = _orphan_theta(prob, seed=3)
    y = np.abs(O.synthesize(prob, th) + 0.02)
    out, _, _ = O.loss_grad(prob, th, y)
    assert out["total"] == pytest.approx(sum(out[t] for t in O.TERMS[:-1]), rel=1e-15)
    assert out == pytest.approx(O.objective(prob, th, y), rel=1e-13)
