"""Pins of the oracle's whole-volume slab layout and stitching (Sec. 2.5:
overlapping 30-slice slabs with a 5-slice overlap, blended by weighted
averaging).  The layout, the blend weights and the fibre matching are
readings; they are pinned by hand-worked layouts, the partition of unity,
exact reconstruction of a field the slabs agree on (also when one slab's
fibre slots are permuted and their signs flipped) and a blend worked out by
hand."""
import math

import numpy as np
import pytest

import oracle as O

C = O.Constants()


def test_slab_ranges_by_hand():
    assert O.slab_ranges(145) == [(0, 30), (25, 30), (50, 30), (75, 30), (100, 30), (125, 20)]
    assert O.slab_ranges(40) == [(0, 30), (25, 15)]
    assert O.slab_ranges(30) == [(0, 30)]
    assert O.slab_ranges(12) == [(0, 12)]
    assert O.slab_ranges(56) == [(0, 30), (25, 30), (50, 6)]
    with pytest.raises(ValueError):
        O.slab_ranges(100, thickness=8, overlap=5)


@pytest.mark.parametrize("nz,T,ov", [(145, 30, 5), (40, 30, 5), (56, 30, 5), (64, 16, 8), (33, 10, 0)])
def test_slab_weights_are_a_partition_of_unity(nz, T, ov):
    r = O.slab_ranges(nz, T, ov)
    w = O.slab_weights([a for a, _ in r], [t for _, t in r])
    tot = np.zeros(nz)
    cover = np.zeros(nz, dtype=int)
    for (a, t), wg in zip(r, w):
        tot[a:a + t] += wg
        cover[a:a + t] += 1
        assert np.all(wg > 0)
    assert np.allclose(tot, 1.0, rtol=0, atol=1e-15)
    assert cover.max() <= 2 and cover.min() == 1


def test_slab_weights_ramp_by_hand():
    w = O.slab_weights([0, 25], [30, 15])
    assert np.allclose(w[0][25:], [5 / 6, 4 / 6, 3 / 6, 2 / 6, 1 / 6])
    assert np.allclose(w[1][:5], [1 / 6, 2 / 6, 3 / 6, 4 / 6, 5 / 6])
    assert np.all(w[0][:25] == 1.0) and np.all(w[1][5:] == 1.0)


def _volume(shape, K, seed, learn=False):
    rng = np.random.default_rng(seed)
    mask = rng.random(shape) < 0.8
    coords = np.argwhere(mask)
    V = coords.shape[0]
    th = dict(s0=rng.normal(0.5, 0.5, V), logits=rng.normal(0, 1, (K + 3, V)),
              v=rng.normal(0, 1, (K, 3, V)), fin=rng.normal(0, 1, V))
    if learn:
        th["dpar"] = rng.normal(0.8, 0.3, V)
        th["dperp"] = rng.normal(-0.5, 0.3, V)
    return mask, coords, th


def _cut(mask, th, ranges, K, learn=False):
    """Slab problems and parameters cut from one volume's parameter field."""
    full = np.argwhere(mask)
    probs, thetas = [], []
    for a, t in ranges:
        sel = (full[:, 2] >= a) & (full[:, 2] < a + t)
        c = full[sel].copy()
        c[:, 2] -= a
        probs.append(O.Problem(coords=c, shape=(mask.shape[0], mask.shape[1], t), bval=np.zeros(1),
                               bvec=np.zeros((1, 3)), K=K, learn_diffusivity=learn))
        thetas.append({k: np.asarray(v)[..., sel].copy() for k, v in th.items()})
    return probs, thetas


@pytest.mark.parametrize("learn", [False, True])
def test_stitch_reconstructs_a_field_the_slabs_agree_on(learn):
    shape, K = (4, 3, 40), 3
    mask, coords, th = _volume(shape, K, seed=1, learn=learn)
    r = O.slab_ranges(shape[2])
    probs, thetas = _cut(mask, th, r, K, learn)
    oc, maps = O.stitch_slabs(shape, [a for a, _ in r], probs, thetas)
    assert np.array_equal(oc, coords)
    full = O.Problem(coords=coords, shape=shape, bval=np.zeros(1), bvec=np.zeros((1, 3)), K=K,
                     learn_diffusivity=learn)
    ref = O.constrained_maps(full, th, C)
    assert np.allclose(maps, ref, rtol=1e-13, atol=1e-13)


def test_stitch_undoes_slot_permutation_and_sign_flips():
    shape, K = (3, 3, 40), 3
    mask, coords, th = _volume(shape, K, seed=2)
    r = O.slab_ranges(shape[2])
    probs, thetas = _cut(mask, th, r, K)
    # the upper slab stores its fibres in another slot order with flipped signs
    perm = [2, 0, 1]
    t1 = thetas[1]
    t1["v"] = -t1["v"][perm]
    lg = t1["logits"].copy()
    lg[2:2 + K] = lg[2:2 + K][perm]
    t1["logits"] = lg
    _, maps = O.stitch_slabs(shape, [a for a, _ in r], probs, thetas)
    full = O.Problem(coords=coords, shape=shape, bval=np.zeros(1), bvec=np.zeros((1, 3)), K=K)
    ref = O.constrained_maps(full, th, C)
    lower = coords[:, 2] < 25 + 5 // 2 + 1       # where the lower slab is the heavier one
    # in the overlap's lower half and below, the output keeps the lower slab's slots
    assert np.allclose(maps[:, lower], ref[:, lower], rtol=1e-12, atol=1e-12)
    # above, the upper slab's (permuted) slot order is kept, with its own signs
    up = coords[:, 2] >= 30
    d_up = maps[1 + K + 3:1 + K + 3 + 3 * K][:, up].reshape(K, 3, -1)
    d_ref = ref[1 + K + 3:1 + K + 3 + 3 * K][:, up].reshape(K, 3, -1)
    assert np.allclose(d_up, -d_ref[perm], atol=1e-12)


def test_stitch_blend_by_hand():
    """One column of voxels; the two slabs disagree only in S0 and in one
    fibre's direction: at the middle slice of the overlap they blend 1:1."""
    shape, K = (1, 1, 40), 1
    mask = np.ones(shape, dtype=bool)
    r = O.slab_ranges(40)
    V = 40
    th = dict(s0=np.full(V, 0.3), logits=np.zeros((K + 3, V)), v=np.tile(np.array([1.0, 0, 0])[None, :, None], (1, 1, V)),
              fin=np.zeros(V))
    probs, thetas = _cut(mask, th, r, K)
    thetas[1]["s0"] = np.full(thetas[1]["s0"].shape, 1.3)
    thetas[1]["v"][0] = np.array([[0.0], [1.0], [0.0]]) * np.ones((1, thetas[1]["v"].shape[2]))
    coords, maps = O.stitch_slabs(shape, [a for a, _ in r], probs, thetas)
    sp = lambda x: math.log1p(math.exp(x))
    z = 27                                           # weights 3/6 and 3/6
    assert maps[0, z] == pytest.approx(0.5 * sp(0.3) + 0.5 * sp(1.3), rel=1e-14)
    d = maps[1 + K + 3:1 + K + 6, z]
    assert np.allclose(d, [math.sqrt(0.5), math.sqrt(0.5), 0.0], atol=1e-14)
    z = 26                                           # weights 4/6 (lower) and 2/6
    assert maps[0, z] == pytest.approx(4 / 6 * sp(0.3) + 2 / 6 * sp(1.3), rel=1e-14)
    assert maps[0, 10] == pytest.approx(sp(0.3), rel=1e-15) and maps[0, 35] == pytest.approx(sp(1.3), rel=1e-15)
