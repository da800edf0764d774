"""CPU tests of the accuracy harness's metrics on hand-built cases."""
import math

import numpy as np
import pytest

from paper_2604_00250_amd import experiments as E


def _rot(deg):
    t = math.radians(deg)
    return np.array([math.cos(t), math.sin(t), 0.0])


def test_axial_angle_is_sign_free_and_symmetric():
    a, b = _rot(0), _rot(35)
    assert E.axial_angle(a, b) == pytest.approx(35.0)
    assert E.axial_angle(a, -b) == pytest.approx(35.0)
    assert E.axial_angle(b, a) == pytest.approx(35.0)
    assert E.axial_angle(a, _rot(150)) == pytest.approx(30.0)


def test_perfect_fit_scores_zero_error_and_full_recall():
    gt = np.stack([np.stack([_rot(0), _rot(0)]), np.stack([_rot(60), _rot(0)])])   # [2, V=2, 3]
    n_fib = np.array([2, 1])
    d = gt.copy()
    d[0, 0] *= -1
    share = np.array([[0.5, 0.97], [0.5, 0.03]])
    m = E.voxel_metrics(d, share, gt, n_fib)
    s = E.summarise(m)
    assert s["error_deg"] == pytest.approx(0.0, abs=1e-6)
    assert s["recall"] == 1.0 and s["precision"] == 1.0 and s["f1"] == 1.0


def test_single_detection_in_a_narrow_crossing():
    """One fibre on the bisector of a 30-degree crossing: both ground-truth
    fibres are 15 degrees away, but only one is a true positive."""
    gt = np.stack([_rot(0)[None], _rot(30)[None]])
    d = np.stack([_rot(15)[None], _rot(90)[None]])
    share = np.array([[0.95], [0.05]])
    m = E.voxel_metrics(d, share, gt, np.array([2]))
    s = E.summarise(m)
    assert s["error_deg"] == pytest.approx(15.0)
    assert m["tp"][0] == 1 and m["n_det"][0] == 1
    assert s["recall"] == 0.5 and s["precision"] == 1.0
    assert s["f1"] == pytest.approx(2 * 0.5 / 1.5)


def test_spurious_fibre_lowers_precision_and_far_fibres_are_not_true_positives():
    gt = np.stack([_rot(0)[None], _rot(0)[None]])
    d = np.stack([_rot(25)[None], _rot(80)[None]])
    share = np.array([[0.7], [0.3]])
    m = E.voxel_metrics(d, share, gt, np.array([1]))
    assert m["n_det"][0] == 2 and m["tp"][0] == 0          # 25 degrees is beyond the 20-degree match
    assert m["err_sum"][0] == pytest.approx(25.0)
    d[0, 0] = _rot(10)
    m = E.voxel_metrics(d, share, gt, np.array([1]))
    s = E.summarise(m)
    assert m["tp"][0] == 1 and s["precision"] == 0.5 and s["recall"] == 1.0


def test_nothing_above_threshold_falls_back_to_the_largest_fibre():
    gt = np.stack([_rot(0)[None], _rot(0)[None]])
    d = np.stack([_rot(5)[None], _rot(70)[None]])
    share = np.array([[0.1], [0.05]])          # as if both shares sat under the threshold
    m = E.voxel_metrics(d, share, gt, np.array([1]))
    assert m["err_sum"][0] == pytest.approx(5.0) and m["tp"][0] == 0 and m["n_det"][0] == 0


def test_fibres_from_raw_parameters():
    K, V = 2, 3
    th = dict(logits=np.zeros((K + 3, V)), v=np.tile(np.array([[3.0], [0.0], [4.0]])[None], (K, 1, V)))
    th["logits"][2] = math.log(3.0)
    d, share = E.fibres(th, K)
    assert d.shape == (K, V, 3) and np.allclose(d[0, 0], [0.6, 0.0, 0.8])
    assert np.allclose(share[:, 0], [0.75, 0.25])
