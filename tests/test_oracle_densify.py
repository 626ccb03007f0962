"""Pins of the oracle's depth loss (Sec. 3.1) and densification pieces
(Sec. 3.2, Eq. 3-4): closed forms, hand-made masks at the threshold, the split
score against a per-pixel brute force over all Gaussians (no tile lists),
and clone / split placement against hand-computed cases."""
import math

import numpy as np
import pytest

from oracle import binning, densify, preprocess, render
from paper_2601_19489_amd import scenes


def test_depth_l1_closed_form():
    D = np.array([[1.0, 2.0], [3.0, 4.0]])
    Dt = np.array([[1.5, 2.0], [2.0, 5.0]])
    loss, g = densify.depth_l1(D, Dt, 0.1)
    assert abs(loss - 0.1 * (0.5 + 0 + 1 + 1) / 4) < 1e-15
    np.testing.assert_array_equal(g, 0.1 / 4 * np.array([[-1, 0], [1, -1]]))


def test_error_mask_by_hand():
    H, W = 1, 5
    target = np.zeros((3, H, W), np.float32)
    image = np.zeros((3, H, W), np.float32)
    # per-pixel L1 errors 0.2, 0.3, 1.2, 2.2, 0.25 (split over channels)
    image[0, 0] = [0.1, 0.1, 0.4, 1.0, 0.25]
    image[1, 0] = [0.1, 0.0, 0.4, 0.7, 0.0]
    image[2, 0] = [0.0, 0.2, 0.4, 0.5, 0.0]
    # normalised: (e - 0.2) / 2.0 = 0, .05, .5, 1, .025 -> > 0.1: F F T T F
    np.testing.assert_array_equal(densify.error_mask(image, target, 0.1)[0],
                                  [False, False, True, True, False])
    # a flat error image has an empty mask
    assert not densify.error_mask(image * 0, target, 0.1).any()
    # strict threshold: an error exactly at min + tau (max - min) is not masked
    image2 = np.zeros((3, 1, 3), np.float32)
    image2[0, 0] = [0.0, 0.25, 1.0]
    np.testing.assert_array_equal(densify.error_mask(image2, np.zeros_like(image2), 0.25)[0],
                                  [False, False, True])


def _pre(d):
    return preprocess.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'],
                                 d['sh'], d['sh_degree'], d['camera'])


def test_split_score_single_isotropic_splat():
    cam = scenes.Camera(48, 40, 60.0, 60.0, 24.0, 20.0, np.eye(3), np.zeros(3))
    sp = dict(u=np.array([20.3]), v=np.array([17.6]), a=np.array([1 / 36.0]), b=np.array([0.0]),
              c=np.array([1 / 36.0]), t=np.array([2 * math.log(255 * 0.8)]),
              opacity=np.array([0.8]), depth=np.array([2.0]), rgb=np.ones((3, 1)),
              visible=np.array([True]))
    vals, ranges, _ = binning.sorted_pairs(sp, cam)
    mask = np.ones((40, 48), bool)
    score, unc = densify.split_score(sp, cam, vals, ranges, mask)
    X, Y = np.meshgrid(np.arange(48) + 0.5, np.arange(40) + 0.5)
    r2 = (X - 20.3) ** 2 + (Y - 17.6) ** 2
    assert score[0] == np.sum(r2 / 36.0 <= sp['t'][0]) and unc[0] == 0
    # half the image masked
    mask[:, 24:] = False
    score, _ = densify.split_score(sp, cam, vals, ranges, mask)
    assert score[0] == np.sum((r2 / 36.0 <= sp['t'][0]) & (X < 24))


def _brute_counts(pre, cam, mask):
    """Per pixel: all Gaussians in (depth bits, index) order, blended set by
    the compositing rule, counted where the mask is set."""
    N = len(pre['u'])
    order = sorted(range(N), key=lambda i: (int(preprocess.depth_key(pre['depth'][i])), i))
    order = [i for i in order if pre['visible'][i] and pre['t'][i] > 0]
    cnt = np.zeros(N, np.int64)
    for y in range(cam.height):
        for x in range(cam.width):
            if not mask[y, x]:
                continue
            T = 1.0
            for i in order:
                Q = render.pixel_q(pre['u'][i], pre['v'][i], pre['a'][i], pre['b'][i],
                                   pre['c'][i], x + 0.5, y + 0.5)[0]
                if Q > pre['t'][i]:
                    continue
                al = min(float(np.float32(0.99)), pre['opacity'][i] * math.exp(-0.5 * Q))
                Tn = T * (1 - al)
                if Tn < float(np.float32(1e-4)):
                    break
                cnt[i] += 1
                T = Tn
    return cnt


def test_split_score_equals_per_pixel_brute_force():
    d = scenes.random_cloud(120, seed=3, width=40, height=36)
    d['log_scales'] = d['log_scales'] + 1.0
    cam = d['camera']
    pre = _pre(d)
    vals, ranges, _ = binning.sorted_pairs(pre, cam)
    rng = np.random.default_rng(4)
    mask = rng.uniform(size=(cam.height, cam.width)) < 0.4
    score, unc = densify.split_score(pre, cam, vals, ranges, mask)
    want = _brute_counts(pre, cam, mask)
    assert unc.sum() == 0
    np.testing.assert_array_equal(score, want)
    assert score.sum() > 100


def test_densify_clone_split_placement():
    N = 4
    means = np.array([[0.0, 1.0, 2.0, 3.0], [0.0] * 4, [0.0] * 4], np.float32)
    ls = np.log(np.array([[0.01, 0.5, 0.02, 0.5], [0.01, 0.1, 0.02, 0.1],
                          [0.01, 0.1, 0.02, 0.1]], np.float32))
    # Gaussian 3 rotated 90 degrees about z: quaternion (cos 45, 0, 0, sin 45)
    c45 = math.cos(math.pi / 4)
    quats = np.array([[1, 1, 1, c45], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, c45]], np.float32)
    op = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    sh = np.arange(12, dtype=np.float32).reshape(1, 3, 4)
    params = dict(means=means, log_scales=ls, quats=quats, opacity_logits=op, sh=sh)
    score = np.array([5, 5, 1, 9])
    eps = np.zeros((2, 3, N), np.float32)
    eps[0, 0] = 1.0
    eps[1, 0] = -2.0
    out, counts = densify.densify(params, 0, score, 5, 0.2, eps)
    # 0 small+selected -> clone; 1 big+selected -> split; 2 unselected; 3 big -> split
    np.testing.assert_array_equal(counts, [2, 2, 1, 2])
    assert out['means'].shape == (3, 7)
    np.testing.assert_array_equal(out['opacity_logits'], op[[0, 0, 1, 1, 2, 3, 3]])
    np.testing.assert_array_equal(out['sh'][0, 0], [0, 0, 1, 1, 2, 3, 3])
    np.testing.assert_allclose(out['means'][:, 2], [1.0 + 0.5, 0, 0], rtol=1e-6)
    np.testing.assert_allclose(out['means'][:, 3], [1.0 - 1.0, 0, 0], atol=1e-7)
    # rotated: the x-axis step maps to +y
    np.testing.assert_allclose(out['means'][:, 5], [3.0, 0.5, 0], atol=1e-6)
    np.testing.assert_allclose(out['means'][:, 6], [3.0, -1.0, 0], atol=1e-6)
    np.testing.assert_allclose(out['log_scales'][:, 2], ls[:, 1] - math.log(1.6), rtol=1e-6)
    np.testing.assert_array_equal(out['log_scales'][:, 0], ls[:, 0])
    np.testing.assert_array_equal(out['means'][:, 1], means[:, 0])


def test_densify_with_pruning_by_hand():
    N = 4
    means = np.array([[0.0, 1.0, 2.0, 3.0], [0.0] * 4, [0.0] * 4], np.float32)
    ls = np.log(np.full((3, N), 0.01, np.float32))
    quats = np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, N))
    op = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    sh = np.arange(12, dtype=np.float32).reshape(1, 3, 4)
    params = dict(means=means, log_scales=ls, quats=quats, opacity_logits=op, sh=sh)
    eps = np.zeros((2, 3, N), np.float32)
    # 0 and 1 selected for growth (clones); 1 and 3 pruned: pruning wins for 1
    prune = np.array([False, True, False, True])
    out, counts = densify.densify(params, 0, np.array([5, 5, 1, 1]), 5, 0.2, eps, prune=prune)
    np.testing.assert_array_equal(counts, [2, 0, 1, 0])
    np.testing.assert_array_equal(out['opacity_logits'], op[[0, 0, 2]])
    np.testing.assert_array_equal(out['means'][0], [0.0, 0.0, 2.0])
    # everything pruned
    out, counts = densify.densify(params, 0, np.zeros(4), 5, 0.2, eps, prune=np.ones(4, bool))
    assert out['means'].shape == (3, 0) and counts.sum() == 0


def _threshold_by_search(score, t_min, cap):
    # definition by exhaustive search over t
    score = np.asarray(score, np.int64)
    for t in range(t_min, densify.SCORE_TOP + 1):
        if int(np.sum(score >= t)) <= cap:
            return t
    return densify.NO_THRESHOLD


def test_growth_threshold_by_hand_and_brute_force():
    s = [0, 3, 3, 7, 1, 9, 3]
    # cap 2: counts >= 4 are {7, 9} -> t = 4 (t = 3 would select 5)
    assert densify.growth_threshold(s, 1, 2) == 4
    # the lower bound wins when the budget is loose
    assert densify.growth_threshold(s, 8, 10) == 8
    assert densify.growth_threshold(s, 1, 7) == 1
    # cap 0: nothing may be selected -> one above the maximum
    assert densify.growth_threshold(s, 1, 0) == 10
    # ties: cap 3 cannot split the three 3s -> t = 4 selects 2
    assert densify.growth_threshold(s, 1, 3) == 4
    # scores at the top of the searched range: no threshold qualifies
    top = densify.SCORE_TOP
    assert densify.growth_threshold([top, top + 5, 2], 1, 1) == densify.NO_THRESHOLD
    assert densify.growth_threshold([top - 1, top + 5, 2], 1, 1) == top
    rng = np.random.default_rng(0)
    for _ in range(40):
        n = int(rng.integers(0, 60))
        sc = rng.integers(0, 40, n) * rng.integers(0, 2, n)
        t_min = int(rng.integers(1, 30))
        cap = int(rng.integers(0, n + 2))
        assert densify.growth_threshold(sc, t_min, cap) == _threshold_by_search(sc, t_min, cap)
