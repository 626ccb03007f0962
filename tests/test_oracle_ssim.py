"""Pins of the oracle's Eq. 5 photometric loss and Eq. 6 pruning score
(Sec. 3.2): the window against scipy's Gaussian filter, SSIM
special cases with closed forms (identical images, a scaled copy, a constant
shift), the SSIM and Eq. 5 gradients against central differences, and the
pruning score and mask on hand cases."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import ssim as ossim


def _gf(img):
    # scipy's Gaussian filter with the same radius (5) and zero padding
    return ndimage.gaussian_filter(img, ossim.SIGMA, mode='constant', cval=0.0,
                                   truncate=5.0 / ossim.SIGMA)


def test_window_matches_scipy_gaussian_filter():
    g = ossim.window_1d()
    assert abs(g.sum() - 1) < 1e-15 and np.allclose(g, g[::-1], rtol=0, atol=0)
    assert abs(g[5] / g[4] - math.exp(1 / (2 * 1.5 ** 2))) < 1e-12
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, (23, 31))
    np.testing.assert_allclose(ossim._filter(img), _gf(img), rtol=0, atol=1e-14)


def test_ssim_of_identical_images_is_one():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (3, 20, 17))
    np.testing.assert_allclose(ossim.ssim_map(x, x), 1.0, rtol=0, atol=1e-14)
    assert abs(ossim.ssim(x, x) - 1.0) < 1e-14


@pytest.mark.parametrize('a', [0.5, 1.7, -0.8])
def test_ssim_of_a_scaled_copy_closed_form(a):
    # y = a x everywhere (padding included): mu_y = a mu_x, var_y = a^2 var_x,
    # cov = a var_x at every pixel, so S has a closed form in (mu_x, var_x)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (1, 19, 24))
    mx = _gf(x[0])
    vx = _gf(x[0] ** 2) - mx ** 2
    C1, C2 = ossim.C1, ossim.C2
    want = ((2 * a * mx ** 2 + C1) * (2 * a * vx + C2) /
            (((1 + a * a) * mx ** 2 + C1) * ((1 + a * a) * vx + C2)))
    np.testing.assert_allclose(ossim.ssim_map(x, a * x)[0], want, rtol=1e-10, atol=1e-12)


def test_ssim_constant_shift_interior_is_the_luminance_term():
    # y = x + c: away from the border (windows inside the image) the variances
    # and the covariance agree, leaving (2 mu_x mu_y + C1) / (mu_x^2 + mu_y^2 + C1)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 0.7, (1, 30, 30))
    c = 0.25
    S = ossim.ssim_map(x, x + c)[0]
    mx = _gf(x[0])
    my = mx + c
    want = (2 * mx * my + ossim.C1) / (mx ** 2 + my ** 2 + ossim.C1)
    np.testing.assert_allclose(S[5:-5, 5:-5], want[5:-5, 5:-5], rtol=1e-9)
    assert np.all(S <= 1 + 1e-12)


def _fd(f, x, h=1e-6):
    g = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        g[idx] = (f(xp) - f(xm)) / (2 * h)
    return g


def test_ssim_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (2, 9, 13))
    y = np.clip(x + rng.normal(0, 0.2, x.shape), 0, 1)
    ana = ossim.ssim_grad(x, y)
    fd = _fd(lambda z: ossim.ssim(z, y), x)
    np.testing.assert_allclose(ana, fd, rtol=1e-6, atol=1e-10 * np.abs(fd).max())


def test_photo_loss_and_gradient():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (3, 8, 10))
    y = rng.uniform(0, 1, (3, 8, 10))
    E, l1, s = ossim.photo_loss(x, y)
    assert abs(l1 - np.mean(np.abs(x - y))) < 1e-15
    assert abs(E - (0.8 * l1 + 0.2 * (1 - s))) < 1e-15
    # away from |x - y| = 0 the L1 term is differentiable
    assert np.min(np.abs(x - y)) > 1e-5
    ana = ossim.photo_loss_grad(x, y)
    fd = _fd(lambda z: ossim.photo_loss(z, y)[0], x)
    np.testing.assert_allclose(ana, fd, rtol=1e-6, atol=1e-10 * np.abs(fd).max())


def test_prune_score_and_mask_by_hand():
    counts = np.array([[0, 3, 5, 1], [2, 0, 5, 1]])
    errors = np.array([0.5, 0.25])
    s = ossim.prune_score(counts, errors)
    np.testing.assert_allclose(s, [0.5, 1.5, 3.75, 0.75])
    # normalised: 0, 1/3.25, 1, 0.25/3.25 -> above 0.2: F T T F
    np.testing.assert_array_equal(ossim.prune_mask(s, 0.2), [False, True, True, False])
    # strict: a score exactly at the threshold is kept
    np.testing.assert_array_equal(ossim.prune_mask([0.0, 0.5, 1.0], 0.5), [False, False, True])
    # all equal: nothing pruned; empty input
    assert not ossim.prune_mask([2.0, 2.0], 0.0).any()
    assert ossim.prune_mask([], 0.5).size == 0
