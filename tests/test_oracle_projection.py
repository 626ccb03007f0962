"""Pins of the oracle's per-Gaussian projection (EWA, Sec. 2.1 preprocess):
closed form on the optical axis, Monte-Carlo covariance of projected
samples, finite-difference Jacobian of the perspective map, culling and the
Eq. (1) threshold."""
import math

import numpy as np

from oracle import preprocess
from paper_2601_19489_amd.scenes import Camera, look_at_camera


def _one(mean, log_scale, quat=(1, 0, 0, 0), logit=0.0, cam=None, sh_deg=0, shc=None):
    cam = cam or look_at_camera((0, 0, -4), (0, 0, 0), 64, 64)
    K = (sh_deg + 1) ** 2
    shc = np.zeros((K, 3, 1)) if shc is None else shc
    return preprocess.preprocess(np.asarray(mean, float).reshape(3, 1),
                                 np.asarray(log_scale, float).reshape(3, 1),
                                 np.asarray(quat, float).reshape(4, 1),
                                 np.array([logit], float), shc, sh_deg, cam,
                                 store=np.float64), cam


def test_isotropic_on_axis_closed_form():
    sigma, z = 0.05, 3.0
    pre, cam = _one((0, 0, z - 4.0), [math.log(sigma)] * 3)
    s2 = (cam.fx * sigma / z) ** 2 + 0.3
    assert abs(pre['a'][0] - 1 / s2) < 1e-12 * (1 / s2)
    assert abs(pre['c'][0] - 1 / s2) < 1e-12 * (1 / s2)
    assert abs(pre['b'][0]) < 1e-15
    assert abs(pre['u'][0] - cam.cx) < 1e-12 and abs(pre['v'][0] - cam.cy) < 1e-12
    assert abs(pre['depth'][0] - z) < 1e-14


def test_projected_covariance_matches_monte_carlo():
    # tiny anisotropic rotated Gaussian off-axis; project samples exactly
    # and compare their covariance with Sigma' - 0.3 I (first-order EWA)
    cam = look_at_camera((1.0, -0.5, -4.0), (0, 0, 0), 200, 150)
    mean = np.array([0.3, -0.2, 0.5])
    ls = np.log([0.004, 0.002, 0.003])
    q = np.array([0.8, 0.3, -0.4, 0.33]); q /= np.linalg.norm(q)
    pre, _ = _one(mean, ls, q, cam=cam)
    R = preprocess.quat_to_rotmat(q.reshape(4, 1))[0]
    L = R @ np.diag(np.exp(ls))
    rng = np.random.default_rng(0)
    X = mean[:, None] + L @ rng.standard_normal((3, 400_000))
    P = cam.R @ X + cam.t[:, None]
    uv = np.stack([cam.fx * P[0] / P[2] + cam.cx, cam.fy * P[1] / P[2] + cam.cy])
    emp = np.cov(uv)
    S2 = pre['_S2'][0] - 0.3 * np.eye(2)
    np.testing.assert_allclose(emp, S2, rtol=2e-2, atol=2e-2 * np.abs(S2).max())
    # centroid = projection of the mean
    np.testing.assert_allclose([pre['u'][0], pre['v'][0]], uv.mean(axis=1), atol=5e-3)


def test_jacobian_matches_finite_differences():
    cam = look_at_camera((0.5, 0.2, -4.0), (0, 0, 0), 120, 90)
    mean = np.array([0.2, 0.1, -0.3])
    pre, _ = _one(mean, [-3, -3, -3], cam=cam)
    p = cam.R @ mean + cam.t

    def proj(pp):
        return np.array([cam.fx * pp[0] / pp[2], cam.fy * pp[1] / pp[2]])

    h = 1e-6
    Jfd = np.stack([(proj(p + h * e) - proj(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    np.testing.assert_allclose(pre['_J'][0], Jfd, rtol=1e-7, atol=1e-9)


def test_jacobian_clamp_outside_fov():
    cam = look_at_camera((0, 0, -4), (0, 0, 0), 64, 64)
    # far off to the side: x/z beyond 1.3 tan(fov/2)
    pre, _ = _one((4.0, 0.0, 0.0), [-3, -3, -3], cam=cam)
    xr = pre['_xr'][0]
    lim = 1.3 * cam.width / (2 * cam.fx)
    assert xr > lim
    assert abs(pre['_J'][0, 0, 2] - (-cam.fx * lim / pre['_pz'][0])) < 1e-12


def test_near_plane_cull():
    pre, _ = _one((0, 0, -3.85), [-3, -3, -3])  # p_z = 0.15 <= 0.2
    assert not pre['visible'][0]
    pre, _ = _one((0, 0, -3.7), [-3, -3, -3])   # p_z = 0.3
    assert pre['visible'][0]


def test_threshold_eq1():
    for logit in (-3.0, 0.0, 2.5):
        pre, _ = _one((0, 0, 0), [-3, -3, -3], logit=logit)
        o = 1 / (1 + math.exp(-logit))
        assert abs(pre['t'][0] - 2 * math.log(255 * o)) < 1e-13
    # o < 1/255 -> t < 0
    pre, _ = _one((0, 0, 0), [-3, -3, -3], logit=-6.0)
    assert pre['t'][0] < 0


def test_view_direction_and_colour():
    # camera at the origin of -z looking at +z; Gaussian straight ahead:
    # dir = (0,0,1), only Y_10 = sqrt(3/4pi) z is nonzero at degree 1
    shc = np.zeros((4, 3, 1))
    shc[2, :, 0] = [1.0, -1.0, 0.2]
    pre, _ = _one((0, 0, 1.0), [-3, -3, -3], sh_deg=1, shc=shc)
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(pre['rgb'][:, 0], np.maximum([0.5 + c1, 0.5 - c1, 0.5 + 0.2 * c1], 0),
                               atol=1e-14)
