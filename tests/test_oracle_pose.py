"""Pins of the oracle's camera pose gradient (global pose refinement, Sec. 2.5
first round): Rodrigues' formula against scipy's rotation vectors, and the
analytic gradient of a random linear functional of the rendered image and
depth with respect to (omega, delta) against central differences of the
FP64 forward under the perturbed camera, with every tile set and blend
decision checked unchanged."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import binning, pose, preprocess, render
from paper_2601_19489_amd import scenes

from test_oracle_grad import _scene


def test_rodrigues_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(5):
        w = rng.normal(0, 0.7, 3)
        np.testing.assert_allclose(pose.rodrigues(w), Rotation.from_rotvec(w).as_matrix(),
                                   atol=1e-14)
    np.testing.assert_allclose(pose.rodrigues(np.zeros(3)), np.eye(3))
    # apply_pose moves camera-space points by p' = Q p + delta
    cam = scenes.look_at_camera((0.5, -0.2, -3.0), (0, 0, 0), 32, 30)
    c2 = pose.apply_pose(cam, [0.1, -0.2, 0.05], [0.01, 0.02, -0.03])
    X = np.array([0.3, -0.1, 0.4])
    p = cam.R @ X + cam.t
    np.testing.assert_allclose(c2.R @ X + c2.t,
                               pose.rodrigues([0.1, -0.2, 0.05]) @ p + [0.01, 0.02, -0.03],
                               atol=1e-14)


def _forward(p, deg, cam, bg):
    pre = preprocess.preprocess(p['means'], p['log_scales'], p['quats'], p['opacity_logits'],
                                p['sh'], deg, cam, store=np.float64)
    vals, ranges, _ = binning.sorted_pairs(pre, cam)
    return pre, vals, ranges, render.render(pre, cam, vals, ranges, bg=bg)


@pytest.mark.parametrize('seed,deg,n,eye,mode', [(0, 3, 12, (0.6, -0.4, -3.5), 0),
                                                 (1, 1, 16, (0.2, 0.3, -3.0), 1),
                                                 (3, -1, 14, (0.3, 0.2, -3.2), 0)])
def test_pose_gradient_matches_central_differences(seed, deg, n, eye, mode):
    cam = scenes.look_at_camera(eye, (0, 0, 0), 32, 30)
    cam.depth_mode = mode
    bg = (0.2, 0.1, 0.3)
    p = _scene(n, seed, deg)
    rng = np.random.default_rng(200 + seed)
    dC = rng.standard_normal((3, cam.height, cam.width))
    dD = rng.standard_normal((cam.height, cam.width)) * (0.3 if mode == 0 else 3.0)
    pre, vals, ranges, out = _forward(p, deg, cam, bg)
    assert out['n_blended'].max() >= 3
    g2d, _ = render.render_backward(pre, cam, vals, ranges, dC, dD, bg=bg)
    ana = pose.pose_gradient(pre, g2d, deg, cam)
    h = 1e-7
    fd = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Ls = []
        for sgn in (1, -1):
            c = pose.apply_pose(cam, sgn * e[:3], sgn * e[3:])
            _, v, r, o = _forward(p, deg, c, bg)
            for a, b in ((v, vals), (r, ranges), (o['n_blended'], out['n_blended']),
                         (o['n_contrib'], out['n_contrib'])):
                assert np.array_equal(a, b), 'perturbation changed a discrete decision'
            Ls.append(np.sum(dC * o['image']) + np.sum(dD * o['depth']))
        fd[k] = (Ls[0] - Ls[1]) / (2 * h)
    scale = np.abs(fd).mean()
    np.testing.assert_allclose(ana, fd, rtol=1e-5, atol=1e-6 * scale)
