"""GPU parity of the camera pose gradient (global pose refinement) against
the oracle through the C ABI, and pose refinement on a synthetically
perturbed camera.

Bars: with the oracle's image-space gradients as input, the 6-vector within
1e-8 relative (both sides FP64 from the same FP32 parameters); end to end
from the GPU backward, within 1e-3 of the oracle in norm (the R11 bar); the
refined pose error at most half the initial one."""
import math

import numpy as np
import pytest
import torch

from oracle import pose as opose
from oracle import render as oren
from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.pose import PoseRefiner, corrected
from paper_2601_19489_amd.rasterizer import Rasterizer, l1_loss, params_to_device

from _parity import oracle_pipeline, oracle_pre

pytestmark = pytest.mark.gpu
NAMES = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')


def _scene(deg, seed, n=3000, w=96, h=80):
    d = scenes.surface_cloud(n, seed=seed, sh_degree=max(deg, 0), width=w, height=h)
    if deg == _lib.GS_DIRECT:   # activated attributes, as the anchor decoder emits them
        c0 = 0.5 / math.sqrt(math.pi)
        d = dict(d, log_scales=np.exp(d['log_scales']).astype(np.float32),
                 opacity_logits=(1 / (1 + np.exp(-d['opacity_logits']))).astype(np.float32),
                 sh=(d['sh'][0] * c0 + 0.5).reshape(1, 3, -1).astype(np.float32), sh_degree=-1)
    d['camera'] = scenes.look_at_camera((0.7, -0.3, -3.6), (0, 0, 0), w, h)
    return d


def _gpu_pose(d, grad2d):
    p = params_to_device(d)
    n = p['means'].shape[1]
    out = torch.zeros(6, dtype=torch.float64, device='cuda')
    # the oracle's [10][n] components as the library's [n][10] records
    g2 = torch.as_tensor(np.ascontiguousarray(np.asarray(grad2d, np.float64).T), device='cuda')
    _lib.gs_pose_grad(_lib.gaussians(*(p[k] for k in NAMES)), n, d['sh_degree'],
                      _lib.camera(d['camera']), g2, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize('deg,mode,seed', [(3, 0, 0), (1, 1, 1), (_lib.GS_DIRECT, 0, 2)])
def test_pose_grad_matches_oracle_on_the_same_image_gradients(deg, mode, seed):
    d = _scene(deg, seed)
    cam = d['camera']
    cam.depth_mode = mode
    rng = np.random.default_rng(seed + 40)
    dI = rng.standard_normal((3, cam.height, cam.width)) * 1e-3
    dD = rng.standard_normal((cam.height, cam.width)) * 1e-3
    o = oracle_pipeline(d, dI, dD)
    want = opose.pose_gradient(o['pre'], o['grad2d'], deg, cam)
    got = _gpu_pose(d, o['grad2d'])
    assert np.linalg.norm(want) > 0
    np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-10 * np.linalg.norm(want))


def test_pose_grad_end_to_end_from_the_gpu_backward():
    d = _scene(2, 5, n=4000)
    cam = d['camera']
    rng = np.random.default_rng(9)
    dI = (rng.standard_normal((3, cam.height, cam.width)) * 1e-3).astype(np.float32)
    p = params_to_device(d)
    n = p['means'].shape[1]
    R = Rasterizer(n, cam, 2)
    R.forward(p)
    R.backward(p, torch.as_tensor(dI, device='cuda'))
    out = torch.zeros(6, dtype=torch.float64, device='cuda')
    _lib.gs_pose_grad(_lib.gaussians(*(p[k] for k in NAMES)), n, 2, R.cam, R.grad2d, out)
    torch.cuda.synchronize()
    o = oracle_pipeline(d, dI.astype(np.float64))
    want = opose.pose_gradient(o['pre'], o['grad2d'], 2, cam)
    got = out.cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-3 * np.linalg.norm(want)


def _pose_error(c, ref):
    Rd = np.asarray(c.R) @ np.asarray(ref.R).T
    ang = math.acos(max(-1.0, min(1.0, (np.trace(Rd) - 1) / 2)))
    centre = lambda k: -np.asarray(k.R).T @ np.asarray(k.t)
    return ang, float(np.linalg.norm(centre(c) - centre(ref)))


def test_refinement_recovers_a_perturbed_camera():
    d = scenes.surface_cloud(20_000, seed=31, sh_degree=0, width=128, height=96)
    true_cam = scenes.look_at_camera((0.4, -0.3, -3.4), (0, 0, 0), 128, 96)
    p = params_to_device(d)
    n = p['means'].shape[1]
    R = Rasterizer(n, true_cam, 0)
    R.forward(p)
    gt = R.image.clone()
    start = corrected(true_cam, [0.012, -0.009, 0.006], [0.03, -0.02, 0.025])
    ref = PoseRefiner([start], lr_rot=1e-3, lr_trans=3e-3, every=1)
    e0 = _pose_error(start, true_cam)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    for s in range(1, 151):
        R.cam = ref.camera(0)
        R.forward(p)
        _, dI = l1_loss(R.image, gt)
        R.backward(p, dI, None, grads)
        ref.accumulate(0, _lib.gaussians(*(p[k] for k in NAMES)), n, 0, R.grad2d)
        ref.step(s)
    e1 = _pose_error(ref.cams[0], true_cam)
    print('pose error (rad, centre distance):', e0, '->', e1)
    assert e1[0] <= 0.5 * e0[0] and e1[1] <= 0.5 * e0[1]
