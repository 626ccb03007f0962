"""The training step's backward fused with the Adam step
(gs_render_bwd_adam) against the two-call sequence it replaces: the image-
and parameter-space backward (Sec. 2.2) into gradient arrays, then
gs_adam_step_grouped. Parameters, both moments and the step count must be
equal bit for bit after every step, for each SH degree and for directly
stored colours, on scenes that hold Gaussians behind the camera and
Gaussians whose projection is rejected after the near-plane test passed
(an overflowing scale)."""
import math

import numpy as np
import pytest
import torch

from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.rasterizer import PARAM_NAMES, Adam, Rasterizer, l1_loss, params_to_device

pytestmark = pytest.mark.gpu

LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3)


def _scene(deg, seed, n=20000, w=320, h=240):
    d = scenes.surface_cloud(n, seed=seed, sh_degree=max(deg, 0), width=w, height=h)
    if deg == _lib.GS_DIRECT:  # activated attributes, as the anchor decoder emits them
        c0 = 0.5 / math.sqrt(math.pi)
        d = dict(d, log_scales=np.exp(d['log_scales']).astype(np.float32),
                 opacity_logits=(1 / (1 + np.exp(-d['opacity_logits']))).astype(np.float32),
                 sh=(d['sh'][0] * c0 + 0.5).reshape(1, 3, -1).astype(np.float32), sh_degree=-1)
    d['camera'] = scenes.look_at_camera((0.5, -0.3, -3.8), (0, 0, 0), w, h)
    m = d['means']
    m[2, :64] = -9.0  # behind the camera
    if deg != _lib.GS_DIRECT:
        d['log_scales'][:, 64:80] = 400.0  # exp overflows: rejected after the near-plane test
    return d


def _bits(t):
    return t.contiguous().view(torch.int32)


def _same(a, b):
    return torch.equal(_bits(a), _bits(b))


@pytest.mark.parametrize('deg', [3, 1, 0, _lib.GS_DIRECT])
def test_fused_step_equals_backward_then_adam(deg):
    d = _scene(deg, seed=21 + deg)
    n = d['means'].shape[1]
    target = torch.as_tensor(d['target'], device='cuda')
    pa = params_to_device(d)
    pb = {k: v.clone() for k, v in pa.items()}
    oa, ob = Adam(pa, LRS), Adam(pb, LRS)
    R = Rasterizer(n, d['camera'], deg)
    for step in range(3):
        img_a, dep_a = R.forward(pa)
        _, dL_a = l1_loss(img_a, target)
        dD_a = (dep_a - 3.0) * 1e-4 if step != 1 else None
        grads = R.backward(pa, dL_a, dD_a)
        oa.step(grads)

        img_b, dep_b = R.forward(pb)
        assert _same(img_b, img_a) and _same(dep_b, dep_a), step  # same parameters so far
        _, dL_b = l1_loss(img_b, target)
        dD_b = (dep_b - 3.0) * 1e-4 if step != 1 else None
        R.backward_adam(pb, dL_b, ob, dD_b)
        torch.cuda.synchronize()
        for k in PARAM_NAMES:
            assert _same(pa[k], pb[k]), (step, k)
            assert _same(oa.m[k], ob.m[k]), (step, k, 'm')
            assert _same(oa.v[k], ob.v[k]), (step, k, 'v')
        assert int(oa.step_count.item()) == int(ob.step_count.item()) == step + 1
    # the step did move the parameters, and the rejected Gaussians only decayed
    p0 = params_to_device(d)
    assert not torch.equal(pb['means'], p0['means'])
    if deg != _lib.GS_DIRECT:
        assert torch.equal(ob.m['sh'][:, :, 64:80], torch.zeros_like(ob.m['sh'][:, :, 64:80]))


def test_fused_step_rejects_bad_arguments():
    d = _scene(0, seed=5, n=500, w=64, h=48)
    p = params_to_device(d)
    R = Rasterizer(500, d['camera'], 0)
    img, _ = R.forward(p)
    _, dL = l1_loss(img, torch.as_tensor(d['target'], device='cuda'))
    opt = Adam(p, LRS)
    good = opt.fused_params()
    bad = opt.fused_params()
    bad.step = None
    with pytest.raises(RuntimeError):
        _lib.gs_render_bwd_adam(_lib.gaussians(*(p[k] for k in PARAM_NAMES)), 500, 0, R.cam,
                                R.splats, R.vals, R.ranges, R.bg, R.T_final, R.n_contrib, dL,
                                None, R.grad2d, bad)
    bad = opt.fused_params()
    bad.v.sh = None
    with pytest.raises(RuntimeError):
        _lib.gs_render_bwd_adam(_lib.gaussians(*(p[k] for k in PARAM_NAMES)), 500, 0, R.cam,
                                R.splats, R.vals, R.ranges, R.bg, R.T_final, R.n_contrib, dL,
                                None, R.grad2d, bad)
    # n = 0 takes the step and touches nothing else
    _lib.gs_render_bwd_adam(_lib.gaussians(*(p[k] for k in PARAM_NAMES)), 0, 0, R.cam, R.splats,
                            R.vals, R.ranges, R.bg, R.T_final, R.n_contrib, dL, None, R.grad2d,
                            good)
    torch.cuda.synchronize()
    assert int(opt.step_count.item()) == 1
