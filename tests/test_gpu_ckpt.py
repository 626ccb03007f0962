"""The checkpointed per-splat backward (the paper's backward design, an
ablation arm here): the checkpointing forward equals the plain forward bit
for bit and reports no overflow when sized from n_contrib; its gradients
match the oracle by the R11 rule (and the pixel-parallel backward's)."""
import math

import numpy as np
import pytest
import torch

from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from _parity import assert_grads_close, exclusions, oracle_pipeline

pytestmark = pytest.mark.gpu
NAMES = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')


def _ckpt_run(R, p, dI, dD, deg):
    n = R.n
    nbk = max(1, math.ceil(int(R.n_contrib.max().item()) / _lib.CKPT_INTERVAL))
    ck = torch.empty(R.n_tiles * nbk * 5 * 256, device='cuda')
    ovf = torch.zeros(1, dtype=torch.int32, device='cuda')
    out = {k: torch.empty_like(getattr(R, k)) for k in ('image', 'depth', 'T_final', 'n_contrib')}
    _lib.gs_render_fwd_ckpt(R.splats, n, R.vals, R.ranges, R.cam, R.bg, out['image'],
                            out['depth'], out['T_final'], out['n_contrib'], ck, nbk, ovf)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    g2 = torch.empty_like(R.grad2d)
    _lib.gs_render_bwd_ckpt(_lib.gaussians(*(p[k] for k in NAMES)), n, deg, R.cam, R.splats,
                            R.vals, R.ranges, out['image'], out['depth'], out['n_contrib'], ck,
                            nbk, dI, dD, g2, _lib.gaussians(*(grads[k] for k in NAMES)))
    torch.cuda.synchronize()
    return out, int(ovf.item()), g2, grads


@pytest.mark.parametrize('n,deg,w,h,depth', [(6000, 2, 200, 136, True), (3000, 0, 96, 64, False)])
def test_checkpointed_backward_matches_oracle(n, deg, w, h, depth):
    d = scenes.surface_cloud(n, seed=31, sh_degree=deg, width=w, height=h)
    cam = d['camera']
    rng = np.random.default_rng(n)
    dI = (rng.standard_normal((3, h, w)) * 1e-3).astype(np.float32)
    dD = (rng.standard_normal((h, w)) * 1e-4).astype(np.float32) if depth else None
    p = params_to_device(d)
    R = Rasterizer(n, cam, deg)
    R.forward(p)
    dIt = torch.as_tensor(dI, device='cuda')
    dDt = None if dD is None else torch.as_tensor(dD, device='cuda')
    plain = R.backward(p, dIt, dDt)
    plain_g2d = R.grad2d.clone()
    out, ovf, g2, grads = _ckpt_run(R, p, dIt, dDt, deg)
    assert ovf == 0
    for k in ('image', 'depth', 'T_final', 'n_contrib'):
        assert torch.equal(out[k], getattr(R, k)), k
    o = oracle_pipeline(d, dI.astype(np.float64), None if dD is None else dD.astype(np.float64))
    ex = exclusions(o['vals'], o['ranges'], cam, o['out'], o['clamp'], n)
    names2d = ('u', 'v', 'a', 'b', 'c', 'opacity', 'r', 'g', 'b_col', 'depth')
    g2n = g2.cpu().numpy().T  # [n][10] records -> [10][n]
    for c, nm in enumerate(names2d):
        if nm == 'depth' and not depth:
            continue
        assert_grads_close(g2n[c], o['grad2d'][c], ex, 'grad2d.' + nm)
    for k in NAMES:
        gg = grads[k].cpu().numpy().reshape(-1, n)
        ww = o['grads'][k].reshape(-1, n)
        pp = plain[k].cpu().numpy().reshape(-1, n)
        for r in range(gg.shape[0]):
            assert_grads_close(gg[r], ww[r], ex, f'{k}[{r}]')
            assert_grads_close(gg[r], pp[r], ex, f'{k}[{r}] vs pixel-parallel')


def test_checkpoint_overflow_is_reported():
    d = scenes.surface_cloud(4000, seed=32, sh_degree=0, width=96, height=64)
    p = params_to_device(d)
    R = Rasterizer(4000, d['camera'], 0)
    R.forward(p)
    assert int(R.n_contrib.max().item()) > _lib.CKPT_INTERVAL  # a second bucket is needed
    ck = torch.empty(R.n_tiles * 1 * 5 * 256, device='cuda')
    ovf = torch.zeros(1, dtype=torch.int32, device='cuda')
    img, dep, Tf = torch.empty_like(R.image), torch.empty_like(R.depth), torch.empty_like(R.T_final)
    nc = torch.empty_like(R.n_contrib)
    _lib.gs_render_fwd_ckpt(R.splats, 4000, R.vals, R.ranges, R.cam, R.bg, img, dep, Tf, nc, ck,
                            1, ovf)
    torch.cuda.synchronize()
    assert int(ovf.item()) != 0
    assert torch.equal(img, R.image)
