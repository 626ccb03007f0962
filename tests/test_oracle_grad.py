"""Pin of the oracle's backward (Sec. 2.2 gradients; 3DGS chain rule): its
analytic gradient of a random linear functional of the rendered image and
depth equals central finite differences of its own FP64 forward, on tiny
scenes, with every tile set and blend decision checked to be unchanged
under the perturbation."""
import math

import numpy as np
import pytest

from oracle import backward, binning, preprocess, render
from paper_2601_19489_amd import scenes

PARAMS = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')


def _scene(n, seed, deg):
    rng = np.random.default_rng(seed)
    if deg == preprocess.DIRECT:   # already-activated attributes (decoder output)
        return dict(
            means=rng.uniform(-0.5, 0.5, (3, n)),
            log_scales=np.exp(rng.normal(-1.6, 0.4, (3, n))),
            quats=rng.standard_normal((4, n)) * np.array([[2.0], [1], [1], [1]]),
            opacity_logits=rng.uniform(0.2, 0.95, n),
            sh=rng.uniform(0.05, 0.95, (1, 3, n)),
        )
    K = (deg + 1) ** 2
    return dict(
        means=rng.uniform(-0.5, 0.5, (3, n)),
        log_scales=rng.normal(-1.6, 0.4, (3, n)),
        quats=rng.standard_normal((4, n)) * np.array([[2.0], [1], [1], [1]]),
        opacity_logits=rng.normal(0.5, 1.0, n),
        sh=np.concatenate([rng.uniform(-0.8, 0.8, (1, 3, n)), rng.normal(0, 0.3, (K - 1, 3, n))]),
    )


def _forward(p, deg, cam, bg):
    pre = preprocess.preprocess(p['means'], p['log_scales'], p['quats'], p['opacity_logits'],
                                p['sh'], deg, cam, store=np.float64)
    vals, ranges, _ = binning.sorted_pairs(pre, cam)
    out = render.render(pre, cam, vals, ranges, bg=bg)
    return pre, vals, ranges, out


@pytest.mark.parametrize('seed,deg,n,eye,mode', [(0, 3, 10, (0.6, -0.4, -4.0), 0),
                                                 (1, 1, 16, (0.0, 0.0, -3.0), 0),
                                                 (2, 0, 20, (-1.0, 0.5, -3.5), 0),
                                                 (3, -1, 14, (0.3, 0.2, -3.2), 0),
                                                 (4, 1, 14, (0.5, 0.3, -3.0), 1)])
def test_backward_matches_central_differences(seed, deg, n, eye, mode):
    cam = scenes.look_at_camera(eye, (0, 0, 0), 32, 30)
    cam.depth_mode = mode   # 1: the depth channel carries inverse depth
    bg = (0.2, 0.1, 0.3)
    p = _scene(n, seed, deg)
    rng = np.random.default_rng(100 + seed)
    dC = rng.standard_normal((3, cam.height, cam.width))
    dD = rng.standard_normal((cam.height, cam.width)) * (0.3 if mode == 0 else 3.0)

    pre, vals, ranges, out = _forward(p, deg, cam, bg)
    assert out['n_blended'].max() >= 3, 'scene too sparse to exercise blending'
    g2d, _ = render.render_backward(pre, cam, vals, ranges, dC, dD, bg=bg)
    grads = backward.preprocess_backward(pre, g2d, deg, cam)

    def L(q):
        _, v, r, o = _forward(q, deg, cam, bg)
        return np.sum(dC * o['image']) + np.sum(dD * o['depth']), v, r, o

    skipped = 0
    for name in PARAMS:
        ana = grads[name]
        fd = np.zeros_like(ana)
        for idx in np.ndindex(*p[name].shape):
            x0 = p[name][idx]
            h = 1e-6 * max(1.0, abs(x0))
            qp = {k: v.copy() for k, v in p.items()}
            qm = {k: v.copy() for k, v in p.items()}
            qp[name][idx] = x0 + h
            qm[name][idx] = x0 - h
            Lp, vp, rp, op = L(qp)
            Lm, vm, rm, om = L(qm)
            same = all(np.array_equal(a, b) for a, b in
                       ((vp, vals), (vm, vals), (rp, ranges), (rm, ranges),
                        (op['n_blended'], out['n_blended']), (om['n_blended'], out['n_blended']),
                        (op['n_contrib'], out['n_contrib']), (om['n_contrib'], out['n_contrib'])))
            if not same:
                fd[idx] = np.nan
                skipped += 1
                continue
            fd[idx] = (Lp - Lm) / (2 * h)
        ok = ~np.isnan(fd)
        scale = np.mean(np.abs(fd[ok])) + 1e-30
        err = np.abs(ana[ok] - fd[ok])
        assert np.all(err <= 1e-5 * (np.abs(fd[ok]) + scale)), (name, err.max(), scale)
    assert skipped <= 3
