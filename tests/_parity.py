"""Shared helpers for the GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import os

import numpy as np

from oracle import backward as obwd
from oracle import binning as obin
from oracle import preprocess as opre
from oracle import render as oren

IMG_TOL = 1e-4        # max-abs on unflagged pixels
FLAG_TOL = 5e-3       # max-abs on flagged (knife-edge) pixels
GRAD_TOL = 1e-3       # relative, per element (with the tensor mean) and per tensor


def oracle_pre(d):
    return opre.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'], d['sh'],
                           d['sh_degree'], d['camera'])


def gpu_splat_fields(splats):
    """Named columns of the FP32 splat records (numpy [n, 12])."""
    s = np.asarray(splats)
    return dict(u=s[:, 0], v=s[:, 1], a=s[:, 2], b=s[:, 3], c=s[:, 4], t=s[:, 5], opacity=s[:, 6],
                dval=s[:, 7], rgb=s[:, 8:11].T)


def assert_preprocess_close(gpu, pre, visible_only=True, max_ulps=2):
    """FP32 outputs of the FP64 computation: equal up to a few ulps (the two
    FP64 evaluations may round differently in the last bit)."""
    vis = pre['visible']
    for k in ('u', 'v', 'a', 'b', 'c', 't', 'opacity', 'dval'):
        g = np.asarray(gpu[k], np.float32)[vis]
        o = np.asarray(pre[k], np.float32)[vis]
        ulp = np.abs(g.view(np.int32).astype(np.int64) - o.view(np.int32).astype(np.int64))
        finite = np.isfinite(o)
        assert np.all(ulp[finite] <= max_ulps), (k, int(ulp[finite].max()))
    g = np.asarray(gpu['rgb'], np.float32)[:, vis]
    o = np.asarray(pre['rgb'], np.float32)[:, vis]
    np.testing.assert_allclose(g, o, rtol=1e-6, atol=1e-6)


def flagged_gaussians(vals, ranges, cam, out):
    """Gaussians whose blending a knife-edge stop test can flip: at each
    flagged pixel, the list entries from its first knife-edge test to one
    past its last contributor. Excluded from the gradient check."""
    ex = set()
    for y, x in zip(*np.nonzero(out['ambiguous'])):
        tid = obin.tile_id(cam, x // cam.tile, y // cam.tile)
        s, e = int(ranges[tid]), int(ranges[tid + 1])
        a = int(out['ambiguous_from'][y, x])
        m = int(out['n_contrib'][y, x])
        ex.update(int(v) for v in vals[s + max(0, min(a, m) - 1):min(e, s + m + 2)])
    return np.array(sorted(ex), np.int64)


# per-test counts of what the parity checks leave out, printed at the end of
# the run (conftest.pytest_terminal_summary)
REPORT = []


def exclusions(vals, ranges, cam, out, clamp, n_gauss):
    """Gaussians left out of the gradient check: those whose blending a
    knife-edge stop test can flip, and those blended with o G within the
    FP32 error of the 0.99 clamp. The counts are recorded for the summary."""
    ex = np.union1d(flagged_gaussians(vals, ranges, cam, out), np.nonzero(clamp)[0])
    done = out.get('done')
    done = np.ones_like(out['ambiguous']) if done is None else done
    REPORT.append(dict(
        test=os.environ.get('PYTEST_CURRENT_TEST', '?').split(' ')[0],
        tile=cam.tile, pixels=int(done.sum()), flagged_px=int((out['ambiguous'] & done).sum()),
        stopped_px=int((out['stopped'] & done).sum()),
        clamped_blends=int(out['n_clamped'][done].sum()),
        gaussians=int(n_gauss), excluded=int(len(ex)), clamp_excluded=int(np.sum(clamp))))
    return ex


def assert_image_close(gpu_img, want_img, flags, done=None, tol=IMG_TOL):
    g = np.asarray(gpu_img, np.float64)
    w = np.asarray(want_img, np.float64)
    mask = ~flags if done is None else (~flags & done)
    if g.ndim == 3:
        err = np.abs(g - w).max(axis=0)
    else:
        err = np.abs(g - w)
    sel = done if done is not None else np.ones_like(flags)
    assert err[mask].max(initial=0.0) <= tol, float(err[mask].max())
    if np.any(flags & sel):
        assert err[flags & sel].max() <= FLAG_TOL, float(err[flags & sel].max())


def assert_grads_close(got, want, exclude=None, name='', tol=GRAD_TOL):
    """Per element |g - w| <= tol (|w| + mean|w|) and ||g - w|| <= tol ||w||
    over the Gaussians (last axis) not excluded."""
    g = np.asarray(got, np.float64)
    w = np.asarray(want, np.float64)
    keep = np.ones(w.shape[-1], bool)
    if exclude is not None and len(exclude):
        keep[exclude] = False
    g, w = g[..., keep], w[..., keep]
    scale = np.mean(np.abs(w))
    if scale == 0:
        assert np.all(g == 0), name
        return
    err = np.abs(g - w)
    bad = err > tol * (np.abs(w) + scale)
    assert not bad.any(), (name, int(bad.sum()), float(err.max()), float(scale))
    rel = np.linalg.norm(g - w) / np.linalg.norm(w)
    assert rel <= tol, (name, rel)


def oracle_pipeline(d, dL_dimage=None, dL_ddepth=None, bg=(0.0, 0.0, 0.0)):
    cam = d['camera']
    pre = oracle_pre(d)
    counts = obin.tile_counts(pre, cam)
    vals, ranges, keys = obin.sorted_pairs(pre, cam)
    out = oren.render(pre, cam, vals, ranges, bg=bg)
    res = dict(pre=pre, counts=counts, vals=vals, ranges=ranges, keys=keys, out=out)
    if dL_dimage is not None:
        g2d, clamp = oren.render_backward(pre, cam, vals, ranges, dL_dimage, dL_ddepth, bg=bg)
        res['grad2d'] = g2d
        res['clamp'] = clamp
        res['grads'] = obwd.preprocess_backward(pre, g2d, d['sh_degree'], cam)
    return res
