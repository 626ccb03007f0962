"""Batched multi-view step: the batched entry points (one preprocess launch,
persistent forward / backward launches over the (view, tile) queue, grouped
Adam with a device step count) against the single-view path and the
oracle, the captured HIP graph against eager steps, and the autotuner.
"""
import numpy as np
import pytest
import torch

from oracle import backward as obwd
from oracle import binning as obin
from oracle import render as oren
from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.batched import BatchedRasterizer, TrainStep, autotune
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from _parity import (assert_grads_close, assert_image_close, exclusions, oracle_pre)

pytestmark = pytest.mark.gpu

SMALL_RES = ((96, 64), (128, 72), (80, 80), (144, 81))
LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3)


def _small(n=3000, seed=3, deg=1):
    d = scenes.surface_cloud(n, seed=seed, sh_degree=deg, width=64, height=64)
    cams = scenes.orbit_cameras(4, seed=seed, radius=3.2, resolutions=SMALL_RES)
    return d, cams


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize('tile', [8, 16, 32])
def test_batched_equals_single_view_calls(tile):
    d, cams = _small()
    p = params_to_device(d)
    n = p['means'].shape[1]
    B = BatchedRasterizer(n, cams, d['sh_degree'], tile=tile)
    B.size_pairs(p)
    B.forward(p)
    rng = np.random.default_rng(9)
    dIs = []
    for b in B.buf:
        dI = torch.as_tensor(rng.standard_normal(b['image'].shape).astype(np.float32) * 1e-3,
                             device='cuda')
        b['dL_dimage'].copy_(dI)
        dIs.append(dI)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    B.backward(p, grads)
    torch.cuda.synchronize()
    acc = {k: torch.zeros_like(v) for k, v in p.items()}
    for v, c in enumerate(cams):
        R = Rasterizer(n, c, d['sh_degree'], tile=tile)
        R.forward(p)
        b = B.buf[v]
        P = B.pair_counts()[v]
        np.testing.assert_array_equal(_u32(R.ranges), _u32(b['ranges']))
        np.testing.assert_array_equal(_u32(R.vals)[:P], _u32(b['vals'])[:P])
        for k in ('image', 'depth', 'T_final'):
            torch.testing.assert_close(getattr(R, k), b[k], rtol=0, atol=0)
        np.testing.assert_array_equal(_u32(R.n_contrib), _u32(b['n_contrib']))
        R.backward(p, dIs[v], None, acc, accumulate=v > 0)
    torch.cuda.synchronize()
    for k in grads:
        torch.testing.assert_close(grads[k], acc[k], rtol=1e-5, atol=1e-9)


def test_batched_matches_oracle():
    d, cams = _small(2000, seed=4, deg=2)
    p = params_to_device(d)
    n = p['means'].shape[1]
    B = BatchedRasterizer(n, cams, d['sh_degree'])
    B.size_pairs(p)
    B.forward(p)
    rng = np.random.default_rng(5)
    dIs = [rng.standard_normal(b['image'].shape) * 1e-3 for b in B.buf]
    for b, dI in zip(B.buf, dIs):
        b['dL_dimage'].copy_(torch.as_tensor(dI.astype(np.float32)))
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    B.backward(p, grads)
    torch.cuda.synchronize()
    want = {k: 0.0 for k in p}
    excl = []
    for v, c in enumerate(cams):
        dv = dict(d, camera=c)
        pre = oracle_pre(dv)
        vals, ranges, _ = obin.sorted_pairs(pre, c)
        b = B.buf[v]
        np.testing.assert_array_equal(_u32(b['ranges']), ranges)
        np.testing.assert_array_equal(_u32(b['vals'])[:len(vals)], vals)
        out = oren.render(pre, c, vals, ranges)
        assert_image_close(b['image'].cpu().numpy(), out['image'], out['ambiguous'])
        dI = b['dL_dimage'].cpu().numpy().astype(np.float64)
        g2d, clamp = oren.render_backward(pre, c, vals, ranges, dI)
        g = obwd.preprocess_backward(pre, g2d, d['sh_degree'], c)
        for k in want:
            want[k] = want[k] + g[k]
        excl.append(exclusions(vals, ranges, c, out, clamp, n))
    ex = np.unique(np.concatenate(excl))
    for k in p:
        gg = grads[k].cpu().numpy()
        ww = want[k]
        gg = gg.reshape(-1, n)
        ww = np.asarray(ww).reshape(-1, n)
        for r in range(gg.shape[0]):
            assert_grads_close(gg[r], ww[r], ex, f'{k}[{r}]')


def test_grouped_adam_equals_per_group_adam():
    d, _ = _small(1001, seed=6)
    p1 = params_to_device(d)
    p2 = {k: v.clone() for k, v in p1.items()}
    rng = np.random.default_rng(7)
    m1 = {k: torch.zeros_like(v) for k, v in p1.items()}
    v1 = {k: torch.zeros_like(v) for k, v in p1.items()}
    m = {k: torch.zeros_like(v) for k, v in p2.items()}
    v2 = {k: torch.zeros_like(v) for k, v in p2.items()}
    step = torch.zeros(1, dtype=torch.int32, device='cuda')
    for it in range(3):
        g = {k: torch.as_tensor(rng.standard_normal(tuple(v.shape)).astype(np.float32),
                                device='cuda') for k, v in p1.items()}
        for k in p1:   # one launch per group, host-side bias corrections
            _lib.gs_adam_step(p1[k], g[k], m1[k], v1[k], p1[k].numel(), LRS[k], 0.9, 0.999,
                              1e-15, it + 1)
        _lib.gs_adam_step_grouped([(p2[k], g[k], m[k], v2[k], LRS[k]) for k in p2], 0.9, 0.999,
                                  1e-15, step)
    torch.cuda.synchronize()
    assert int(step.item()) == 3
    for k in p1:
        torch.testing.assert_close(p1[k], p2[k], rtol=2e-6, atol=1e-7)


def _train_setup(tile=16, n=4000, seed=8):
    d, cams = _small(n, seed=seed)
    p = params_to_device(d)
    B = BatchedRasterizer(p['means'].shape[1], cams, d['sh_degree'], tile=tile)
    B.size_pairs(p)
    targets = [torch.as_tensor(scenes.random_image((3, c.height, c.width), 100 + i), device='cuda')
               for i, c in enumerate(cams)]
    return TrainStep(B, p, targets, LRS)


def test_graph_replay_equals_eager_steps():
    st = _train_setup()
    st.run()                       # warm-up (first launches outside capture)
    torch.cuda.synchronize()
    state0 = {k: v.clone() for k, v in st.p.items()}
    m0 = {k: v.clone() for k, v in st.m.items()}
    v0 = {k: v.clone() for k, v in st.v.items()}
    s0 = st.step_count.clone()
    eager, losses = [], []
    for _ in range(3):
        st.run()
        torch.cuda.synchronize()
        eager.append({k: v.clone() for k, v in st.p.items()})
        losses.append(st.loss.item())

    def restore():
        for k in st.p:
            st.p[k].copy_(state0[k])
            st.m[k].copy_(m0[k])
            st.v[k].copy_(v0[k])
        st.step_count.copy_(s0)
        torch.cuda.synchronize()

    restore()
    st.capture()
    restore()
    for i in range(3):
        st.replay()
        torch.cuda.synchronize()
        # the program's own eager work between replays
        _ = (st.p['means'] * 2).sum().item()
        assert abs(st.loss.item() - losses[i]) <= 1e-5 * abs(losses[i])
        for k in st.p:
            torch.testing.assert_close(st.p[k], eager[i][k], rtol=1e-5, atol=1e-7)
    assert int(st.step_count.item()) == int(s0.item()) + 3
    st.check_capacity()


def test_autotuner_picks_a_valid_config_and_results_do_not_change():
    d, cams = _small(3000, seed=10)

    def make(tile):
        st = _train_setup(tile=tile, n=3000, seed=10)
        return st

    best, table = autotune(make, persist=(4, 16), warmup=1, iters=2)
    # the tuner starts from 12 persistent workgroups per CU and keeps it unless
    # a candidate is faster
    assert best['tile'] in (8, 16, 32) and best['persist_wgs'] in (4, 12, 16)
    assert len(table) >= 4 and all(ms > 0 for _, ms in table)
    # at the chosen configuration the tile lists are the oracle's
    p = params_to_device(d)
    B = BatchedRasterizer(p['means'].shape[1], cams, d['sh_degree'], tile=best['tile'])
    B.size_pairs(p)
    B.forward(p)
    torch.cuda.synchronize()
    for v, c in enumerate(cams):
        c.tile = best['tile']
        pre = oracle_pre(dict(d, camera=c))
        vals, ranges, _ = obin.sorted_pairs(pre, c)
        np.testing.assert_array_equal(_u32(B.buf[v]['ranges']), ranges)
        np.testing.assert_array_equal(_u32(B.buf[v]['vals'])[:len(vals)], vals)
    _lib.gs_set_tuning(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=0, bwd_batch=0)


@pytest.mark.parametrize('bwd_px', [4, 1])
def test_lds_batch_knobs_do_not_change_results(bwd_px):
    # the splats staged per LDS batch (forward batch 64 / 128 / 256, backward
    # bucket 32 / 64 / 128) change the launch, not the results: images, depth,
    # T_final and n_contrib bit for bit; gradients up to the order of the FP64
    # atomic adds across tiles
    d, cams = _small(3000, seed=12, deg=2)
    p = params_to_device(d)
    n = p['means'].shape[1]
    rng = np.random.default_rng(13)
    dIs = None
    res = {}
    for fb, bb in ((0, 0), (64, 32), (128, 64), (256, 128)):
        _lib.gs_set_tuning(fwd_px=1, bwd_px=bwd_px, persist_wgs=12, fwd_batch=fb, bwd_batch=bb)
        B = BatchedRasterizer(n, cams, d['sh_degree'], tile=16)
        B.size_pairs(p)
        B.forward(p)
        if dIs is None:
            dIs = [torch.as_tensor(rng.standard_normal(b['image'].shape).astype(np.float32) * 1e-3,
                                   device='cuda') for b in B.buf]
        for b, dI in zip(B.buf, dIs):
            b['dL_dimage'].copy_(dI)
        grads = {k: torch.empty_like(v) for k, v in p.items()}
        B.backward(p, grads)
        torch.cuda.synchronize()
        res[(fb, bb)] = ([{k: b[k].clone() for k in ('image', 'depth', 'T_final', 'n_contrib')}
                          for b in B.buf], grads)
    _lib.gs_set_tuning(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=0, bwd_batch=0)
    base_img, base_g = res[(0, 0)]
    for key, (img, g) in res.items():
        for a, b in zip(img, base_img):
            for k in a:
                assert torch.equal(a[k], b[k]), (key, k)
        for k in g:
            torch.testing.assert_close(g[k], base_g[k], rtol=1e-9, atol=1e-12, msg=str(key))


def test_tuning_knobs_are_checked():
    with pytest.raises(RuntimeError):
        _lib.gs_set_tuning(fwd_batch=96)
    with pytest.raises(RuntimeError):
        _lib.gs_set_tuning(bwd_batch=256)
    assert _lib.gs_get_tuning()['fwd_batch'] == 0


@pytest.mark.parametrize('tile,fb', [(8, 0), (16, 64), (16, 0), (32, 128)])
def test_deferred_batched_equals_full_lists(tile, fb):
    # the deferred binning over the views (each with its own workspace) and
    # the persistent forward that writes the lists: images, depth, T_final
    # and n_contrib bit for bit, the list positions below each tile's largest
    # n_contrib equal, the gradients up to the order of the FP64 atomic adds
    d, cams = _small(6000, seed=14, deg=1)
    p = params_to_device(d)
    n = p['means'].shape[1]
    rng = np.random.default_rng(15)
    res = {}
    _lib.gs_set_tuning(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=fb, bwd_batch=0)
    try:
        for deferred in (False, True):
            B = BatchedRasterizer(n, cams, d['sh_degree'], tile=tile, deferred=deferred)
            B.size_pairs(p)
            for b in B.buf:
                b['vals'].fill_(-1)
            B.forward(p)
            if not res:
                dIs = [torch.as_tensor(rng.standard_normal(b['image'].shape).astype(np.float32)
                                       * 1e-3, device='cuda') for b in B.buf]
            for b, dI in zip(B.buf, dIs):
                b['dL_dimage'].copy_(dI)
            grads = {k: torch.empty_like(v) for k, v in p.items()}
            B.backward(p, grads)
            torch.cuda.synchronize()
            res[deferred] = ([{k: b[k].clone() for k in ('image', 'depth', 'T_final', 'n_contrib',
                                                         'ranges', 'vals')} for b in B.buf],
                             grads, B.pair_counts())
    finally:
        _lib.gs_set_tuning(fwd_px=1, bwd_px=4, persist_wgs=12, fwd_batch=0, bwd_batch=0)
    (fa, ga, pa), (fd, gd, pd) = res[False], res[True]
    assert pa == pd
    for c, a, b in zip(cams, fa, fd):
        for k in ('image', 'depth', 'T_final', 'n_contrib', 'ranges'):
            assert torch.equal(a[k].view(torch.int32), b[k].view(torch.int32)), k
        nc = _u32(b['n_contrib'])
        T = tile
        H, W = nc.shape
        ty_n = -(-H // T)
        Y, X = np.mgrid[0:H, 0:W]
        m = np.zeros((-(-W // T)) * ty_n, np.int64)
        np.maximum.at(m, ((X // T) * ty_n + Y // T).ravel(), nc.ravel().astype(np.int64))
        r, va, vd = _u32(a['ranges']), _u32(a['vals']), _u32(b['vals'])
        for t in np.nonzero(m)[0]:
            s = int(r[t])
            np.testing.assert_array_equal(vd[s:s + m[t]], va[s:s + m[t]])
    for k in ga:
        x, y = ga[k].double().cpu().numpy(), gd[k].double().cpu().numpy()
        assert np.all(np.abs(x - y) <= 1e-5 * (np.abs(x) + np.abs(x).mean() + 1e-30)), k


def test_deferred_batched_graph_replay_equals_eager_steps():
    d, cams = _small(4000, seed=8)
    p = params_to_device(d)
    B = BatchedRasterizer(p['means'].shape[1], cams, d['sh_degree'], tile=16, deferred=True)
    B.size_pairs(p)
    targets = [torch.as_tensor(scenes.random_image((3, c.height, c.width), 100 + i), device='cuda')
               for i, c in enumerate(cams)]
    st = TrainStep(B, p, targets, LRS)
    st.run()
    torch.cuda.synchronize()
    state0 = {k: v.clone() for k, v in st.p.items()}
    m0 = {k: v.clone() for k, v in st.m.items()}
    v0 = {k: v.clone() for k, v in st.v.items()}
    s0 = st.step_count.clone()
    eager, losses = [], []
    for _ in range(3):
        st.run()
        torch.cuda.synchronize()
        eager.append({k: v.clone() for k, v in st.p.items()})
        losses.append(st.loss.item())

    def restore():
        for k in st.p:
            st.p[k].copy_(state0[k])
            st.m[k].copy_(m0[k])
            st.v[k].copy_(v0[k])
        st.step_count.copy_(s0)
        torch.cuda.synchronize()

    restore()
    st.capture()
    restore()
    for i in range(3):
        st.replay()
        torch.cuda.synchronize()
        _ = (st.p['means'] * 2).sum().item()
        assert abs(st.loss.item() - losses[i]) <= 1e-5 * abs(losses[i])
        for k in st.p:
            torch.testing.assert_close(st.p[k], eager[i][k], rtol=1e-5, atol=1e-7)
    st.check_capacity()
