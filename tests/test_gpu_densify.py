"""GPU parity of the depth loss (Sec. 3.1) and the densification pieces
(Sec. 3.2, Eq. 3-4) against the oracle, through the C ABI.

Bars: the Eq. 3 mask bit-exact (both sides decide in FP32 in the same
order, on the same seeded images); split-score counts bit-exact except at
Gaussians a masked knife-edge pixel can flip (those within the oracle's
count of such pixels); clone / split layout and copies bit-exact, split
children within 1 FP32 ulp of the oracle's FP64 placement.
"""
import math

import numpy as np
import pytest
import torch

from oracle import densify as oden
from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from oracle import binning as obin

from _parity import oracle_pre

pytestmark = pytest.mark.gpu


def test_depth_l1_matches_oracle():
    rng = np.random.default_rng(1)
    D = rng.uniform(1, 5, (37, 53)).astype(np.float32)
    Dt = (D * (1 + 0.01 * rng.standard_normal(D.shape))).astype(np.float32)
    Dt[0, :5] = D[0, :5]   # zero differences: sign 0
    d, t = torch.as_tensor(D, device='cuda'), torch.as_tensor(Dt, device='cuda')
    g = torch.empty_like(d)
    loss = torch.zeros(1, device='cuda')
    _lib.gs_depth_l1_loss(d, t, D.size, 0.1, g, loss)
    torch.cuda.synchronize()
    wl, wg = oden.depth_l1(D, Dt, 0.1)
    np.testing.assert_allclose(g.cpu().numpy(), wg, rtol=1e-6, atol=0)
    assert abs(loss.item() - wl) <= 1e-6 * wl


@pytest.mark.parametrize('H,W,seed', [(1, 1, 0), (67, 129, 1), (1066, 1600, 2)])
def test_error_mask_bit_exact(H, W, seed):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    tgt = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    mask = torch.empty((H, W), dtype=torch.uint8, device='cuda')
    mm = torch.empty(2, dtype=torch.int32, device='cuda')
    _lib.gs_error_mask(torch.as_tensor(img, device='cuda'), torch.as_tensor(tgt, device='cuda'),
                       H * W, 0.1, mask, mm)
    torch.cuda.synchronize()
    want = oden.error_mask(img, tgt, 0.1)
    np.testing.assert_array_equal(mask.cpu().numpy().astype(bool), want)


def _score_case(d, mask_np, tile=16):
    cam = d['camera']
    p = params_to_device(d)
    n = p['means'].shape[1]
    R = Rasterizer(n, cam, d['sh_degree'], tile=tile)
    R.forward(p)
    score = torch.zeros(n, dtype=torch.int32, device='cuda')
    mask = torch.as_tensor(mask_np.astype(np.uint8), device='cuda')
    _lib.gs_split_score(R.splats, n, R.vals, R.ranges, R.cam, mask, score)
    _lib.gs_split_score(R.splats, n, R.vals, R.ranges, R.cam, mask, score)  # adds: two views
    torch.cuda.synchronize()
    got = score.cpu().numpy().view(np.uint32).astype(np.int64)
    pre = oracle_pre(d)
    vals, ranges, _ = obin.sorted_pairs(pre, cam)
    want, unc = oden.split_score(pre, cam, vals, ranges, mask_np)
    return got, 2 * want, 2 * unc


@pytest.mark.parametrize('tile', [8, 16, 32])
def test_split_score_matches_oracle(tile):
    d = scenes.surface_cloud(6000, seed=5, sh_degree=1, width=200, height=136)
    d['camera'].tile = tile
    rng = np.random.default_rng(6)
    mask = rng.uniform(size=(136, 200)) < 0.3
    mask[40:80, 50:120] = True
    got, want, unc = _score_case(d, mask, tile)
    sure = unc == 0
    np.testing.assert_array_equal(got[sure], want[sure])
    assert np.all(np.abs(got[~sure] - want[~sure]) <= unc[~sure])
    assert want.sum() > 10000 and (~sure).sum() < 0.02 * len(want) + 5


def test_split_score_empty_mask_and_ragged_tiles():
    d = scenes.random_cloud(500, seed=7, width=37, height=29)
    got, want, _ = _score_case(d, np.zeros((29, 37), bool))
    assert got.sum() == 0 and want.sum() == 0
    m = np.zeros((29, 37), bool)
    m[-1, :] = True     # last (partial) tile row only
    m[:, -1] = True     # last (partial) tile column only
    got, want, unc = _score_case(d, m)
    np.testing.assert_array_equal(got[unc == 0], want[unc == 0])


def _densify_gpu(d, score, thr, split_scale, eps, prune=None, prune_thr=0.0):
    p = params_to_device(d)
    n = p['means'].shape[1]
    sc = torch.as_tensor(score.astype(np.uint32).view(np.int32), device='cuda')
    ws = torch.empty(_lib.gs_densify_workspace(n), dtype=torch.uint8, device='cuda')
    n_out_d = torch.zeros(1, dtype=torch.int32, device='cuda')
    if prune is None:
        _lib.gs_densify_plan(sc, p['log_scales'], n, thr, split_scale, ws, n_out_d)
    else:
        ps = torch.as_tensor(np.asarray(prune, np.float64), device='cuda')
        _lib.gs_densify_prune_plan(sc, p['log_scales'], n, thr, split_scale, ps, prune_thr, ws,
                                   n_out_d)
    n_out = int(n_out_d.item())
    K = p['sh'].shape[0]
    out = dict(means=torch.empty((3, n_out), device='cuda'),
               log_scales=torch.empty((3, n_out), device='cuda'),
               quats=torch.empty((4, n_out), device='cuda'),
               opacity_logits=torch.empty(n_out, device='cuda'),
               sh=torch.empty((K, 3, n_out), device='cuda'))
    names = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')
    g = _lib.gaussians(*(p[k] for k in names))
    o = _lib.gaussians(*(out[k] for k in names))
    e = torch.as_tensor(eps, device='cuda').contiguous()
    _lib.gs_densify_apply(g, n, d['sh_degree'], e, ws, n_out, False, o)
    # moments mode on a stand-in moment array (the parameters themselves)
    mo = {k: torch.empty_like(v) for k, v in out.items()}
    _lib.gs_densify_apply(g, n, d['sh_degree'], None, ws, n_out, True,
                          _lib.gaussians(*(mo[k] for k in names)))
    torch.cuda.synchronize()
    return n_out, {k: v.cpu().numpy() for k, v in out.items()}, {k: v.cpu().numpy()
                                                                 for k, v in mo.items()}


@pytest.mark.parametrize('n,seed', [(1, 0), (5000, 1), (300_001, 2)])
def test_densify_matches_oracle(n, seed):
    d = scenes.surface_cloud(n, seed=seed, sh_degree=2, width=64, height=64)
    rng = np.random.default_rng(seed + 50)
    score = rng.integers(0, 12, n)
    eps = rng.standard_normal((2, 3, n)).astype(np.float32)
    split_scale = float(np.float32(0.05))
    n_out, got, mom = _densify_gpu(d, score, 6, split_scale, eps)
    params = {k: d[k] for k in ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')}
    want, counts = oden.densify(params, 2, score, 6, split_scale, eps)
    assert n_out == int(counts.sum())
    for k in ('quats', 'opacity_logits', 'sh'):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    for k in ('means', 'log_scales'):
        gu = got[k].view(np.int32).astype(np.int64)
        wu = np.asarray(want[k], np.float32).view(np.int32).astype(np.int64)
        assert np.abs(gu - wu).max() <= 1, k
    # moments: copies of originals, zero for new entries
    src = np.repeat(np.arange(n), counts)
    first = np.r_[True, src[1:] != src[:-1]]
    sel = score >= 6
    big = np.exp(d['log_scales'].astype(np.float64)).max(axis=0) > split_scale
    new = ~first | (sel & big)[src]
    for k in ('means', 'log_scales', 'quats', 'opacity_logits', 'sh'):
        m = mom[k]
        assert np.all(m[..., new] == 0), k
        np.testing.assert_array_equal(m[..., ~new], np.asarray(d[k])[..., src[~new]])


def _threshold_gpu(score_np, t_min, cap):
    score = torch.as_tensor(score_np.astype(np.uint32).view(np.int32), device='cuda')
    scratch = torch.empty(_lib.SCORE_BINS, dtype=torch.int32, device='cuda')
    out = torch.zeros(1, dtype=torch.int32, device='cuda')
    _lib.gs_densify_threshold(score, len(score_np), t_min, cap, scratch, out)
    torch.cuda.synchronize()
    return int(out.item()) & 0xFFFFFFFF


@pytest.mark.parametrize('n', [0, 1, 1000, 65536 + 3, 1_000_003])
def test_growth_threshold_bit_exact(n):
    rng = np.random.default_rng(n + 5)
    # mostly small counts, a heavy tail and some above the histogram's range
    sc = rng.geometric(0.05, n) - 1
    sc[rng.random(n) < 0.3] = 0
    tail = rng.random(n) < 0.002
    sc[tail] = rng.integers(1000, 100_000, int(tail.sum()))
    for t_min, cap in ((1, n // 10), (20, n // 3), (1, 0), (5, n), (1, int(tail.sum()) // 2),
                       (65535, 1), (100, 7)):
        want = oden.growth_threshold(sc, t_min, cap)
        assert _threshold_gpu(sc, t_min, cap) == want, (t_min, cap, want)


def test_growth_threshold_all_at_the_top():
    sc = np.full(5000, 70_000, np.int64)
    assert _threshold_gpu(sc, 1, 4999) == oden.NO_THRESHOLD == oden.growth_threshold(sc, 1, 4999)
    assert _threshold_gpu(sc, 1, 5000) == 1 == oden.growth_threshold(sc, 1, 5000)
