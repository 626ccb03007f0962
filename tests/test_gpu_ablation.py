"""Binning ablation pieces (Sec. 2.1: compact tiles and load-balanced writing
against loose boxes and per-Gaussian sequential writing): the tile counts of
the three tile-set variants bit-exact against the oracle, and the sequential
walk producing exactly the load-balanced walk's tile counts, lists and
ranges."""
import numpy as np
import pytest
import torch

from oracle import binning as obin
from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from _parity import oracle_pre

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize('n,w,h,tile', [(6000, 200, 136, 8), (6000, 200, 136, 16),
                                        (6000, 200, 136, 32), (300_000, 1600, 1066, 16)])
def test_tile_count_variants_bit_exact(n, w, h, tile):
    d = scenes.surface_cloud(n, seed=21, width=w, height=h)
    c = d['camera']
    c.tile = tile
    p = params_to_device(d)
    R = Rasterizer(n, c, d['sh_degree'], tile=tile)
    R.preprocess(p)
    counts = torch.empty(n, dtype=torch.int32, device='cuda')
    got = {}
    for v in (_lib.TILES_COMPACT, _lib.TILES_SNUGBOX, _lib.TILES_3SIGMA):
        _lib.gs_tile_count_variant(R.splats, n, R.cam, v, counts)
        got[v] = _u32(counts).astype(np.int64)
    pre = oracle_pre(d)
    np.testing.assert_array_equal(got[_lib.TILES_COMPACT], _u32(R.tile_counts))
    np.testing.assert_array_equal(got[_lib.TILES_SNUGBOX], obin.snugbox_counts(pre, c))
    np.testing.assert_array_equal(got[_lib.TILES_3SIGMA], obin.sigma3_counts(pre, c))
    if n == 6000:
        np.testing.assert_array_equal(got[_lib.TILES_COMPACT], obin.tile_counts(pre, c))
    print({v: int(x.sum()) for v, x in got.items()})


def test_sequential_walk_gives_identical_lists():
    d = scenes.surface_cloud(50_000, seed=22, width=640, height=480)
    p = params_to_device(d)
    n = p['means'].shape[1]
    res = []
    try:
        for seq in (0, 1):
            _lib.gs_set_tuning(seq_walk=seq)
            R = Rasterizer(n, d['camera'], d['sh_degree'])
            R.forward(p)
            torch.cuda.synchronize()
            P = int(R.pair_count.item())
            res.append((_u32(R.tile_counts), _u32(R.ranges), _u32(R.vals)[:P],
                        R.image.cpu().numpy()))
    finally:
        _lib.gs_set_tuning(seq_walk=0)
    for a, b in zip(*res):
        np.testing.assert_array_equal(a, b)
