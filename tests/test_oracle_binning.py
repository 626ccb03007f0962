"""Pins of the oracle's tile-set variants for the binning ablation (Sec. 2.1
contrasts the compact tile set with loose boxes): SnugBox and 3-sigma box
counts against a brute-force interval-overlap count over every tile, the
inclusion compact <= SnugBox, the isotropic closed form of the 3-sigma radius,
and the 3-sigma box's indifference to opacity."""
import math

import numpy as np

from oracle import binning, preprocess
from paper_2601_19489_amd import scenes



def _brute_box(u, v, hx, hy, cam):
    # tiles whose closed cell [T tx, T tx + T] x [T ty, T ty + T] meets the box,
    # by interval overlap over every tile of the grid
    n = 0
    T = cam.tile
    for tx in range(cam.tiles_x):
        if T * tx > u + hx or T * tx + T < u - hx:
            continue
        for ty in range(cam.tiles_y):
            if T * ty <= v + hy and T * ty + T >= v - hy:
                n += 1
    return n


def test_box_variant_counts_brute_force_and_inclusion():
    d = scenes.surface_cloud(400, seed=12, width=96, height=72)
    pre = preprocess.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'],
                                d['sh'], d['sh_degree'], d['camera'])
    cam = d['camera']
    compact = binning.tile_counts(pre, cam).astype(np.int64)
    snug = binning.snugbox_counts(pre, cam)
    s3 = binning.sigma3_counts(pre, cam)
    assert np.all(snug >= compact)          # the ellipse lies inside its box
    assert snug.sum() > compact.sum()
    _, hx, hy = binning.half_extents(pre['a'], pre['b'], pre['c'], pre['t'])
    ok = binning.has_tiles(pre['visible'], pre['a'], pre['b'], pre['c'], pre['t'])
    for i in range(0, 400, 7):
        want = _brute_box(float(pre['u'][i]), float(pre['v'][i]), hx[i], hy[i], cam) if ok[i] else 0
        assert snug[i] == want, i
    # 3-sigma: an isotropic splat (Sigma' = s2 I) has lambda = s2 + sqrt(0.1)
    s2 = 6.25
    sp = dict(u=np.array([40.3]), v=np.array([31.7]), a=np.array([1 / s2]), b=np.array([0.0]),
              c=np.array([1 / s2]), t=np.array([3.0]), visible=np.array([True]))
    r = math.ceil(3 * math.sqrt(s2 + math.sqrt(0.1)))
    assert binning.sigma3_counts(sp, cam)[0] == _brute_box(40.3, 31.7, r, r, cam)
    # it ignores the opacity: t <= 0 still bins under 3 sigma, never under the others
    sp['t'] = np.array([-1.0])
    assert binning.sigma3_counts(sp, cam)[0] > 0 and binning.snugbox_counts(sp, cam)[0] == 0
