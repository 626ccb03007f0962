"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: tile counts, tile lists, sort order and keys bit-exact; preprocess
records within 2 ulp of the oracle's FP32 rounding; images within 1e-4
max-abs outside knife-edge pixels; gradients within 1e-3 relative.
"""
import numpy as np
import pytest
import torch

from paper_2601_19489_amd import scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from _parity import (assert_grads_close, assert_image_close, assert_preprocess_close, exclusions,
                     gpu_splat_fields, oracle_pipeline)

pytestmark = pytest.mark.gpu

PNAMES = ('means', 'log_scales', 'quats', 'opacity_logits', 'sh')


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _gpu_run(d, tile=16, bg=(0.0, 0.0, 0.0), dL_dimage=None, dL_ddepth=None):
    cam = d['camera']
    p = params_to_device(d)
    n = p['means'].shape[1]
    R = Rasterizer(n, cam, d['sh_degree'], bg=bg, tile=tile)
    R.preprocess(p)
    P = R.bin_sort()
    keys = torch.empty(R.capacity, dtype=torch.int64, device='cuda')
    R.bin_sort(keys_out=keys)
    R.render_fwd()
    res = dict(R=R, P=P, splats=R.splats.cpu().numpy(), depth_keys=_u32(R.depth_keys),
               counts=_u32(R.tile_counts), vals=_u32(R.vals)[:P], ranges=_u32(R.ranges),
               keys=keys.cpu().numpy().view(np.uint64)[:P], image=R.image.cpu().numpy(),
               depth=R.depth.cpu().numpy(), T_final=R.T_final.cpu().numpy(),
               n_contrib=_u32(R.n_contrib))
    if dL_dimage is not None:
        dI = torch.as_tensor(dL_dimage, dtype=torch.float32, device='cuda').contiguous()
        dD = None if dL_ddepth is None else torch.as_tensor(
            dL_ddepth, dtype=torch.float32, device='cuda').contiguous()
        grads = R.backward(p, dI, dD)
        torch.cuda.synchronize()
        res['grads'] = {k: v.cpu().numpy() for k, v in grads.items()}
        res['grad2d'] = R.grad2d.cpu().numpy().T  # [n][10] records -> [10][n]
    return res


def _with_tile(d, tile):
    d = dict(d)
    c = d['camera']
    d['camera'] = scenes.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.R, c.t, c.near, tile)
    return d


def _check_forward(d, g, o):
    cam = d['camera']
    pre = o['pre']
    assert_preprocess_close(gpu_splat_fields(g['splats']), pre)
    # integer work: bit-exact
    np.testing.assert_array_equal(g['counts'], o['counts'])
    zk = np.where(o['counts'] > 0, pre['depth'].astype(np.float32).view(np.uint32), 0xFFFFFFFF)
    np.testing.assert_array_equal(g['depth_keys'], zk)
    assert g['P'] == len(o['vals'])
    np.testing.assert_array_equal(g['vals'], o['vals'])
    np.testing.assert_array_equal(g['ranges'], o['ranges'])
    np.testing.assert_array_equal(g['keys'], o['keys'])
    out = o['out']
    flags = out['ambiguous']
    assert flags.mean() < 1e-2, flags.sum()  # knife-edge stop tests: expected ~0.1%
    assert_image_close(g['image'], out['image'], flags)
    assert_image_close(g['depth'], out['depth'], flags, tol=5e-4)
    assert_image_close(g['T_final'], out['T_final'], flags)
    ok = ~flags
    np.testing.assert_array_equal(g['n_contrib'][ok], out['n_contrib'][ok])


def _check_backward(d, g, o, max_excluded=0.02):
    ex = exclusions(o['vals'], o['ranges'], d['camera'], o['out'], o['clamp'],
                    d['means'].shape[1])
    # keep the check meaningful (about 1% at most on these scenes)
    assert len(ex) < max_excluded * d['means'].shape[1] + 10, len(ex)
    names = ('u', 'v', 'a', 'b', 'c', 'opacity', 'r', 'g', 'b_col', 'depth')
    for k, nm in enumerate(names):
        assert_grads_close(g['grad2d'][k], o['grad2d'][k], ex, 'grad2d.' + nm)
    for nm in PNAMES:
        gg = g['grads'][nm].reshape(-1, g['grads'][nm].shape[-1])
        oo = o['grads'][nm].reshape(-1, o['grads'][nm].shape[-1])
        for r in range(gg.shape[0]):
            assert_grads_close(gg[r], oo[r], ex, f'{nm}[{r}]')
    return ex


def _random_upstream(cam, seed, depth=True):
    rng = np.random.default_rng(seed)
    dI = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32) * 1e-3
    dD = (rng.standard_normal((cam.height, cam.width)).astype(np.float32) * 1e-4) if depth else None
    return dI, dD


def test_tiny_cloud_64px_forward_backward():
    d = scenes.random_cloud(1000, seed=0)
    dI, dD = _random_upstream(d['camera'], 1)
    g = _gpu_run(d, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD)
    _check_forward(d, g, o)
    _check_backward(d, g, o)


@pytest.mark.parametrize('tile', [8, 16, 32])
def test_surface_cloud_ragged_tiles_sh3(tile):
    # 200 x 136 px: a ragged last tile row/column at every tile size
    d = _with_tile(scenes.surface_cloud(6000, seed=21, width=200, height=136), tile)
    dI, dD = _random_upstream(d['camera'], 2)
    bg = (0.1, 0.3, 0.2)
    g = _gpu_run(d, tile=tile, bg=bg, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD, bg=bg)
    _check_forward(d, g, o)
    _check_backward(d, g, o)


def test_inverse_depth_mode_forward_backward():
    # the depth channel carries 1 / p_z (disparity supervision); keys stay p_z
    d = scenes.surface_cloud(4000, seed=23, sh_degree=2, width=160, height=120)
    d['camera'].depth_mode = 1
    dI, dD = _random_upstream(d['camera'], 5)
    dD = dD * 10.0
    g = _gpu_run(d, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD)
    _check_forward(d, g, o)
    _check_backward(d, g, o)
    assert float(np.max(g['depth'])) < 1.0 / 2.0   # inverse depths of a scene 3-5 units away


def test_empty_scene_and_culled_gaussians():
    d = scenes.random_cloud(300, seed=3)
    d['means'][2] = -5.0  # all behind the camera (p_z = -1)
    dI, _ = _random_upstream(d['camera'], 4, depth=False)
    g = _gpu_run(d, bg=(0.2, 0.4, 0.6), dL_dimage=dI)
    assert g['P'] == 0
    assert np.all(g['counts'] == 0) and np.all(g['depth_keys'] == 0xFFFFFFFF)
    assert np.all(g['ranges'] == 0)
    np.testing.assert_allclose(g['image'], np.broadcast_to(np.array([0.2, 0.4, 0.6])[:, None, None],
                                                           g['image'].shape), atol=0)
    assert np.all(g['T_final'] == 1) and np.all(g['n_contrib'] == 0)
    for v in g['grads'].values():
        assert np.all(v == 0)


def test_faint_and_huge_gaussians():
    d = scenes.random_cloud(400, seed=5, width=96, height=80)
    d['opacity_logits'][:50] = -7.0            # o < 1/255: no tiles
    d['log_scales'][:, 50:53] = 0.5            # covers the whole image
    d['opacity_logits'][50:53] = 4.0
    dI, dD = _random_upstream(d['camera'], 6)
    g = _gpu_run(d, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD)
    assert np.all(g['counts'][:50] == 0)
    assert np.all(g['counts'][50:53] == d['camera'].tiles_x * d['camera'].tiles_y)
    _check_forward(d, g, o)
    _check_backward(d, g, o)


def test_pair_capacity_overflow_is_reported_and_recovered():
    d = scenes.random_cloud(800, seed=7)
    p = params_to_device(d)
    R = Rasterizer(800, d['camera'], 0, capacity=16)
    R.preprocess(p)
    P = R.bin_sort(check_overflow=False)
    assert P is None
    assert int(R.pair_count.item()) > 16
    assert np.all(_u32(R.ranges) == 0)        # overflow: every tile empty, nothing written
    P = R.bin_sort()                          # re-runs with a large enough capacity
    assert R.capacity >= P > 16
    o = oracle_pipeline(d)
    np.testing.assert_array_equal(_u32(R.vals)[:P], o['vals'])


def test_many_pair_blocks_per_column():
    # ~30k pairs per tile column: every column is cut into many pair blocks,
    # and runs of large Gaussians straddle block boundaries
    d = scenes.surface_cloud(30000, seed=31, width=320, height=200, large_frac=0.2)
    dI, dD = _random_upstream(d['camera'], 9)
    g = _gpu_run(d, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD)
    assert g['P'] > 20 * 2048 * d['camera'].tiles_x // 4
    _check_forward(d, g, o)
    _check_backward(d, g, o)


def _wide_scene(n, seed, width, height, tile):
    """A thin horizontal band of Gaussians seen by a wide, short camera, so
    that the tile grid has many columns."""
    d = scenes.random_cloud(n, seed=seed, width=width, height=height)
    rng = np.random.default_rng(seed + 100)
    d['means'][0] = rng.uniform(-12.0, 12.0, n).astype(np.float32)
    d['means'][1] = rng.uniform(-0.06, 0.06, n).astype(np.float32)
    d['means'][2] = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    d['camera'] = scenes.Camera(width, height, 1800.0, 1800.0, width / 2.0, height / 2.0,
                                np.eye(3), np.array([0.0, 0.0, 4.0]), 0.2, tile)
    return d


def test_wide_grid_of_columns():
    # 2000 tile columns (the most the binning takes is 2048): every column's
    # runs are bucketed from the per-block counts, many blocks per column
    d = _wide_scene(1500, seed=12, width=16000, height=96, tile=8)
    d['opacity_logits'] -= np.float32(1.5)  # shallow stacks: few knife-edge pixels
    assert d['camera'].tiles_x == 2000
    dI, dD = _random_upstream(d['camera'], 13)
    g = _gpu_run(d, tile=8, dL_dimage=dI, dL_ddepth=dD)
    o = oracle_pipeline(d, dI, dD)
    assert g['P'] > 100000
    touched = np.diff(o['ranges']).reshape(2000, -1).sum(axis=1) > 0
    assert touched.sum() > 1500, touched.sum()
    _check_forward(d, g, o)
    _check_backward(d, g, o)


def test_grid_wider_than_2048_columns_is_rejected():
    d = _wide_scene(200, seed=14, width=2049 * 8, height=16, tile=8)
    p = params_to_device(d)
    R = Rasterizer(200, d['camera'], 0, tile=8)
    R.preprocess(p)
    with pytest.raises(RuntimeError):
        R.bin_sort()
