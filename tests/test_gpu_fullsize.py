"""GPU parity at the benchmark's full size, in the launch configuration the
benchmark times (1,000,000 Gaussians, SH degree 3, 1600x1066, 16x16 tiles,
default tuning): every Gaussian's record and tile count, the pair total,
and for sampled tiles the exact sorted list, keys, image and the gradients
of a loss whose image gradient lives only on those tiles (the backward is
linear in dL/dimage, so the oracle needs only those tiles)."""
import numpy as np
import pytest
import torch

from oracle import backward as obwd
from oracle import binning as obin
from oracle import render as oren
from paper_2601_19489_amd import scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from _parity import (assert_grads_close, assert_image_close, assert_preprocess_close,
                     exclusions, gpu_splat_fields, oracle_pre)

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope='module')
def full():
    d = scenes.surface_cloud(1_000_000, seed=2, sh_degree=3, width=1600, height=1066)
    cam = d['camera']
    p = params_to_device(d)
    R = Rasterizer(1_000_000, cam, 3)
    R.preprocess(p)
    P = R.bin_sort()
    keys = torch.empty(R.capacity, dtype=torch.int64, device='cuda')
    R.bin_sort(keys_out=keys)
    R.render_fwd()
    # sampled tiles: dense centre, ragged last row, left edge, corner
    tiles = [(50, 33), (49, 34), (60, 28), (50, cam.tiles_y - 1), (0, 30), (cam.tiles_x - 1, 0)]
    rng = np.random.default_rng(77)
    dI = np.zeros((3, cam.height, cam.width), np.float32)
    for tx, ty in tiles:
        ys = slice(ty * 16, min(ty * 16 + 16, cam.height))
        xs = slice(tx * 16, tx * 16 + 16)
        dI[:, ys, xs] = rng.standard_normal(dI[:, ys, xs].shape).astype(np.float32) * 1e-3
    grads = R.backward(p, torch.as_tensor(dI, device='cuda'))
    torch.cuda.synchronize()
    pre = oracle_pre(d)
    return dict(d=d, cam=cam, R=R, P=P, keys=keys.cpu().numpy().view(np.uint64), tiles=tiles,
                dI=dI, grads={k: v.cpu().numpy() for k, v in grads.items()},
                grad2d=R.grad2d.cpu().numpy().T, pre=pre)


def test_records_counts_and_pair_total(full):
    R, pre, cam = full['R'], full['pre'], full['cam']
    assert_preprocess_close(gpu_splat_fields(R.splats.cpu().numpy()), pre)
    counts = obin.tile_counts(pre, cam)
    np.testing.assert_array_equal(_u32(R.tile_counts), counts)
    assert full['P'] == int(counts.sum())
    ranges = _u32(R.ranges).astype(np.int64)
    assert ranges[0] == 0 and ranges[-1] == full['P'] and np.all(np.diff(ranges) >= 0)


def test_sampled_tile_lists_keys_and_image(full):
    R, pre, cam = full['R'], full['pre'], full['cam']
    ranges = _u32(R.ranges).astype(np.int64)
    vals = _u32(R.vals)
    zb = pre['depth'].astype(np.float32).view(np.uint32).astype(np.uint64)
    lists = {}
    for tx, ty in full['tiles']:
        tid = obin.tile_id(cam, tx, ty)
        mem = obin.tile_members(pre, cam, tx, ty)
        lists[(tx, ty)] = mem
        np.testing.assert_array_equal(vals[ranges[tid]:ranges[tid + 1]], mem)
        want_keys = (np.uint64(tid) << np.uint64(32)) | zb[mem]
        np.testing.assert_array_equal(full['keys'][ranges[tid]:ranges[tid + 1]], want_keys)
    vals_o, ranges_o = _local_lists(cam, lists)
    out = oren.render(pre, cam, vals_o, ranges_o, tiles=full['tiles'])
    done = out['done']
    flags = out['ambiguous']
    assert_image_close(R.image.cpu().numpy(), out['image'], flags, done=done)
    assert_image_close(R.T_final.cpu().numpy(), out['T_final'], flags, done=done)
    assert_image_close(R.depth.cpu().numpy(), out['depth'], flags, done=done, tol=5e-4)
    nc = _u32(R.n_contrib)
    ok = done & ~flags
    np.testing.assert_array_equal(nc[ok], out['n_contrib'][ok])
    full['lists'] = (vals_o, ranges_o, out)


def _local_lists(cam, lists):
    n_tiles = cam.tiles_x * cam.tiles_y
    ranges = np.zeros(n_tiles + 1, np.int64)
    chunks = []
    for tid in range(n_tiles):
        tx, ty = divmod(tid, cam.tiles_y)
        m = lists.get((tx, ty))
        if m is not None:
            chunks.append(m)
        ranges[tid + 1] = ranges[tid] + (0 if m is None else len(m))
    return np.concatenate(chunks), ranges


def test_gradients_of_sampled_tiles(full):
    if 'lists' not in full:
        pytest.skip('needs the sampled-tile lists of the previous test')
    pre, cam = full['pre'], full['cam']
    vals_o, ranges_o, out = full['lists']
    g2d, clamp = oren.render_backward(pre, cam, vals_o, ranges_o, full['dI'], tiles=full['tiles'])
    grads = obwd.preprocess_backward(pre, g2d, 3, cam)
    ex = exclusions(vals_o, ranges_o, cam, out, clamp, 1_000_000)
    touched_mask = np.any(g2d != 0, axis=0)
    touched = np.nonzero(touched_mask)[0]
    assert len(touched) > 100 and len(ex) < 0.15 * len(touched) + 10
    # Gaussians outside the sampled tiles get exactly zero on the GPU too
    untouched = ~touched_mask
    untouched[ex] = False
    assert np.all(full['grad2d'][:, untouched] == 0)
    # the relative bar is applied over the Gaussians the sampled tiles touch
    ex = np.union1d(ex, np.nonzero(~touched_mask)[0])
    names = ('u', 'v', 'a', 'b', 'c', 'opacity', 'r', 'g', 'b_col', 'depth')
    for k, nm in enumerate(names):
        assert_grads_close(full['grad2d'][k], g2d[k], ex, 'grad2d.' + nm)
    for nm in ('means', 'log_scales', 'quats', 'opacity_logits', 'sh'):
        gg = full['grads'][nm].reshape(-1, 1_000_000)
        oo = grads[nm].reshape(-1, 1_000_000)
        for r in range(gg.shape[0]):
            assert_grads_close(gg[r], oo[r], ex, f'{nm}[{r}]')
