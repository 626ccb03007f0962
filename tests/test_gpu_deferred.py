"""The deferred binning (gs_bin_sort_deferred + gs_render_fwd_deferred: the
forward takes each tile's depth-sorted list of Sec. 2.1 from the binning's
column runs and writes it only as far as its compositing reaches) against
the full binning and forward: the same tile ranges and pair count, images,
depth, final transmittance and n_contrib bit for bit, the list positions the
backward reads equal to the full lists, and the backward on them equal to
the backward on the full lists up to the order of its FP64 atomic sums. Tile sizes 8, 16 and 32, one, two and four
pixels per thread, an empty scene, a capacity overflow and a grid of 2000
columns."""
import numpy as np
import pytest
import torch

from paper_2601_19489_amd import _lib, scenes
from paper_2601_19489_amd.rasterizer import Rasterizer, params_to_device

from test_gpu_parity import _wide_scene

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _with_tile(cam, tile):
    return scenes.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.R, cam.t,
                         cam.near, tile)


def _run(d, deferred, tile, capacity=0, dI=None):
    cam = _with_tile(d['camera'], tile)
    p = params_to_device(d)
    n = p['means'].shape[1]
    R = Rasterizer(n, cam, d['sh_degree'], tile=tile, capacity=capacity, deferred=deferred)
    R.preprocess(p)
    P = R.bin_sort(check_overflow=capacity == 0)
    if deferred:  # stale values everywhere the forward does not write
        R.vals.fill_(-1)
    R.render_fwd()
    out = dict(R=R, P=P, image=R.image.clone(), depth=R.depth.clone(), T=R.T_final.clone(),
               nc=_u32(R.n_contrib), ranges=_u32(R.ranges), vals=_u32(R.vals),
               pc=int(R.pair_count.item()) & 0xFFFFFFFF)
    if dI is not None:
        grads = R.backward(p, dI)
        torch.cuda.synchronize()
        out['grad2d'] = R.grad2d.clone()
        out['grads'] = {k: v.clone() for k, v in grads.items()}
    return out


def _tile_max_contrib(nc, tiles_x, tiles_y, tile):
    H, W = nc.shape
    Y, X = np.mgrid[0:H, 0:W]
    tid = (X // tile) * tiles_y + (Y // tile)
    m = np.zeros(tiles_x * tiles_y, np.int64)
    np.maximum.at(m, tid.ravel(), nc.ravel().astype(np.int64))
    return m


def _same(a, b):
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def _compare(d, tile, px=1, with_bwd=True):
    saved = _lib.gs_get_tuning()
    _lib.gs_set_tuning(fwd_px=px)
    try:
        cam = d['camera']
        dI = None
        if with_bwd:
            g = torch.Generator().manual_seed(5)
            dI = (torch.randn((3, cam.height, cam.width), generator=g) * 1e-3).cuda()
        a = _run(d, False, tile, dI=dI)
        b = _run(d, True, tile, dI=dI)
    finally:
        _lib.gs_set_tuning(**saved)
    assert a['P'] == b['P'] and a['pc'] == b['pc']
    np.testing.assert_array_equal(a['ranges'], b['ranges'])
    assert _same(a['image'], b['image']) and _same(a['depth'], b['depth'])
    assert _same(a['T'], b['T'])
    np.testing.assert_array_equal(a['nc'], b['nc'])
    R = b['R']
    m = _tile_max_contrib(b['nc'], R.tiles_x, R.tiles_y, tile)
    ranges = a['ranges']
    for k in np.nonzero(m)[0]:
        s = int(ranges[k])
        np.testing.assert_array_equal(b['vals'][s:s + m[k]], a['vals'][s:s + m[k]], err_msg=k)
    if with_bwd:
        # the same terms, summed across tiles by FP64 atomics in whatever
        # order the tiles finish: equal up to that order
        _close(a['grad2d'], b['grad2d'], 1e-12)
        for k in a['grads']:
            _close(a['grads'][k], b['grads'][k], 1e-5, k)
    return a, b


def _close(x, y, tol, name=''):
    x, y = x.double().cpu().numpy(), y.double().cpu().numpy()
    scale = np.abs(x).mean() + 1e-300
    assert np.all(np.abs(x - y) <= tol * (np.abs(x) + scale)), name


@pytest.mark.parametrize('tile,px', [(8, 1), (16, 1), (16, 2), (16, 4), (32, 2), (32, 4)])
def test_deferred_matches_full_lists(tile, px):
    d = scenes.surface_cloud(20000, seed=2, sh_degree=3, width=320, height=240)
    _compare(d, tile, px)


def test_deferred_writes_what_is_composited():
    # deep lists: the tiles saturate long before their ends, and the
    # deferred forward leaves most of the lists unwritten
    d = scenes.surface_cloud(300000, seed=2, sh_degree=1, width=320, height=240)
    a, b = _compare(d, 16, with_bwd=False)
    unwritten = int(np.sum(b['vals'][:a['P']] == 0xFFFFFFFF))
    assert unwritten > a['P'] // 2, (unwritten, a['P'])


def test_deferred_empty_and_culled():
    d = scenes.random_cloud(50, seed=0, width=64, height=64)
    d['means'][2] = -10.0  # all behind the camera: every list is empty
    a, b = _compare(d, 16)
    assert a['P'] == 0


def test_deferred_capacity_overflow_then_rerun():
    d = scenes.surface_cloud(3000, seed=3, sh_degree=1, width=160, height=120)
    full = _run(d, False, 16)
    P = full['P']
    o = _run(d, True, 16, capacity=max(P // 3, 1))  # overflow: every tile empty, no fault
    assert o['pc'] == P
    torch.cuda.synchronize()
    c = _run(d, True, 16, capacity=P)  # exactly enough
    assert _same(c['image'], full['image'])
    np.testing.assert_array_equal(c['nc'], full['nc'])


def test_deferred_wide_grid():
    d = _wide_scene(1500, seed=12, width=16000, height=96, tile=8)
    d['opacity_logits'] -= np.float32(1.5)
    assert d['camera'].tiles_x == 2000
    _compare(d, 8, with_bwd=False)


def test_split_score_on_deferred_lists():
    # the Eq. (4) replay reads the lists in the forward's batches and stops
    # where the forward stopped: the same counts on the deferred lists
    d = scenes.surface_cloud(40000, seed=6, sh_degree=1, width=320, height=240)
    target = torch.as_tensor(d['target'], device='cuda')
    counts = []
    for deferred in (False, True):
        r = _run(d, deferred, 16)
        R = r['R']
        H, W = R.image.shape[1:]
        mask = torch.empty((H, W), dtype=torch.uint8, device='cuda')
        mm = torch.empty(2, dtype=torch.int32, device='cuda')
        score = torch.zeros(R.n, dtype=torch.int32, device='cuda')
        _lib.gs_error_mask(R.image, target, H * W, 0.1, mask, mm)
        _lib.gs_split_score(R.splats, R.n, R.vals, R.ranges, R.cam, mask, score)
        torch.cuda.synchronize()
        counts.append(score.cpu().numpy())
    assert counts[0].sum() > 0
    np.testing.assert_array_equal(counts[0], counts[1])
