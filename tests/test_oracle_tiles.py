"""Pins of the oracle's compact tile sets (Sec. 2.1, Eq. 1-2) and sort:
SnugBox extents against the Eq. (2) worked examples and brute force, the
column walk against a brute-force closed-cell predicate and dense sampling,
the isotropic closed form, and the sorted pair list against Python's sort."""
import math
import os

import numpy as np
import pytest

from oracle import binning, preprocess, render
from paper_2601_19489_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), 'golden', 'eq2_snugbox.txt')


def _rows():
    return [list(map(float, l.split())) for l in open(GOLD) if l.strip() and not l.startswith('#')]


@pytest.mark.parametrize('row', _rows())
def test_snugbox_matches_eq2_worked_examples(row):
    a, b, c, t, hx, hy, xd, ymin = row
    _, ohx, ohy = binning.half_extents(a, b, c, t)
    assert abs(ohx - hx) <= 1e-13 * hx and abs(ohy - hy) <= 1e-13 * hy
    assert abs(ymin + hy) <= 1e-12 * hy
    # the topmost point of the ellipse is at dx = x_d: the column rows over a
    # zero-width slab at u + x_d reach exactly v - hy
    u, v = 100.0, 100.0
    ell = dict(u=u, v=v, a=a, b=b, c=c, t=t)
    Q = render.pixel_q(u, v, a, b, c, u + xd, v + ymin)[0]
    assert abs(Q - t) < 1e-9 * t


def _cell_min_q(u, v, a, b, c, x0, x1, y0, y1):
    """Brute-force minimum of Q over the closed cell: 0 if the centre is
    inside, else the minimum over the four edges of the 1-D quadratic."""
    X0, X1, Y0, Y1 = x0 - u, x1 - u, y0 - v, y1 - v
    if X0 <= 0 <= X1 and Y0 <= 0 <= Y1:
        return 0.0
    best = math.inf
    for X in (X0, X1):
        dy = min(max(-b * X / c, Y0), Y1)
        best = min(best, a * X * X + 2 * b * X * dy + c * dy * dy)
    for Yv in (Y0, Y1):
        dx = min(max(-b * Yv / a, X0), X1)
        best = min(best, a * dx * dx + 2 * b * dx * Yv + c * Yv * Yv)
    return best


def _random_ellipses(n, seed, W=160, H=128):
    rng = np.random.default_rng(seed)
    sx = np.exp(rng.uniform(np.log(0.5), np.log(60), n))
    sy = sx * np.exp(rng.uniform(-2.5, 2.5, n))
    th = rng.uniform(0, np.pi, n)
    ct, st = np.cos(th), np.sin(th)
    Sxx = ct * ct * sx * sx + st * st * sy * sy
    Syy = st * st * sx * sx + ct * ct * sy * sy
    Sxy = ct * st * (sx * sx - sy * sy)
    det = Sxx * Syy - Sxy * Sxy
    f32 = lambda x: np.asarray(x, np.float32).astype(np.float64)
    o = rng.uniform(0.002, 0.999, n)
    return dict(u=f32(rng.uniform(-40, W + 40, n)), v=f32(rng.uniform(-40, H + 40, n)),
                a=f32(Syy / det), b=f32(-Sxy / det), c=f32(Sxx / det),
                t=f32(2 * np.log(255 * o)), opacity=f32(o), visible=np.ones(n, bool),
                depth=f32(rng.uniform(1, 5, n)))


def test_column_walk_equals_closed_cell_predicate():
    cam = scenes.Camera(160, 128, 100, 100, 80, 64, np.eye(3), np.zeros(3))
    sp = _random_ellipses(400, seed=11)
    counts = binning.tile_counts(sp, cam)
    knife = 0
    for i in range(400):
        got = set(binning.tile_set(sp, cam, i).tolist())
        assert len(got) == counts[i]
        want = set()
        if sp['t'][i] > 0:
            for ty in range(cam.tiles_y):
                for tx in range(cam.tiles_x):
                    q = _cell_min_q(sp['u'][i], sp['v'][i], sp['a'][i], sp['b'][i], sp['c'][i],
                                    16 * tx, 16 * tx + 16, 16 * ty, 16 * ty + 16)
                    if abs(q - sp['t'][i]) <= 1e-9 * max(1.0, sp['t'][i]):
                        knife += 1
                        if (binning.tile_id(cam, tx, ty)) in got:
                            want.add(binning.tile_id(cam, tx, ty))
                    elif q <= sp['t'][i]:
                        want.add(binning.tile_id(cam, tx, ty))
        assert got == want, i
    assert knife < 5


def test_dense_sampling_and_pixel_centres_are_covered():
    cam = scenes.Camera(160, 128, 100, 100, 80, 64, np.eye(3), np.zeros(3))
    sp = _random_ellipses(150, seed=12)
    g = np.linspace(0, 16, 33)
    GX, GY = np.meshgrid(g, g)
    for i in range(150):
        got = set(binning.tile_set(sp, cam, i).tolist())
        if sp['t'][i] <= 0:
            assert not got
            continue
        for ty in range(cam.tiles_y):
            for tx in range(cam.tiles_x):
                Q = render.pixel_q(sp['u'][i], sp['v'][i], sp['a'][i], sp['b'][i], sp['c'][i],
                                   16 * tx + GX, 16 * ty + GY)[0]
                if np.any(Q < sp['t'][i] * (1 - 1e-9)):
                    assert binning.tile_id(cam, tx, ty) in got, (i, tx, ty)


def test_isotropic_tile_set_closed_form():
    # isotropic conic 1/s^2: cell in set iff distance(centre, cell) <= s sqrt(t)
    cam = scenes.Camera(256, 256, 100, 100, 128, 128, np.eye(3), np.zeros(3))
    rng = np.random.default_rng(3)
    for _ in range(60):
        s = float(np.float32(rng.uniform(1, 40)))
        a = float(np.float32(1 / (s * s)))
        u, v = (float(np.float32(x)) for x in rng.uniform(0, 256, 2))
        t = float(np.float32(rng.uniform(0.5, 11)))
        sp = dict(u=np.array([u]), v=np.array([v]), a=np.array([a]), b=np.array([0.0]),
                  c=np.array([a]), t=np.array([t]), visible=np.array([True]))
        got = set(binning.tile_set(sp, cam, 0).tolist())
        r = math.sqrt(t / a)
        for ty in range(16):
            for tx in range(16):
                dx = max(16 * tx - u, 0, u - 16 * tx - 16)
                dy = max(16 * ty - v, 0, v - 16 * ty - 16)
                d = math.hypot(dx, dy)
                if abs(d - r) < 1e-6 * r:
                    continue
                assert (binning.tile_id(cam, tx, ty) in got) == (d <= r)


def test_snugbox_extent_by_brute_force():
    sp = _random_ellipses(30, seed=4)
    for i in range(30):
        if sp['t'][i] <= 0:
            continue
        _, hx, hy = binning.half_extents(sp['a'][i], sp['b'][i], sp['c'][i], sp['t'][i])
        # sample the boundary densely: points d = sqrt(t) L^-T (cos, sin)
        ang = np.linspace(0, 2 * np.pi, 200001)
        Cm = np.array([[sp['a'][i], sp['b'][i]], [sp['b'][i], sp['c'][i]]])
        Lc = np.linalg.cholesky(Cm)
        pts = np.linalg.solve(Lc.T, np.stack([np.cos(ang), np.sin(ang)])) * math.sqrt(sp['t'][i])
        assert abs(np.abs(pts[0]).max() - hx) <= 1e-8 * hx
        assert abs(np.abs(pts[1]).max() - hy) <= 1e-8 * hy


def test_sorted_pairs_match_python_sort_and_scan():
    d = scenes.random_cloud(300, seed=9)
    pre = preprocess.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'],
                                d['sh'], 0, d['camera'])
    cam = d['camera']
    vals, ranges, keys = binning.sorted_pairs(pre, cam)
    zb = preprocess.depth_key(pre['depth'])
    tuples = []
    for i in range(300):
        for tid in binning.tile_set(pre, cam, i):
            tuples.append((int(tid), int(zb[i]), i))
    tuples.sort()
    assert [t[2] for t in tuples] == vals.tolist()
    counts = np.bincount([t[0] for t in tuples], minlength=cam.tiles_x * cam.tiles_y)
    assert ranges.tolist() == [0] + np.cumsum(counts).tolist()
    assert keys.tolist() == [(t[0] << 32) | t[1] for t in tuples]
    # per-tile query gives the same slices
    for tid in range(cam.tiles_x * cam.tiles_y):
        tx, ty = divmod(tid, cam.tiles_y)
        np.testing.assert_array_equal(binning.tile_members(pre, cam, tx, ty),
                                      vals[ranges[tid]:ranges[tid + 1]])


def test_counts_match_tile_sets_and_zero_for_faint():
    d = scenes.random_cloud(200, seed=4)
    d['opacity_logits'][:20] = -6.0  # o < 1/255: t < 0, no tiles
    pre = preprocess.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'],
                                d['sh'], 0, d['camera'])
    counts = binning.tile_counts(pre, d['camera'])
    assert np.all(counts[:20] == 0)
    for i in range(200):
        assert counts[i] == len(binning.tile_set(pre, d['camera'], i))
