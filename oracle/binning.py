"""Compact tile sets and the (tile, depth)-sorted pair list, FP64 (oracle).

Sec. 2.1, Eq. (1)-(2): with conic (a, b, c), centroid (u, v) and opacity o,
a pixel is blended only where alpha = o exp(-Q/2) >= 1/255, i.e. where
Q(d) = a dx^2 + 2 b dx dy + c dy^2 <= t with t = 2 ln(255 o) (Eq. 1).
The ellipse Q = t has half-extents
    hx = sqrt(t * Sigma'_xx) = sqrt(t c / (a c - b^2)),
    hy = sqrt(t * Sigma'_yy) = sqrt(t a / (a c - b^2))
(the SnugBox; Eq. 2 as printed has b^2 - ac where the tangent condition
gives ac - b^2, since ac > b^2 for any positive-definite conic).

The tile set follows the paper's column walk: for each column of tiles
inside the SnugBox, the y-range of the ellipse over that column's slab
[x_tmin, x_tmax] is computed analytically from the branch formula of Eq. 2,
y(dx) = (-b dx +- sqrt((b^2 - ac) dx^2 + c t)) / c,
and every tile of the column whose closed cell overlaps that y-range is
written. Tile (tx, ty) is the closed cell [T tx, T tx + T] x [T ty, T ty + T]
in continuous pixel units (T = tile size); the grid has ceil(W/T) x ceil(H/T)
tiles. This equals "the closed cell meets the ellipse" exactly in real
arithmetic (the slab-ellipse intersection is convex).

Everything here is evaluated in FP64 on the FP32-stored (u, v, a, b, c, t),
in a fixed order of operations, so that the tile set is a function of the
stored record.

Sort (Sec. 2.1: each tile writes the tile id and the centroid depth for the
later depth sort): pairs are ordered by (tile id, FP32 depth bits), ties by
ascending Gaussian index. The paper fixes no tile numbering; tiles are
numbered column-major, id = tx * tiles_y + ty, so that one column of the
column walk covers consecutive ids.
"""
from __future__ import annotations

import numpy as np

from .preprocess import depth_key


def _f(x):
    return np.asarray(x, np.float64)


def tile_id(cam, tx, ty):
    """Column-major tile id."""
    return tx * cam.tiles_y + ty


def half_extents(a, b, c, t):
    a, b, c, t = _f(a), _f(b), _f(c), _f(t)
    det = a * c - b * b
    with np.errstate(invalid='ignore', divide='ignore'):
        hx = np.sqrt((t * c) / det)
        hy = np.sqrt((t * a) / det)
    return det, hx, hy


def has_tiles(visible, a, b, c, t):
    a, b, c, t = _f(a), _f(b), _f(c), _f(t)
    det = a * c - b * b
    return np.asarray(visible, bool) & (t > 0.0) & (det > 0.0)


def column_span(u, a, b, c, t, tile, tiles_x):
    """First and last tile column (inclusive) whose closed slab meets
    [u - hx, u + hx], clamped to the grid."""
    _, hx, _ = half_extents(a, b, c, t)
    u = _f(u)
    with np.errstate(invalid='ignore'):
        tx0 = np.maximum(0.0, np.ceil((u - hx) / tile) - 1.0)
        tx1 = np.minimum(float(tiles_x - 1), np.floor((u + hx) / tile))
    return tx0, tx1


def column_rows(u, v, a, b, c, t, tx, tile, tiles_y):
    """Row range [ty0, ty1] of the ellipse over the slab of column tx.

    Returns float arrays; the column is empty where ty0 > ty1.
    """
    u, v, a, b, c, t, tx = _f(u), _f(v), _f(a), _f(b), _f(c), _f(t), _f(tx)
    det, hx, hy = half_extents(a, b, c, t)
    ct = c * t
    xl = tile * tx - u
    xr = (tile * tx + tile) - u
    dl = np.maximum(xl, -hx)
    dr = np.minimum(xr, hx)
    with np.errstate(invalid='ignore', divide='ignore'):
        sl = np.sqrt(np.maximum(ct - det * (dl * dl), 0.0))
        sr = np.sqrt(np.maximum(ct - det * (dr * dr), 0.0))
        bl = b * dl
        br = b * dr
        lo = np.minimum(-(bl + sl) / c, -(br + sr) / c)   # lower branch at both ends
        hi = np.maximum((sl - bl) / c, (sr - br) / c)     # upper branch at both ends
        dxt = (b * hy) / a                                # x-offset of the topmost point
        ymin = np.where((dl <= dxt) & (dxt <= dr), -hy, lo)
        ymax = np.where((dl <= -dxt) & (-dxt <= dr), hy, hi)
        ty0 = np.maximum(0.0, np.ceil((v + ymin) / tile) - 1.0)
        ty1 = np.minimum(float(tiles_y - 1), np.floor((v + ymax) / tile))
    empty = ~(dl <= dr)
    ty0 = np.where(empty, 1.0, ty0)
    ty1 = np.where(empty, 0.0, ty1)
    return ty0, ty1


def tile_counts(sp, cam):
    """Exact number of tiles per Gaussian (uint32)."""
    ok = has_tiles(sp['visible'], sp['a'], sp['b'], sp['c'], sp['t'])
    idx = np.nonzero(ok)[0]
    n = np.zeros(len(sp['u']), np.int64)
    if len(idx) == 0:
        return n.astype(np.uint32)
    g = {k: sp[k][idx] for k in ('u', 'v', 'a', 'b', 'c', 't')}
    tx0, tx1 = column_span(g['u'], g['a'], g['b'], g['c'], g['t'], cam.tile, cam.tiles_x)
    ncols = np.maximum(tx1 - tx0 + 1.0, 0.0).astype(np.int64)
    acc = np.zeros(len(idx), np.int64)
    for k in range(int(ncols.max(initial=0))):
        act = k < ncols
        ty0, ty1 = column_rows(g['u'][act], g['v'][act], g['a'][act], g['b'][act], g['c'][act],
                               g['t'][act], tx0[act] + k, cam.tile, cam.tiles_y)
        acc[act] += np.maximum(ty1 - ty0 + 1.0, 0.0).astype(np.int64)
    n[idx] = acc
    return n.astype(np.uint32)


def tile_set(sp, cam, i):
    """Sorted list of tile ids of Gaussian i."""
    if not has_tiles(sp['visible'][i], sp['a'][i], sp['b'][i], sp['c'][i], sp['t'][i]):
        return np.zeros(0, np.int64)
    tx0, tx1 = column_span(sp['u'][i], sp['a'][i], sp['b'][i], sp['c'][i], sp['t'][i],
                           cam.tile, cam.tiles_x)
    out = []
    for tx in range(int(tx0), int(tx1) + 1):
        ty0, ty1 = column_rows(sp['u'][i], sp['v'][i], sp['a'][i], sp['b'][i], sp['c'][i],
                               sp['t'][i], tx, cam.tile, cam.tiles_y)
        for ty in range(int(ty0), int(ty1) + 1):
            out.append(tile_id(cam, tx, ty))
    return np.sort(np.asarray(out, np.int64))


def tile_members(sp, cam, tx, ty):
    """Gaussian ids whose tile set contains (tx, ty), in sort order
    (depth bits, then index)."""
    ok = has_tiles(sp['visible'], sp['a'], sp['b'], sp['c'], sp['t'])
    tx0, tx1 = column_span(sp['u'], sp['a'], sp['b'], sp['c'], sp['t'], cam.tile, cam.tiles_x)
    cand = np.nonzero(ok & (tx0 <= tx) & (tx <= tx1))[0]
    ty0, ty1 = column_rows(sp['u'][cand], sp['v'][cand], sp['a'][cand], sp['b'][cand],
                           sp['c'][cand], sp['t'][cand], tx, cam.tile, cam.tiles_y)
    mem = cand[(ty0 <= ty) & (ty <= ty1)]
    keys = depth_key(sp['depth'][mem])
    order = np.lexsort((mem, keys))
    return mem[order]


def sorted_pairs(sp, cam):
    """Full pair list: (vals = Gaussian ids, ranges[n_tiles+1], keys u64).

    keys = tile_id << 32 | depth bits. Small scenes only (materialises P).
    """
    counts = tile_counts(sp, cam).astype(np.int64)
    gids, tiles = [], []
    for i in np.nonzero(counts)[0]:
        ts = tile_set(sp, cam, i)
        assert len(ts) == counts[i]
        gids.append(np.full(len(ts), i, np.int64))
        tiles.append(ts)
    n_tiles = cam.tiles_x * cam.tiles_y
    if not gids:
        return (np.zeros(0, np.uint32), np.zeros(n_tiles + 1, np.uint32),
                np.zeros(0, np.uint64))
    gids = np.concatenate(gids)
    tiles = np.concatenate(tiles)
    z = depth_key(sp['depth'][gids]).astype(np.int64)
    order = np.lexsort((gids, z, tiles))
    vals = gids[order].astype(np.uint32)
    st = tiles[order]
    ranges = np.searchsorted(st, np.arange(n_tiles + 1)).astype(np.uint32)
    keys = (st.astype(np.uint64) << np.uint64(32)) | z[order].astype(np.uint64)
    return vals, ranges, keys


# ---------------------------------------------------------------------------
# Tile-set variants of the binning ablation (Sec. 2.1 contrasts the compact
# tile set with loose boxes). Counts per Gaussian on the stored record, FP64.

def _box_cells(lo, hi, tile, n):
    c0 = np.maximum(0.0, np.ceil(lo / tile) - 1.0)
    c1 = np.minimum(float(n - 1), np.floor(hi / tile))
    return c0, c1


def _box_counts(u, v, hx, hy, ok, cam):
    x0, x1 = _box_cells(u - hx, u + hx, cam.tile, cam.tiles_x)
    y0, y1 = _box_cells(v - hy, v + hy, cam.tile, cam.tiles_y)
    nx = np.maximum(x1 - x0 + 1.0, 0.0)
    ny = np.maximum(y1 - y0 + 1.0, 0.0)
    return np.where(ok, nx * ny, 0.0).astype(np.int64)


def snugbox_counts(sp, cam):
    """Tiles whose closed cell meets the SnugBox rectangle."""
    ok = has_tiles(sp['visible'], sp['a'], sp['b'], sp['c'], sp['t'])
    with np.errstate(invalid='ignore', divide='ignore'):
        _, hx, hy = half_extents(sp['a'], sp['b'], sp['c'], sp['t'])
    hx = np.where(ok, hx, 0.0)
    hy = np.where(ok, hy, 0.0)
    return _box_counts(_f(sp['u']), _f(sp['v']), hx, hy, ok, cam)


def sigma3_counts(sp, cam):
    """Tiles whose closed cell meets the square of half-width
    r = ceil(3 sqrt(lambda)) about the centroid, lambda = mid + sqrt(max(0.1,
    mid^2 - det(Sigma'))) from Sigma' = conic^-1 (3DGS's binning radius; the
    opacity is not considered)."""
    a, b, c = _f(sp['a']), _f(sp['b']), _f(sp['c'])
    det = a * c - b * b
    ok = np.asarray(sp['visible'], bool) & (det > 0.0)
    d = np.where(ok, det, 1.0)
    sxx, syy, sxy = c / d, a / d, -b / d
    mid = 0.5 * (sxx + syy)
    lam = mid + np.sqrt(np.maximum(0.1, mid * mid - (sxx * syy - sxy * sxy)))
    r = np.where(ok, np.ceil(3.0 * np.sqrt(np.maximum(lam, 0.0))), 0.0)
    return _box_counts(_f(sp['u']), _f(sp['v']), r, r, ok, cam)
