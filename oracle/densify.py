"""Depth supervision (Sec. 3.1, depth regularisation) and multi-view
score-guided densification (Sec. 3.2, Eq. 3-4). Test infrastructure only.

Depth loss: the blended (centroid) depth D is supervised by a depth map D~
with an L1 term of weight w: L_d = w mean |D - D~|, dL_d/dD = w sign(D - D~)/n
with sign(0) = 0.

Eq. 3: the per-pixel photometric error of view j is the L1 norm over the
colour channels of (rendered - ground truth), normalised over the view;
pixels whose normalised error exceeds tau form the mask M^j. Reading:
normalise = min-max over the view, so e' > tau is decided as
(e - min e) > tau (max e - min e); a view with max e = min e has an empty
mask. This decision sets an integer (the mask), so it is taken in FP32
with the operations in this order: e = (|r0 - g0| + |r1 - g1|) + |r2 - g2|,
then the subtraction, the product and the comparison, each rounded to FP32.

Eq. 4: s_i^+ = (1/K) sum_j sum_{(u,v)} M^j(u,v) over the pixels to which
primitive i contributes. Reading: "contributes" = i is blended at that
pixel (the forward's contributor set); the score is kept as the integer
count sum_j sum M^j (the 1/K factor is applied to the threshold).

Growth: a primitive whose count reaches the threshold is cloned when its
largest scale is at most `split_scale`, else split in two. Reading (the
paper names clone and split only): the 3DGS rule, with the split children
placed at mu + R S eps_k for two standard-normal draws eps_k (given as
inputs) and scales divided by 1.6; all other attributes are copied. The
output keeps index order: Gaussian i's one or two entries follow those of
i - 1; a clone's copy follows the original.

Threshold: the paper uses a predefined threshold on s_i^+. Reading: that
constant is a lower bound t_min on the count, and a densification event also
has a growth budget (at most `cap` selected Gaussians), so its threshold is
the smallest t >= t_min with #{i : count_i >= t} <= cap, searched for
t <= 65535; none qualifying gives 0xFFFFFFFF.
"""
from __future__ import annotations

import math

import numpy as np

from . import preprocess as _pre
from . import render as _ren

SPLIT_SCALE_DIV = 1.6
SCORE_TOP = 65535
NO_THRESHOLD = 0xFFFFFFFF


def depth_l1(depth, target, weight):
    d = np.asarray(depth, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return weight * np.abs(d).mean(), weight * np.sign(d) / n


def error_mask(image, target, tau):
    """Eq. 3 mask [H, W] (bool) from images [3, H, W], decided in FP32."""
    f = np.float32
    x = np.asarray(image, f)
    g = np.asarray(target, f)
    e = (np.abs(x[0] - g[0]) + np.abs(x[1] - g[1])) + np.abs(x[2] - g[2])
    mn, mx = e.min(), e.max()
    return (e - mn) > f(tau) * (mx - mn)


def split_score(sp, cam, vals, ranges, mask):
    """Eq. 4 counts [N] for one view: masked pixels where each Gaussian is
    blended. Also returns `uncertain` [N]: masked knife-edge pixels (R8
    flags) whose blended set near the stop can differ between FP32 and FP64,
    counted for the Gaussians at list positions from the first knife-edge
    test - 1 to one past the last contributor."""
    N = len(sp['u'])
    score = np.zeros(N, np.int64)
    unc = np.zeros(N, np.int64)
    mask = np.asarray(mask, bool)
    for tx in range(cam.tiles_x):
        for ty in range(cam.tiles_y):
            tid = tx * cam.tiles_y + ty
            ids = np.asarray(vals[int(ranges[tid]):int(ranges[tid + 1])], np.int64)
            if len(ids) == 0:
                continue
            X, Y = _ren._tile_pixels(cam, tx, ty)
            m = mask[Y, X]
            if not m.any():
                continue
            rec, _T, n, (amb, amb_first), _nb = _ren._replay(sp, ids, X + 0.5, Y + 0.5)
            for g, _a, _Tb, blend, *_ in rec:
                score[g] += int(np.sum(blend & m))
            for p in np.nonzero(amb & m)[0]:
                lo = max(0, min(int(amb_first[p]), int(n[p])) - 1)
                hi = min(len(ids), int(n[p]) + 2)
                unc[ids[lo:hi]] += 1
    return score, unc


def densify(params, sh_degree, score, threshold, split_scale, eps, prune=None):
    """Clone / split the Gaussians whose count reaches `threshold`, and
    remove those marked in `prune` (Eq. 6; removal wins over growth).

    params: means[3,N], log_scales[3,N], quats[4,N], opacity_logits[N],
    sh[K,3,N]; eps[2,3,N] standard-normal draws for the split children.
    Returns the new parameter dict (FP32) and per-input output counts.
    """
    f = np.float64
    mu = np.asarray(params['means'], f)
    s = np.asarray(params['log_scales'], f)
    q = np.asarray(params['quats'], f)
    N = mu.shape[1]
    gone = np.zeros(N, bool) if prune is None else np.asarray(prune, bool)
    sel = (np.asarray(score, np.int64) >= int(threshold)) & ~gone
    big = np.exp(s).max(axis=0) > split_scale
    split = sel & big
    clone = sel & ~big
    counts = np.where(gone, 0, np.where(sel, 2, 1))
    qn = q / np.sqrt(np.sum(q * q, axis=0))
    R = _pre.quat_to_rotmat(qn)                                  # [N,3,3]
    scale = np.exp(s)
    out = {k: [] for k in params}
    child = {}
    for k in (0, 1):
        local = scale * np.asarray(eps[k], f)                   # S eps
        child[k] = mu + np.einsum('nij,jn->in', R, local)
    ls_child = s - math.log(SPLIT_SCALE_DIV)
    idx = []   # (source, kind) kind: 0 original, 1 clone copy, 2/3 split child
    for i in range(N):
        if gone[i]:
            continue
        if split[i]:
            idx += [(i, 2), (i, 3)]
        elif clone[i]:
            idx += [(i, 0), (i, 1)]
        else:
            idx.append((i, 0))
    src = np.array([a for a, _ in idx], np.int64)
    kind = np.array([b for _, b in idx], np.int64)
    res = {}
    for k, v in params.items():
        res[k] = np.asarray(v, np.float32)[..., src].copy()
    for c, kk in ((2, 0), (3, 1)):
        sel_c = kind == c
        res['means'][:, sel_c] = child[kk][:, src[sel_c]].astype(np.float32)
        res['log_scales'][:, sel_c] = ls_child[:, src[sel_c]].astype(np.float32)
    return res, counts


def growth_threshold(score, t_min, cap):
    """Smallest t >= t_min with at most `cap` counts >= t (t <= 65535), from
    the counts sorted in descending order: count(>= t) <= cap exactly when the
    (cap + 1)-th largest count is below t."""
    s = np.sort(np.asarray(score, np.int64))[::-1]
    if cap >= len(s) or s[cap] < t_min:
        return int(t_min)
    t = int(s[cap]) + 1
    return t if t <= SCORE_TOP else NO_THRESHOLD
