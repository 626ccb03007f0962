"""Per-pixel compositing over the depth-sorted tile lists, and its backward
with respect to the 2D splat quantities, FP64 (oracle).

Sec. 2.1 (second step): every pixel walks the depth-sorted Gaussians of its
tile, computes each Gaussian's weight and alpha-blends front to back. The
blended depth of Sec. 3.1 uses each Gaussian's centroid depth.

Compositing model (3DGS formulation the paper builds on), pixel (x, y)
sampling the point (x + 0.5, y + 0.5):
    Q_i   = a dx^2 + 2 b dx dy + c dy^2,   d = (x+0.5 - u_i, y+0.5 - v_i)
    alpha_i = min(0.99f, o_i exp(-Q_i / 2))
    skip i if alpha_i < 1/255, decided as Q_i > t_i (equivalent by Eq. 1
        because 0.99 > 1/255), with Q_i evaluated in FP64 from the stored
        FP32 record in the fixed order dx*(a*dx + 2*(b*dy)) + dy*(c*dy)
    T' = T (1 - alpha_i); if T' < 1e-4f stop before blending i
    else C += c_i alpha_i T, D += z_i alpha_i T, T = T', n = i + 1
    output C + T bg, D, T_final = T, n_contrib = n

Backward (Sec. 2.2 computes the same gradients per splat instead of per
pixel; the values are those of the plain per-pixel chain rule), with the
contributor set held fixed and
    S^C_i = sum_{j>i} c_j alpha_j T_j + T_final bg,
    S^D_i = sum_{j>i} z_j alpha_j T_j:
    dC/dc_i = alpha_i T_i
    dC/dalpha_i = T_i c_i - S^C_i / (1 - alpha_i)
    dD/dalpha_i = T_i z_i - S^D_i / (1 - alpha_i)
    dD/dz_i = alpha_i T_i
    dalpha/d(oG) = 1 unless clamped at 0.99, dG/dQ = -G/2.

Constants. The clamp 0.99 and the stop threshold 1e-4 are the FP32 values
of those decimals (0.99f, 1e-4f): the compositing model is a single-precision
one, and with the FP64 decimals two stacked clamped splats would land on the
other side of the stop test ((1 - 0.99f)^2 < 1e-4f, (1 - 0.99)^2 > 1e-4).

Knife edges. The kernels evaluate alpha and the running product T in FP32
from the same stored records; the stop test can therefore differ from this
FP64 one only where T' lies within the FP32 error of T' from the threshold.
That error is bounded per pixel and carried along the list: an FP32
evaluation of o exp(-Q/2) has relative error at most
    eps_i = U (ALPHA_REL_M M_i + ALPHA_REL_0),  M_i = a dx^2 + 2|b dx dy| + c dy^2
(U = 2^-24; Q's three products and two roundings, the exponent scaling, the
exp2 and the product with o), so the factor (1 - alpha_i) carries relative
error alpha_i eps_i / (1 - alpha_i) (none once o G clears the clamp by more
than its error), and each factor and product adds a rounding:
    E_i = E_{i-1} + alpha_i eps_i / (1 - alpha_i) + 2 U   over blended splats.
A pixel is flagged ambiguous where a stop test has |T' - 1e-4| <=
STOP_SAFETY E_i T'. A Gaussian blended with |o G - 0.99| within
STOP_SAFETY eps_i o G is flagged for the gradient check (its clamp decision,
and with it the zero gradient through the clamp, may differ).
"""
from __future__ import annotations

import numpy as np

ALPHA_MAX = float(np.float32(0.99))   # 0.99f
T_STOP = float(np.float32(1e-4))      # 1e-4f
U32 = 2.0 ** -24        # unit roundoff of FP32
ALPHA_REL_M = 6.0       # FP32 relative error of o G, in U per unit of M (2x the derived 3)
ALPHA_REL_0 = 8.0       # and in U independent of M (2x the derived 4)
STOP_SAFETY = 2.0       # second-order terms of the running-product bound


def alpha_rel_error(a, b, c, dx, dy):
    """Bound on the relative error of an FP32 evaluation of o exp(-Q/2)."""
    M = a * dx * dx + 2.0 * np.abs(b * dx * dy) + c * dy * dy
    return U32 * (ALPHA_REL_M * M + ALPHA_REL_0)


def pixel_q(u, v, a, b, c, px, py):
    """Q at pixel-centre points, FP64, in the fixed order of operations."""
    dx = px - u
    dy = py - v
    return dx * (a * dx + 2.0 * (b * dy)) + dy * (c * dy), dx, dy


def _tile_pixels(cam, tx, ty):
    T = cam.tile
    xs = np.arange(tx * T, min(tx * T + T, cam.width))
    ys = np.arange(ty * T, min(ty * T + T, cam.height))
    X, Y = np.meshgrid(xs, ys)
    return X.ravel(), Y.ravel()


def _replay(sp, ids, px, py):
    """Front-to-back replay over a tile list for a set of pixels.

    Returns per-(splat, pixel) arrays (alpha, T before, blend mask, Q, dx, dy)
    truncated to the last splat any pixel blends, and per-pixel T, n and the
    ambiguity flags.
    """
    npix = len(px)
    T = np.ones(npix)
    E = np.zeros(npix)      # bound on the relative FP32 error of T
    n = np.zeros(npix, np.int64)
    nb = np.zeros(npix, np.int64)
    done = np.zeros(npix, bool)
    amb = np.zeros(npix, bool)
    amb_first = np.full(npix, -1, np.int64)
    stopped = np.zeros(npix, bool)
    n_clamped = np.zeros(npix, np.int64)
    rec = []
    for j, g in enumerate(ids):
        if done.all():
            break
        Q, dx, dy = pixel_q(sp['u'][g], sp['v'][g], sp['a'][g], sp['b'][g], sp['c'][g], px, py)
        use = ~done & (Q <= sp['t'][g])
        G = np.exp(-0.5 * Q)
        oG = sp['opacity'][g] * G
        alpha = np.minimum(ALPHA_MAX, oG)
        Tn = T * (1.0 - alpha)
        stop = use & (Tn < T_STOP)
        blend = use & ~stop
        eps = alpha_rel_error(sp['a'][g], sp['b'][g], sp['c'][g], dx, dy)
        clear = oG * (1.0 - eps) > ALPHA_MAX          # clamped on both sides
        En = E + np.where(clear, 0.0, alpha * eps / (1.0 - alpha)) + 2.0 * U32
        knife = use & (np.abs(Tn - T_STOP) <= STOP_SAFETY * En * Tn)
        amb_first = np.where(knife & (amb_first < 0), j, amb_first)
        amb |= knife
        rec.append((g, alpha, T.copy(), blend, G, oG, dx, dy, eps))
        T = np.where(blend, Tn, T)
        E = np.where(blend, En, E)
        n = np.where(blend, j + 1, n)
        nb += blend
        n_clamped += blend & (oG > ALPHA_MAX)
        stopped |= stop
        done |= stop
    last = int(n.max(initial=0))
    return rec[:last], T, n, (amb, amb_first), (nb, stopped, n_clamped)


def render(sp, cam, vals, ranges, bg=(0.0, 0.0, 0.0), tiles=None):
    """Forward compositing. `tiles` restricts to a list of (tx, ty).

    Returns dict(image[3,H,W], depth[H,W], T_final[H,W], n_contrib[H,W],
    ambiguous[H,W], ambiguous_from[H,W] (first list position of a knife-edge
    stop test, -1 if none), n_blended[H,W], stopped[H,W] (the pixel reached
    the early stop), n_clamped[H,W] (blended splats with alpha at the clamp),
    done[H,W], clamped_gaussians[N] (blended at the clamp at some pixel));
    pixels outside `tiles` are left at the initial values and `done` marks
    the ones computed.
    """
    H, W = cam.height, cam.width
    bg = np.asarray(bg, np.float64)
    image = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    T_final = np.ones((H, W))
    n_contrib = np.zeros((H, W), np.uint32)
    amb = np.zeros((H, W), bool)
    amb_first = np.full((H, W), -1, np.int64)
    n_blended = np.zeros((H, W), np.int64)
    stopped = np.zeros((H, W), bool)
    n_clamped = np.zeros((H, W), np.int64)
    done = np.zeros((H, W), bool)
    clamped_g = np.zeros(len(sp['u']), bool)
    if tiles is None:
        tiles = [(tx, ty) for tx in range(cam.tiles_x) for ty in range(cam.tiles_y)]
    for tx, ty in tiles:
        tid = tx * cam.tiles_y + ty   # column-major tile id (binning.tile_id)
        ids = np.asarray(vals[int(ranges[tid]):int(ranges[tid + 1])], np.int64)
        X, Y = _tile_pixels(cam, tx, ty)
        px, py = X + 0.5, Y + 0.5
        rec, T, n, a, nb = _replay(sp, ids, px, py)
        C = np.zeros((3, len(px)))
        D = np.zeros(len(px))
        for g, alpha, Tb, blend, _G, oG, *_rest in rec:
            clamped_g[g] |= bool(np.any(blend & (oG > ALPHA_MAX)))
            w = np.where(blend, alpha * Tb, 0.0)
            C += sp['rgb'][:, g][:, None] * w
            D += sp.get('dval', sp['depth'])[g] * w
        image[:, Y, X] = C + T * bg[:, None]
        depth[Y, X] = D
        T_final[Y, X] = T
        n_contrib[Y, X] = n
        amb[Y, X] = a[0]
        amb_first[Y, X] = a[1]
        n_blended[Y, X], stopped[Y, X], n_clamped[Y, X] = nb
        done[Y, X] = True
    return dict(image=image, depth=depth, T_final=T_final, n_contrib=n_contrib,
                ambiguous=amb, ambiguous_from=amb_first, n_blended=n_blended, stopped=stopped,
                n_clamped=n_clamped, done=done, clamped_gaussians=clamped_g)


GRAD2D = ('u', 'v', 'a', 'b', 'c', 'opacity', 'r', 'g', 'b_col', 'depth')


def render_backward(sp, cam, vals, ranges, dL_dimage, dL_ddepth=None, bg=(0.0, 0.0, 0.0),
                    tiles=None):
    """Gradients of L w.r.t. the 2D quantities of every Gaussian.

    Returns (grad2d[10, N] in the GRAD2D order, clamp_flag[N]) where
    clamp_flag marks Gaussians blended with o G within the FP32 error of 0.99.
    """
    N = len(sp['u'])
    bg = np.asarray(bg, np.float64)
    dC_img = np.asarray(dL_dimage, np.float64)
    dD_img = None if dL_ddepth is None else np.asarray(dL_ddepth, np.float64)
    grad = np.zeros((10, N))
    clamp_flag = np.zeros(N, bool)
    if tiles is None:
        tiles = [(tx, ty) for tx in range(cam.tiles_x) for ty in range(cam.tiles_y)]
    for tx, ty in tiles:
        tid = tx * cam.tiles_y + ty   # column-major tile id (binning.tile_id)
        ids = np.asarray(vals[int(ranges[tid]):int(ranges[tid + 1])], np.int64)
        X, Y = _tile_pixels(cam, tx, ty)
        px, py = X + 0.5, Y + 0.5
        rec, T_fin, _n, _a, _nb = _replay(sp, ids, px, py)
        if not rec:
            continue
        dC = dC_img[:, Y, X]
        dD = np.zeros(len(px)) if dD_img is None else dD_img[Y, X]
        # contributions w_j c_j and w_j z_j, then suffix sums behind each splat
        L = len(rec)
        wc = np.zeros((L, 3, len(px)))
        wz = np.zeros((L, len(px)))
        for j, (g, alpha, Tb, blend, *_rest) in enumerate(rec):
            w = np.where(blend, alpha * Tb, 0.0)
            wc[j] = sp['rgb'][:, g][:, None] * w
            wz[j] = sp.get('dval', sp['depth'])[g] * w
        SC = np.cumsum(wc[::-1], axis=0)[::-1] - wc + (T_fin * bg[:, None])[None]
        SD = np.cumsum(wz[::-1], axis=0)[::-1] - wz
        for j, (g, alpha, Tb, blend, G, oG, dx, dy, eps) in enumerate(rec):
            if not blend.any():
                continue
            col = sp['rgb'][:, g][:, None]
            z = sp.get('dval', sp['depth'])[g]
            w = alpha * Tb
            dL_dalpha = (np.sum(dC * (Tb * col - SC[j] / (1.0 - alpha)), axis=0)
                         + dD * (Tb * z - SD[j] / (1.0 - alpha)))
            clamped = oG > ALPHA_MAX
            dL_doG = np.where(clamped, 0.0, dL_dalpha)
            dL_dQ = dL_doG * sp['opacity'][g] * (-0.5 * G)
            m = blend
            a_, b_, c_ = sp['a'][g], sp['b'][g], sp['c'][g]
            grad[0, g] += np.sum(m * dL_dQ * (-2.0 * (a_ * dx + b_ * dy)))
            grad[1, g] += np.sum(m * dL_dQ * (-2.0 * (b_ * dx + c_ * dy)))
            grad[2, g] += np.sum(m * dL_dQ * dx * dx)
            grad[3, g] += np.sum(m * dL_dQ * 2.0 * dx * dy)
            grad[4, g] += np.sum(m * dL_dQ * dy * dy)
            grad[5, g] += np.sum(m * np.where(clamped, 0.0, dL_dalpha * G))
            grad[6:9, g] += np.sum(m * dC * w, axis=1)
            grad[9, g] += np.sum(m * dD * w)
            clamp_flag[g] |= bool(np.any(m & (np.abs(oG - ALPHA_MAX) <= STOP_SAFETY * eps * oG)))
    return grad, clamp_flag


def l1_loss_grad(image, target):
    """Mean absolute error over all 3HW values and its gradient
    sign(C - target) / (3HW), with sign(0) = 0."""
    image = np.asarray(image, np.float64)
    target = np.asarray(target, np.float64)
    diff = image - target
    return np.mean(np.abs(diff)), np.sign(diff) / diff.size
