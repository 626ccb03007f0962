"""Anchor (neural-Gaussian) decoder, FP64 (oracle). Test infrastructure only.

Sec. 2.3 (Representation: Neural-Gaussians, after Scaffold-GS): each anchor
holds a learned feature vector, and a single small network shared by all
anchors turns that vector (with the viewing direction) into the attributes
of the anchor's child Gaussians at every render. The children go through
the ordinary rasterizer; training adjusts the features and the network
weights rather than per-Gaussian attributes.

Readings (the paper gives no architecture):
  * k = 10 children per anchor; feature width 32; the MLP input is the
    feature followed by the unit direction from the anchor to the camera
    centre (35 values).
  * three heads (opacity, colour, covariance), each Linear(35 -> 32), ReLU,
    Linear(32 -> k d) with d = 1, 3, 7. Stacked: W1[96, 35] (rows 32 h .. 32 h
    + 31 are head h), b1[96], W2[110, 32] (rows 0-9 opacity, 10-39 colour,
    40-109 covariance; head h reads hidden units 32 h .. 32 h + 31), b2[110].
  * child j of anchor i (Gaussian j A + i of A anchors):
        opacity = max(0, tanh(y_op[j]))
        rgb[ch] = sigmoid(y_col[3 j + ch])
        scale[a] = scaling[3 + a] sigmoid(y_cov[7 j + a]),  a < 3
        quat = y_cov[7 j + 3 .. 7 j + 6] / |.|              (w, x, y, z)
        mean = pos + offsets[3 j .. 3 j + 2] * scaling[0 .. 2]
    scaling[6, A] is given as positive (already exponentiated) values.
  * BF16 rounding points: the input x, W1, the hidden activation h and W2
    are rounded (round to nearest even, through FP32); products are then
    exact, sums FP64 here. The backward treats each rounding as the identity
    (straight-through) and uses the rounded values where the forward did.
"""
from __future__ import annotations

import numpy as np

K_CHILD = 10
FEAT = 32
HID = 32
IN = FEAT + 3
HEAD_OUT = (10, 30, 70)          # opacity, colour, covariance outputs per anchor
HEAD_ROW = (0, 10, 40, 110)      # first row of each head in W2


def bf16(x):
    """Round to BF16 (round to nearest, ties to even) through FP32; returned
    as float64. The BF16 value keeps the top 16 bits of the FP32 pattern."""
    u = np.asarray(np.asarray(x, np.float64), np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_midpoint_distance(x):
    """|x - m| for the nearest point m at which the BF16 rounding of x
    changes: the midpoints between bf16(x) and its two BF16 neighbours (the
    neighbours differ from bf16(x) by one unit in the 8-bit significand,
    whose size depends on the exponent on each side)."""
    x = np.asarray(x, np.float64)
    v = bf16(x)
    b = np.abs(v).astype(np.float32).view(np.uint32).astype(np.int64)
    up = (b + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    dn = np.maximum(b - 0x10000, 0).astype(np.uint32).view(np.float32).astype(np.float64)
    a = np.abs(x)
    av = np.abs(v)
    return np.minimum(np.abs(a - 0.5 * (av + up)), np.abs(a - 0.5 * (av + dn)))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def view_dirs(pos, campos):
    """Unit directions from each anchor to the camera centre, [3, A]."""
    d = np.asarray(campos, np.float64)[:, None] - np.asarray(pos, np.float64)
    n = np.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    return d / n


def decode(anchors, mlp, campos, rounding=True):
    """Child Gaussians of all anchors for one camera centre.

    anchors: feat[32, A], pos[3, A], offsets[3 k, A], scaling[6, A].
    mlp: w1[96, 35], b1[96], w2[110, 32], b2[110].
    Returns (children, cache): children = means[3, N], scales[3, N],
    quats[4, N], opacity[N], rgb[3, N] with N = k A (child j of anchor i at
    j A + i); cache holds the intermediates the backward uses and the
    relative distance of each pre-activation to a BF16 rounding midpoint.
    """
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    feat = np.asarray(anchors['feat'], np.float64)
    pos = np.asarray(anchors['pos'], np.float64)
    off = np.asarray(anchors['offsets'], np.float64)
    scl = np.asarray(anchors['scaling'], np.float64)
    A = feat.shape[1]
    dirs = view_dirs(pos, campos)
    x = r(np.concatenate([feat, dirs], axis=0))                    # [35, A]
    w1, w2 = r(mlp['w1']), r(mlp['w2'])
    b1 = np.asarray(mlp['b1'], np.float64)
    b2 = np.asarray(mlp['b2'], np.float64)
    z = w1 @ x + b1[:, None]                                        # [96, A]
    h = r(np.maximum(z, 0.0))
    y = np.empty((HEAD_ROW[-1], A))
    for hd in range(3):
        rows = slice(HEAD_ROW[hd], HEAD_ROW[hd + 1])
        y[rows] = w2[rows] @ h[HID * hd:HID * (hd + 1)] + b2[rows][:, None]
    k = K_CHILD
    y_op = y[0:10]                                                  # [k, A]
    y_col = y[10:40].reshape(k, 3, A)
    y_cov = y[40:110].reshape(k, 7, A)
    th = np.tanh(y_op)
    opacity = np.maximum(th, 0.0)
    s_col = _sigmoid(y_col)
    s_scl = _sigmoid(y_cov[:, 0:3])
    scales = scl[None, 3:6] * s_scl
    qr = y_cov[:, 3:7]
    qn_norm = np.sqrt(np.sum(qr * qr, axis=1))
    quats = qr / qn_norm[:, None]
    offs = off.reshape(k, 3, A)
    means = pos[None] + offs * scl[None, 0:3]
    flat = lambda v: np.transpose(v, (1, 0, 2)).reshape(v.shape[1], k * A)
    children = dict(means=flat(means), scales=flat(scales), quats=flat(quats),
                    opacity=opacity.reshape(k * A), rgb=flat(s_col))
    # distance of every value that is rounded to BF16 after a sum, for the
    # knife-edge allowance of the parity tests
    zmag = np.abs(w1) @ np.abs(x) + np.abs(b1)[:, None]
    cache = dict(x=x, w1=w1, w2=w2, z=z, h=h, y=y, th=th, s_col=s_col, s_scl=s_scl, qr=qr,
                 qn_norm=qn_norm, quats=quats, offs=offs, scl=scl, dirs=dirs, zmag=zmag,
                 h_edge=np.where(z > 0, bf16_midpoint_distance(np.maximum(z, 0.0)), np.inf))

    return children, cache


def decode_backward(cache, dchild):
    """Gradients of the decoder from the child-Gaussian gradients.

    dchild: means[3, N], scales[3, N], quats[4, N], opacity[N], rgb[3, N].
    Returns feat[32, A], w1[96, 35], b1[96], w2[110, 32], b2[110],
    offsets[3 k, A], scaling[6, A].
    """
    k = K_CHILD
    A = cache['x'].shape[1]
    un = lambda v, d: np.transpose(np.asarray(v, np.float64).reshape(d, k, A), (1, 0, 2))
    dmean = un(dchild['means'], 3)
    dscale = un(dchild['scales'], 3)
    dquat = un(dchild['quats'], 4)
    dop = np.asarray(dchild['opacity'], np.float64).reshape(k, A)
    drgb = un(dchild['rgb'], 3)

    dy = np.zeros((HEAD_ROW[-1], A))
    th = cache['th']
    dy[0:10] = np.where(th > 0.0, dop * (1.0 - th * th), 0.0)
    s_col = cache['s_col']
    dy[10:40] = (drgb * s_col * (1.0 - s_col)).reshape(30, A)
    dyc = np.zeros((k, 7, A))
    s_scl, scl = cache['s_scl'], cache['scl']
    dyc[:, 0:3] = dscale * scl[None, 3:6] * s_scl * (1.0 - s_scl)
    qn, nrm = cache['quats'], cache['qn_norm']
    dyc[:, 3:7] = (dquat - qn * np.sum(qn * dquat, axis=1)[:, None]) / nrm[:, None]
    dy[40:110] = dyc.reshape(70, A)

    h, x, w1, w2 = cache['h'], cache['x'], cache['w1'], cache['w2']
    dw2 = np.zeros_like(w2)
    dh = np.zeros_like(h)
    for hd in range(3):
        rows = slice(HEAD_ROW[hd], HEAD_ROW[hd + 1])
        hs = slice(HID * hd, HID * (hd + 1))
        dw2[rows] = dy[rows] @ h[hs].T
        dh[hs] = w2[rows].T @ dy[rows]
    db2 = dy.sum(axis=1)
    dz = np.where(cache['z'] > 0.0, dh, 0.0)
    dw1 = dz @ x.T
    db1 = dz.sum(axis=1)
    dx = w1.T @ dz
    doff = (dmean * scl[None, 0:3]).reshape(3 * k, A)
    dscl = np.zeros((6, A))
    dscl[0:3] = np.sum(dmean * cache['offs'], axis=0)
    dscl[3:6] = np.sum(dscale * s_scl, axis=0)
    return dict(feat=dx[:FEAT], w1=dw1, b1=db1, w2=dw2, b2=db2, offsets=doff, scaling=dscl)
