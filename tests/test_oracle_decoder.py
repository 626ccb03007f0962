"""Pins of the oracle's anchor decoder (Sec. 2.3, Neural-Gaussians): BF16
rounding against torch's conversion, closed-form networks whose outputs can
be written down (zero second layer, a wiring that copies chosen features
and view-direction components to chosen children), the child-mean
placement, and the analytic backward against central differences of the
unrounded FP64 forward. Also the direct-mode preprocess (decoder output
attributes) against the activated standard path."""
import math

import numpy as np
import pytest
import torch

from oracle import backward, decoder, preprocess
from paper_2601_19489_amd import scenes


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                         -1.0 - 2 ** -8, 65504.0, 3.0e38, 1e-40]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = decoder.bf16(x32)
    np.testing.assert_array_equal(got, want)


def test_bf16_midpoint_distance():
    # BF16 keeps 8 significant bits: between 1 and 2 the spacing is 2^-7,
    # between 2 and 4 it is 2^-6; a midpoint is at distance 0
    d = decoder.bf16_midpoint_distance
    assert d(np.array([1.0]))[0] == 2.0 ** -9          # down: spacing below 1 is 2^-8
    assert d(np.array([1.5]))[0] == 2.0 ** -8
    assert d(np.array([3.0]))[0] == 2.0 ** -7
    assert d(np.array([1.0 + 2.0 ** -8]))[0] == 0.0
    assert d(np.array([3.0 + 2.0 ** -7]))[0] == 0.0
    # brute force: the rounding of x does not change within the distance and
    # changes just beyond it on one side (margins well above FP32 resolution)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.01, 50.0, 4000)
    dist = d(x)
    x, dist = x[dist > 1e-4 * x], dist[dist > 1e-4 * x]
    v = decoder.bf16(x)
    for sign in (-1, 1):
        assert np.all(decoder.bf16(x + sign * dist * 0.99) == v)
    beyond = (decoder.bf16(x + dist * 1.01) != v) | (decoder.bf16(x - dist * 1.01) != v)
    assert np.all(beyond)


def _one_anchor_model(A=4, seed=1):
    a = scenes.anchor_cloud(A, seed=seed)
    m = {k: np.zeros_like(v) for k, v in scenes.decoder_mlp().items()}
    return a, m


def test_zero_second_layer_gives_activated_biases():
    a = scenes.anchor_cloud(5, seed=2)
    m = scenes.decoder_mlp(seed=3)
    m['w2'][:] = 0.0
    ch, _ = decoder.decode(a, m, np.array([0.0, 0.0, -4.0]))
    b2 = m['b2'].astype(np.float64)
    k, A = 10, 5
    for j in range(k):
        sl = slice(j * A, (j + 1) * A)
        np.testing.assert_allclose(ch['opacity'][sl], max(0.0, math.tanh(b2[j])), rtol=1e-15)
        for c in range(3):
            np.testing.assert_allclose(ch['rgb'][c, sl], 1 / (1 + math.exp(-b2[10 + 3 * j + c])),
                                       rtol=1e-15)
            np.testing.assert_allclose(
                ch['scales'][c, sl],
                a['scaling'][3 + c].astype(np.float64) / (1 + math.exp(-b2[40 + 7 * j + c])),
                rtol=1e-14)
        q = b2[40 + 7 * j + 3:40 + 7 * j + 7]
        np.testing.assert_allclose(ch['quats'][:, sl], (q / np.linalg.norm(q))[:, None] *
                                   np.ones((1, A)), rtol=1e-14)


def test_wired_network_copies_features_and_view_direction():
    # opacity head: hidden unit j = feature j (j < 10), child j reads unit j;
    # colour head: hidden units 0-2 = view direction, child j channel c reads
    # unit c; covariance head: zero weights, biases give unit sigmoid scale
    # factor (saturated) and the identity rotation.
    A = 6
    a = scenes.anchor_cloud(A, seed=7)
    a['feat'][:] = np.linspace(-0.75, 0.75, 32 * A).reshape(32, A)
    m = {k: np.zeros_like(v) for k, v in scenes.decoder_mlp().items()}
    for j in range(10):
        m['w1'][j, j] = 1.0
        m['w2'][j, j] = 1.0
    for c in range(3):
        m['w1'][32 + c, 32 + c] = 1.0
        for j in range(10):
            m['w2'][10 + 3 * j + c, c] = 1.0
    for j in range(10):
        m['b2'][40 + 7 * j:40 + 7 * j + 3] = 40.0
        m['b2'][40 + 7 * j + 3] = 3.0
    campos = np.array([0.3, -0.2, -4.0])
    ch, _ = decoder.decode(a, m, campos, rounding=False)
    f = a['feat'].astype(np.float64)
    pos = a['pos'].astype(np.float64)
    d = campos[:, None] - pos
    d /= np.linalg.norm(d, axis=0)
    for j in range(10):
        sl = slice(j * A, (j + 1) * A)
        np.testing.assert_allclose(ch['opacity'][sl], np.tanh(np.maximum(f[j], 0.0)), rtol=1e-14)
        np.testing.assert_allclose(ch['rgb'][:, sl], 1 / (1 + np.exp(-np.maximum(d, 0.0))),
                                   rtol=1e-14)
        np.testing.assert_allclose(ch['scales'][:, sl], a['scaling'][3:6], rtol=1e-12)
        np.testing.assert_allclose(ch['quats'][:, sl], np.array([[1.0], [0.0], [0.0], [0.0]]) *
                                   np.ones((1, A)), atol=0)
        want_mean = pos + a['offsets'][3 * j:3 * j + 3].astype(np.float64) * a['scaling'][0:3]
        np.testing.assert_allclose(ch['means'][:, sl], want_mean, rtol=1e-15)


def test_rounded_forward_uses_bf16_operands():
    # with inputs and weights already BF16-exact and a wiring that keeps the
    # hidden units BF16-exact, rounding changes nothing
    A = 3
    a = scenes.anchor_cloud(A, seed=8)
    a['feat'][:] = decoder.bf16(a['feat'])
    m = scenes.decoder_mlp(seed=9)
    m['w1'][:, 32:] = 0.0
    m['b1'][:] = 0.0
    for k in ('w1', 'w2'):
        m[k][:] = decoder.bf16(m[k])
    m['w1'][:] = 0.0
    m['w1'][np.arange(32), np.arange(32)] = 1.0
    ch_r, _ = decoder.decode(a, m, np.array([0.0, 0.0, -4.0]), rounding=True)
    ch_u, _ = decoder.decode(a, m, np.array([0.0, 0.0, -4.0]), rounding=False)
    for k in ch_r:
        np.testing.assert_array_equal(ch_r[k], ch_u[k])


def test_decoder_backward_matches_central_differences():
    A = 3
    a = {k: v.astype(np.float64) for k, v in scenes.anchor_cloud(A, seed=11).items()}
    a['feat'] *= 8.0
    m = {k: v.astype(np.float64) for k, v in scenes.decoder_mlp(seed=12).items()}
    campos = np.array([0.2, 0.1, -4.0])
    rng = np.random.default_rng(13)
    ch, cache = decoder.decode(a, m, campos, rounding=False)
    assert np.min(np.abs(cache['z'])) > 1e-4 and np.min(np.abs(cache['y'][:10])) > 1e-4
    dch = {k: rng.standard_normal(v.shape) for k, v in ch.items()}
    g = decoder.decode_backward(cache, dch)

    def L(aa, mm):
        c, _ = decoder.decode(aa, mm, campos, rounding=False)
        return sum(np.sum(dch[k] * c[k]) for k in c)

    for group, src in (('feat', a), ('offsets', a), ('scaling', a), ('w1', m), ('b1', m),
                       ('w2', m), ('b2', m)):
        ana = g[group]
        fd = np.zeros_like(ana)
        for idx in np.ndindex(*src[group].shape):
            x0 = src[group][idx]
            h = 1e-6 * max(1.0, abs(x0))
            src[group][idx] = x0 + h
            Lp = L(a, m)
            src[group][idx] = x0 - h
            Lm = L(a, m)
            src[group][idx] = x0
            fd[idx] = (Lp - Lm) / (2 * h)
        scale = np.mean(np.abs(fd)) + 1e-30
        err = np.abs(ana - fd)
        assert np.all(err <= 1e-6 * (np.abs(fd) + scale)), (group, err.max(), scale)


def test_direct_mode_equals_activated_standard_path():
    d = scenes.random_cloud(300, seed=5)
    cam = d['camera']
    std = preprocess.preprocess(d['means'], d['log_scales'], d['quats'], d['opacity_logits'],
                                d['sh'], 0, cam)
    f = np.float64
    scale = np.exp(d['log_scales'].astype(f))
    op = 1 / (1 + np.exp(-d['opacity_logits'].astype(f)))
    rgb = np.maximum(d['sh'][0].astype(f) * (0.5 / math.sqrt(math.pi)) + 0.5, 0.0)
    dr = preprocess.preprocess(d['means'], scale, d['quats'], op, rgb[None], preprocess.DIRECT,
                               cam)
    for k in ('u', 'v', 'a', 'b', 'c', 'depth', 'opacity', 't', 'rgb'):
        np.testing.assert_allclose(dr[k], std[k], rtol=2e-7, atol=1e-30, err_msg=k)
    np.testing.assert_array_equal(dr['visible'], std['visible'])
    # gradients: chain rule through exp, sigmoid and the degree-0 colour term
    rng = np.random.default_rng(6)
    g2d = rng.standard_normal((10, 300))
    gs = backward.preprocess_backward(std, g2d, 0, cam)
    gd = backward.preprocess_backward(dr, g2d, preprocess.DIRECT, cam)
    vis = std['visible']
    np.testing.assert_allclose(gd['means'], gs['means'], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd['quats'], gs['quats'], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd['log_scales'] * scale, gs['log_scales'], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gd['opacity_logits'] * op * (1 - op), gs['opacity_logits'],
                               rtol=1e-9, atol=1e-15)
    live = vis[None] & (std['_rgb_raw'] >= 0)
    np.testing.assert_allclose(np.where(live, gd['sh'][0] * 0.5 / math.sqrt(math.pi), 0),
                               gs['sh'][0], rtol=1e-12, atol=1e-15)
