"""Seeded synthetic inputs: Gaussian scenes, cameras and target images.

This module only draws and lays out inputs. It contains none of the
rasterizer's arithmetic, so the CPU oracle and the GPU path can both be fed
from it without sharing any of the method's computation.

Layout (structure of arrays, component-major, C-contiguous float32):
    means          [3, N]          world-space centres
    log_scales     [3, N]          per-axis log standard deviations
    quats          [4, N]          raw rotation quaternions (w, x, y, z)
    opacity_logits [N]             opacity before the sigmoid
    sh             [K, 3, N]       SH coefficients, K = (degree + 1)**2,
                                   coefficient index k = l*l + l + m

The workloads are synthetic stand-ins for the paper's scenes (the paper
trains on Tanks-and-Temples and on the challenge data, neither of which is
used here): a tiny random cloud, and a cloud sampled on noisy planes and
spheres with a heavy-tailed scale mix that makes a few Gaussians cover many
tiles (the imbalance the load-balanced tile writing of Sec. 2.1 targets).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point X maps to camera space as p = R @ X + t; the image point is
    (fx * p_x / p_z + cx, fy * p_y / p_z + cy) in continuous pixel units,
    where pixel (i, j) covers [i, i+1) x [j, j+1).
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float64, world -> camera rotation
    t: np.ndarray  # (3,) float64, world -> camera translation
    near: float = 0.2
    tile: int = 16
    depth_mode: int = 0  # blended depth channel: 0 = depth p_z, 1 = inverse depth 1 / p_z

    @property
    def tiles_x(self) -> int:
        return -(-self.width // self.tile)

    @property
    def tiles_y(self) -> int:
        return -(-self.height // self.tile)


def look_at_camera(eye, target, width, height, hfov_deg=60.0, up=(0.0, -1.0, 0.0),
                   near=0.2, tile=16) -> Camera:
    """Camera at `eye` looking at `target`; `up` is world-space image-up.

    With OpenCV axes image-up is -y, so the default up vector (0, -1, 0) makes
    an eye on the -z axis give R = I.
    """
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, np.float64)
    # camera y axis points down: the component of -up orthogonal to fwd
    down = -upv - np.dot(-upv, fwd) * fwd
    down /= np.linalg.norm(down)
    right = np.cross(down, fwd)
    R = np.stack([right, down, fwd])  # rows: camera axes in world coords
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(width, height, fx, fx, width / 2.0, height / 2.0, R, t, near, tile)


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


# 1/(2*sqrt(pi)) is the value of the degree-0 basis function; the DC
# coefficient is drawn so that the DC term plus the 0.5 offset equals a
# uniformly drawn colour (the colour model of the cited 3DGS formulation).
_DC_SCALE = 2.0 * math.sqrt(math.pi)


def random_cloud(n=1000, seed=0, width=64, height=64):
    """Tiny workload: N Gaussians in [-1,1]^3, SH degree 0, one 64x64 view.

    Draw order: means U[-1,1]^3, log-scales N(-3, 0.5), quaternions
    normalize(N(0, I4)), opacity logits N(0, 1), colour U[0,1]^3.
    The target image is U[0,1] with seed + 1.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (3, n))
    log_scales = rng.normal(-3.0, 0.5, (3, n))
    quats = _unit_quats(rng, n)
    opac = rng.normal(0.0, 1.0, n)
    colour = rng.uniform(0.0, 1.0, (3, n))
    sh = ((colour - 0.5) * _DC_SCALE)[None]
    cam = look_at_camera((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), width, height)
    target = np.random.default_rng(seed + 1).uniform(0.0, 1.0, (3, height, width))
    return dict(means=_f32(means), log_scales=_f32(log_scales), quats=_f32(quats),
                opacity_logits=_f32(opac), sh=_f32(sh), sh_degree=0, camera=cam,
                target=_f32(target))


def opaque_stack(seed=41, n=700, n_opaque=240, width=320, height=240):
    """Opaque scene for the alpha clamp and the early stop.

    The tiny cloud's generator (n Gaussians, SH degree 0), then:
    - the first n_opaque Gaussians made broad and nearly opaque: means
      U[-1.3,1.3] x U[-1,1] x U[-0.5,0.5], log-scales N(-1.0, 0.3), opacity
      logits U[5.3, 9] (opacity 0.995 and up);
    - the next 96 as 48 front pairs on an 8 x 6 grid (x in 8 steps over
      [-1.4, 1.4], y in 6 steps over [-1, 1], jitter N(0, 0.01^2)): two
      isotropic Gaussians of log-scale -2.5 and identity rotation at z = -1.3
      and -1.25, opacity logits U[7, 10]. Near a pair's centre both are
      saturated, so the second would take the transmittance to (1 - 0.99)^2.
    """
    d = random_cloud(n, seed=seed, width=width, height=height)
    rng = np.random.default_rng(seed + 1)
    m, s, o, q = d['means'], d['log_scales'], d['opacity_logits'], d['quats']
    m[0, :n_opaque] = rng.uniform(-1.3, 1.3, n_opaque)
    m[1, :n_opaque] = rng.uniform(-1.0, 1.0, n_opaque)
    m[2, :n_opaque] = rng.uniform(-0.5, 0.5, n_opaque)
    s[:, :n_opaque] = rng.normal(-1.0, 0.3, (3, n_opaque))
    o[:n_opaque] = rng.uniform(5.3, 9.0, n_opaque)
    gx, gy = np.meshgrid(np.linspace(-1.4, 1.4, 8), np.linspace(-1.0, 1.0, 6))
    k = gx.size
    for j in range(2):
        sl = slice(n_opaque + j, n_opaque + 2 * k, 2)
        m[0, sl] = gx.ravel() + rng.normal(0.0, 0.01, k)
        m[1, sl] = gy.ravel() + rng.normal(0.0, 0.01, k)
        m[2, sl] = -1.3 + 0.05 * j
        s[:, sl] = -2.5
        q[:, sl] = np.array([1.0, 0.0, 0.0, 0.0], np.float32)[:, None]
        o[sl] = rng.uniform(7.0, 10.0, k)
    return d


_PLANES = ((0, -0.8), (1, -0.2), (2, 0.4))  # (axis, offset): unit squares [-1,1]^2
_SPHERES = (((0.4, 0.4, 0.3), 0.35), ((-0.5, 0.3, -0.4), 0.30),
            ((0.3, -0.5, 0.5), 0.25), ((-0.4, -0.4, 0.0), 0.40))


def surface_cloud(n=500_000, seed=2, sh_degree=3, width=1600, height=1066,
                  large_frac=0.1, target_seed=None):
    """Heavy-tailed scene: Gaussians sampled on 3 planes and 4 spheres.

    Draw order: surface index (uniform over 7), in-surface position, position
    noise N(0, 0.01^2), large flag Bernoulli(large_frac), log-scales
    (N(-1.5, 0.5) if large else N(-4, 0.5), iid per axis), quaternions,
    opacity logits N(0, 1), DC colour U[0,1]^3, higher SH N(0, 0.1).
    The camera sits at (0, 0, -4) looking at the origin, hfov 60 degrees.
    """
    rng = np.random.default_rng(seed)
    surf = rng.integers(0, 7, n)
    uv = rng.uniform(-1.0, 1.0, (2, n))
    sdir = rng.standard_normal((3, n))
    sdir /= np.linalg.norm(sdir, axis=0, keepdims=True)
    means = np.empty((3, n))
    for k, (axis, off) in enumerate(_PLANES):
        sel = surf == k
        others = [a for a in range(3) if a != axis]
        means[axis, sel] = off
        means[others[0], sel] = uv[0, sel]
        means[others[1], sel] = uv[1, sel]
    for k, (centre, radius) in enumerate(_SPHERES):
        sel = surf == (3 + k)
        means[:, sel] = np.asarray(centre)[:, None] + radius * sdir[:, sel]
    means += rng.normal(0.0, 0.01, (3, n))
    large = rng.uniform(0.0, 1.0, n) < large_frac
    log_scales = np.where(large[None], rng.normal(-1.5, 0.5, (3, n)),
                          rng.normal(-4.0, 0.5, (3, n)))
    quats = _unit_quats(rng, n)
    opac = rng.normal(0.0, 1.0, n)
    colour = rng.uniform(0.0, 1.0, (3, n))
    K = (sh_degree + 1) ** 2
    sh = np.empty((K, 3, n))
    sh[0] = (colour - 0.5) * _DC_SCALE
    if K > 1:
        sh[1:] = rng.normal(0.0, 0.1, (K - 1, 3, n))
    cam = look_at_camera((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), width, height)
    ts = seed * 10 if target_seed is None else target_seed
    target = np.random.default_rng(ts).uniform(0.0, 1.0, (3, height, width)).astype(np.float32)
    return dict(means=_f32(means), log_scales=_f32(log_scales), quats=_f32(quats),
                opacity_logits=_f32(opac), sh=_f32(sh), sh_degree=sh_degree, camera=cam,
                target=target)


ORBIT_RESOLUTIONS = ((960, 540), (1024, 576), (1280, 720), (1440, 810), (1600, 900),
                     (1600, 1066), (1920, 1080), (1920, 1080))


def orbit_cameras(n_views=8, seed=3, radius=4.0, jitter=0.2, resolutions=ORBIT_RESOLUTIONS):
    """Views on a circle about the y axis, azimuth 2*pi*k/n + U(-j, j) and
    elevation U(-j, j); resolutions assigned by a seeded permutation."""
    rng = np.random.default_rng(seed)
    az = 2.0 * math.pi * np.arange(n_views) / n_views + rng.uniform(-jitter, jitter, n_views)
    el = rng.uniform(-jitter, jitter, n_views)
    perm = rng.permutation(len(resolutions))
    cams = []
    for k in range(n_views):
        w, h = resolutions[perm[k % len(resolutions)]]
        eye = radius * np.array([math.sin(az[k]) * math.cos(el[k]), -math.sin(el[k]),
                                 -math.cos(az[k]) * math.cos(el[k])])
        cams.append(look_at_camera(eye, (0.0, 0.0, 0.0), w, h))
    return cams


def random_image(shape, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, shape).astype(np.float32)


def anchor_cloud(n_anchors=100_000, seed=4, k=10, feat_dim=32, source_means=None):
    """Anchors for the neural-Gaussian decoder, drawn as the decoder reads them.

    Draw order: anchor positions (a random subset of `source_means` plus
    N(0, 0.02^2) noise, or points of the plane-and-sphere surfaces when none
    is given), features N(0, 0.1^2), child offsets N(0, 0.5^2), scaling
    exp(N(log 0.02, 0.3^2)) for the 3 offset axes and the 3 child-scale axes.
    Layout: feat[32, A], pos[3, A], offsets[3 k, A] (child j, axis d at row
    3 j + d), scaling[6, A] (positive values).
    """
    rng = np.random.default_rng(seed)
    if source_means is None:
        source_means = surface_cloud(n_anchors, seed=seed + 1000, sh_degree=0, width=16,
                                     height=16)['means']
    src = np.asarray(source_means, np.float64)
    pick = rng.choice(src.shape[1], n_anchors, replace=src.shape[1] < n_anchors)
    pos = src[:, pick] + rng.normal(0.0, 0.02, (3, n_anchors))
    feat = rng.normal(0.0, 0.1, (feat_dim, n_anchors))
    offsets = rng.normal(0.0, 0.5, (3 * k, n_anchors))
    scaling = np.exp(rng.normal(math.log(0.02), 0.3, (6, n_anchors)))
    return dict(feat=_f32(feat), pos=_f32(pos), offsets=_f32(offsets), scaling=_f32(scaling))


def sparse_init(gt_means, n, seed=5, sh_degree=3, noise=0.01, opacity=0.1):
    """Sparse starting point for a densifying fit: a random subset of the
    ground-truth means plus N(0, noise^2), isotropic log-scales from the mean
    distance to the 3 nearest neighbours, colour 0 (all SH coefficients 0,
    i.e. grey 0.5), opacity logit of `opacity`, identity rotations.
    Draw order: the subset, then the noise."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    src = np.asarray(gt_means, np.float64)
    pick = rng.choice(src.shape[1], n, replace=src.shape[1] < n)
    means = src[:, pick] + rng.normal(0.0, noise, (3, n))
    d, _ = cKDTree(means.T).query(means.T, k=4)
    dist = np.maximum(d[:, 1:].mean(axis=1), 1e-7)
    log_scales = np.repeat(np.log(dist)[None], 3, axis=0)
    quats = np.zeros((4, n))
    quats[0] = 1.0
    K = (sh_degree + 1) ** 2
    return dict(means=_f32(means), log_scales=_f32(log_scales), quats=_f32(quats),
                opacity_logits=_f32(np.full(n, math.log(opacity / (1.0 - opacity)))),
                sh=_f32(np.zeros((K, 3, n))), sh_degree=sh_degree)


def decoder_mlp(seed=5, in_dim=35, hidden=32, head_out=(10, 30, 70), bias_scale=1.0):
    """Weights of the three decoder heads, drawn like a default linear-layer
    initialisation: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    (biases scaled by `bias_scale`). Layout: w1[3 hidden, in_dim] (head h at
    rows h*hidden ..), b1[3 hidden], w2[sum(head_out), hidden], b2[sum]."""
    rng = np.random.default_rng(seed)
    nh = len(head_out)
    b_in, b_hid = 1.0 / math.sqrt(in_dim), 1.0 / math.sqrt(hidden)
    w1 = rng.uniform(-b_in, b_in, (nh * hidden, in_dim))
    b1 = rng.uniform(-b_in, b_in, nh * hidden) * bias_scale
    w2 = rng.uniform(-b_hid, b_hid, (sum(head_out), hidden))
    b2 = rng.uniform(-b_hid, b_hid, sum(head_out)) * bias_scale
    return dict(w1=_f32(w1), b1=_f32(b1), w2=_f32(w2), b2=_f32(b2))
