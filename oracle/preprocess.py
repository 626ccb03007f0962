"""Per-Gaussian preprocess, FP64 (oracle).

Sec. 2.1 of the paper: the preprocess step projects each 3D Gaussian to the
image plane with an approximate affine (EWA) transform, giving a 2D centroid
and covariance, and derives the opacity-aware threshold t = 2 ln(255 o) of
Eq. (1) from which the compact (SnugBox) tile set is built.

Definitions (3DGS image formation model, which the paper builds on):
    S = diag(exp(s)), q_hat = q / |q|, R = R(q_hat), Sigma = (R S)(R S)^T
    o = sigmoid(omega)
    p = W mu + t_cam                           camera-space mean
    culled if p_z <= near
    x' = clamp(p_x / p_z, +-1.3 tan(fov_x / 2)), y' likewise
    J = [[fx / p_z, 0, -fx x' / p_z], [0, fy / p_z, -fy y' / p_z]]
    Sigma' = J W Sigma W^T J^T + 0.3 I          (low-pass dilation)
    conic (a, b, c) = (Sigma'_yy, -Sigma'_xy, Sigma'_xx) / det(Sigma')
    (u, v) = (fx p_x / p_z + cx, fy p_y / p_z + cy)
    z = p_z                                      (the sort depth)
    dval = p_z, or 1 / p_z for an inverse-depth camera (depth_mode 1)
    dir = (mu - campos) / |mu - campos|, campos = -W^T t_cam
    rgb = max(0, sum_k sh_k Y_k(dir) + 0.5)
    t = 2 ln(255 o)                              Eq. (1)

The blended depth channel carries `dval`: the centroid depth (Sec. 3.1,
depth regularisation), or its inverse when the camera asks for disparity
(the paper supervises disparity rather than depth). The sort key stays the
depth in both cases.

Everything is evaluated in FP64; the outputs the rasterizer stores are then
rounded to FP32 (`store`), because tile sets, sort keys and compositing are
defined on the stored record.

Direct mode (sh_degree = DIRECT = -1) takes Gaussians whose attributes are
already activated, as the anchor decoder of Sec. 2.3 produces them: the
scale, opacity and RGB colour are used as given (no exp, no sigmoid, no SH,
no offset or clamp); the projection is unchanged.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh

LOWPASS = 0.3
CLAMP_FOV = 1.3
DIRECT = -1
INVERSE_DEPTH = 1


def depth_mode(cam):
    return int(getattr(cam, 'depth_mode', 0))


def quat_to_rotmat(q):
    """Rotation matrices [N,3,3] from unit quaternions q[4,N] = (w,x,y,z)."""
    w, x, y, z = q
    R = np.empty((q.shape[1], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def camera_arrays(cam):
    W = np.asarray(cam.R, np.float64).reshape(3, 3)
    tc = np.asarray(cam.t, np.float64).reshape(3)
    return W, tc, -W.T @ tc


def preprocess(means, log_scales, quats, opacity_logits, sh, sh_degree, cam,
               store=np.float32):
    """Project N Gaussians. Returns a dict of per-Gaussian arrays.

    Stored outputs (rounded through `store`, returned as float64):
        u, v, a, b, c, opacity, t, depth, rgb[3]
    plus `visible` (not culled by the near plane) and FP64 intermediates
    used by the backward oracle.
    """
    f = np.float64
    mu = np.asarray(means, f)
    s = np.asarray(log_scales, f)
    q = np.asarray(quats, f)
    om = np.asarray(opacity_logits, f)
    direct = sh_degree == DIRECT
    K = 1 if direct else (sh_degree + 1) ** 2
    shc = np.asarray(sh, f).reshape(-1, 3, mu.shape[1])[:K]
    W, tc, campos = camera_arrays(cam)

    scale = s if direct else np.exp(s)
    qnorm = np.sqrt(np.sum(q * q, axis=0))
    qn = q / qnorm
    R = quat_to_rotmat(qn)
    M = R * scale.T[:, None, :]                  # M = R S
    Sigma = M @ np.transpose(M, (0, 2, 1))       # [N,3,3]
    opacity = om if direct else 1.0 / (1.0 + np.exp(-om))

    p = W @ mu + tc[:, None]                     # [3,N]
    px, py, pz = p
    visible = pz > cam.near
    pzs = np.where(visible, pz, 1.0)             # avoid dividing by culled depths
    limx = CLAMP_FOV * (cam.width / (2.0 * cam.fx))
    limy = CLAMP_FOV * (cam.height / (2.0 * cam.fy))
    xr, yr = px / pzs, py / pzs
    xc = np.clip(xr, -limx, limx)
    yc = np.clip(yr, -limy, limy)
    J = np.zeros((mu.shape[1], 2, 3))
    J[:, 0, 0] = cam.fx / pzs
    J[:, 0, 2] = -cam.fx * xc / pzs
    J[:, 1, 1] = cam.fy / pzs
    J[:, 1, 2] = -cam.fy * yc / pzs
    T = J @ W                                    # [N,2,3]
    S2 = T @ Sigma @ np.transpose(T, (0, 2, 1))  # [N,2,2]
    S2[:, 0, 0] += LOWPASS
    S2[:, 1, 1] += LOWPASS
    det = S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] * S2[:, 0, 1]
    visible &= det > 0.0
    dets = np.where(det > 0.0, det, 1.0)
    a = S2[:, 1, 1] / dets
    b = -S2[:, 0, 1] / dets
    c = S2[:, 0, 0] / dets
    u = cam.fx * xr + cam.cx
    v = cam.fy * yr + cam.cy

    d = mu - campos[:, None]
    dnorm = np.sqrt(np.sum(d * d, axis=0))
    dirs = d / dnorm
    if direct:
        Y = np.ones((1, mu.shape[1]))
        rgb_raw = shc[0].copy()
        rgb = rgb_raw
    else:
        Y = _sh.basis(dirs, sh_degree)           # [K,N]
        rgb_raw = np.einsum('kcn,kn->cn', shc, Y) + 0.5
        rgb = np.maximum(rgb_raw, 0.0)
    with np.errstate(divide='ignore'):
        t = 2.0 * np.log(255.0 * opacity)

    def st(x):
        return np.asarray(x, store).astype(f)

    return dict(
        u=st(u), v=st(v), a=st(a), b=st(b), c=st(c), opacity=st(opacity), t=st(t),
        depth=st(pz), dval=st(1.0 / pzs if depth_mode(cam) == INVERSE_DEPTH else pzs),
        rgb=st(rgb), visible=visible,
        # FP64 intermediates for the backward oracle
        _mu=mu, _scale=scale, _q=q, _qnorm=qnorm, _qn=qn, _R=R, _M=M, _Sigma=Sigma,
        _p=p, _pz=pzs, _xr=xr, _yr=yr, _limx=limx, _limy=limy, _J=J, _T=T, _S2=S2,
        _det=dets, _dirs=dirs, _dnorm=dnorm, _Y=Y, _rgb_raw=rgb_raw, _sh=shc,
        _opacity=opacity, _W=W, _direct=direct, _inverse=depth_mode(cam) == INVERSE_DEPTH,
    )


def depth_key(depth_f32):
    """Sort key of a stored depth: the IEEE bits of the FP32 value (positive
    floats order as unsigned integers)."""
    return np.asarray(depth_f32, np.float32).view(np.uint32)
