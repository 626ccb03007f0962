"""Per-Gaussian backward from the 2D splat gradients to the 3D parameters,
FP64 (oracle).

Sec. 2.2: the preprocess step back-propagates per Gaussian. This is the
plain chain rule of the forward in preprocess.py, written in matrix form:
    conic C_hat = Sigma'^-1:      G_Sigma' = -C_hat G_Chat C_hat, where
                                  G_Chat = [[g_a, g_b/2], [g_b/2, g_c]]
    Sigma' = T Sigma T^T + 0.3 I: G_T = (G + G^T) T Sigma, G_Sigma = T^T G T
    T = J W:                      G_J = G_T W^T
    J(p) with the x/z, y/z clamp (zero derivative through an active clamp)
    (u, v) = f p_xy / p_z + c;    dval = p_z (or 1 / p_z, inverse-depth camera);  p = W mu + t
    Sigma = M M^T:                G_M = (G_Sigma + G_Sigma^T) M
    M = R S:                      G_R = G_M S, G_s = diag(R^T G_M) * exp(s)
    R(q_hat), q_hat = q/|q|:      G_q = (G_qhat - q_hat (q_hat . G_qhat)) / |q|
    o = sigmoid(omega):           G_omega = G_o o (1 - o)
    rgb = max(0, sum_k sh_k Y_k(dir) + 0.5): zero where the clamp is active
    (raw value < 0); G_sh_k = G_rgb Y_k; G_mu += P(dir) G_dir / |mu - campos|
The thresholds (near cull, tile sets, alpha skip, early stop) are held fixed.
In direct mode (attributes already activated) the last three steps are the
identity: G_scale, G_opacity and G_rgb are returned as they are, and the
colour does not depend on the mean.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh


def _dR_dq(q):
    """dR[N, 3, 3, 4]: derivative of R(q) entries w.r.t. (w, x, y, z)."""
    w, x, y, z = q
    N = q.shape[1]
    d = np.zeros((N, 3, 3, 4))
    # R00 = 1 - 2(y^2 + z^2)
    d[:, 0, 0, 2] = -4 * y; d[:, 0, 0, 3] = -4 * z
    # R01 = 2(xy - wz)
    d[:, 0, 1, 0] = -2 * z; d[:, 0, 1, 1] = 2 * y; d[:, 0, 1, 2] = 2 * x; d[:, 0, 1, 3] = -2 * w
    # R02 = 2(xz + wy)
    d[:, 0, 2, 0] = 2 * y; d[:, 0, 2, 1] = 2 * z; d[:, 0, 2, 2] = 2 * w; d[:, 0, 2, 3] = 2 * x
    # R10 = 2(xy + wz)
    d[:, 1, 0, 0] = 2 * z; d[:, 1, 0, 1] = 2 * y; d[:, 1, 0, 2] = 2 * x; d[:, 1, 0, 3] = 2 * w
    # R11 = 1 - 2(x^2 + z^2)
    d[:, 1, 1, 1] = -4 * x; d[:, 1, 1, 3] = -4 * z
    # R12 = 2(yz - wx)
    d[:, 1, 2, 0] = -2 * x; d[:, 1, 2, 1] = -2 * w; d[:, 1, 2, 2] = 2 * z; d[:, 1, 2, 3] = 2 * y
    # R20 = 2(xz - wy)
    d[:, 2, 0, 0] = -2 * y; d[:, 2, 0, 1] = 2 * z; d[:, 2, 0, 2] = -2 * w; d[:, 2, 0, 3] = 2 * x
    # R21 = 2(yz + wx)
    d[:, 2, 1, 0] = 2 * x; d[:, 2, 1, 1] = 2 * w; d[:, 2, 1, 2] = 2 * z; d[:, 2, 1, 3] = 2 * y
    # R22 = 1 - 2(x^2 + y^2)
    d[:, 2, 2, 1] = -4 * x; d[:, 2, 2, 2] = -4 * y
    return d


def preprocess_backward(pre, grad2d, sh_degree, cam, intermediates=False):
    """3D parameter gradients from grad2d[10, N] (render.GRAD2D order).

    `pre` is the dict returned by preprocess.preprocess. Returns a dict of
    means[3,N], log_scales[3,N], quats[4,N], opacity_logits[N], sh[K,3,N]
    (FP64). Culled Gaussians get zero gradients. With `intermediates`, also
    returns a second dict: gp[3,N] = dL/dp (camera-space mean, with the
    camera-space covariance and the view direction held fixed), GS2[N,2,2] =
    dL/dSigma' (symmetric) and gdir[3,N] = dL/d(mu - campos) through the view
    direction (zero in direct mode), all zero for culled Gaussians.
    """
    g = np.asarray(grad2d, np.float64)
    vis = pre['visible']
    g = np.where(vis[None], g, 0.0)
    N = g.shape[1]
    W = pre['_W']
    fx, fy = cam.fx, cam.fy
    pz = pre['_pz']
    px, py = pre['_p'][0], pre['_p'][1]
    Sig, T, S2, M, R = pre['_Sigma'], pre['_T'], pre['_S2'], pre['_M'], pre['_R']

    # conic -> Sigma'
    Chat = np.linalg.inv(S2)
    Gc = np.zeros((N, 2, 2))
    Gc[:, 0, 0] = g[2]
    Gc[:, 0, 1] = Gc[:, 1, 0] = 0.5 * g[3]
    Gc[:, 1, 1] = g[4]
    GS2 = -Chat @ Gc @ Chat
    # Sigma' = T Sigma T^T
    GS2s = GS2 + np.transpose(GS2, (0, 2, 1))
    GT = GS2s @ T @ Sig
    GSig = np.transpose(T, (0, 2, 1)) @ GS2 @ T
    # T = J W
    GJ = GT @ W.T
    gp = np.zeros((3, N))
    # J00 = fx/pz, J11 = fy/pz
    gp[2] += GJ[:, 0, 0] * (-fx / pz**2) + GJ[:, 1, 1] * (-fy / pz**2)
    # J02 = -fx xc / pz with xc = clamp(px/pz)
    unx = np.abs(pre['_xr']) <= pre['_limx']
    xc = np.clip(pre['_xr'], -pre['_limx'], pre['_limx'])
    gp[0] += np.where(unx, GJ[:, 0, 2] * (-fx / pz**2), 0.0)
    gp[2] += np.where(unx, GJ[:, 0, 2] * (2.0 * fx * px / pz**3), GJ[:, 0, 2] * (fx * xc / pz**2))
    uny = np.abs(pre['_yr']) <= pre['_limy']
    yc = np.clip(pre['_yr'], -pre['_limy'], pre['_limy'])
    gp[1] += np.where(uny, GJ[:, 1, 2] * (-fy / pz**2), 0.0)
    gp[2] += np.where(uny, GJ[:, 1, 2] * (2.0 * fy * py / pz**3), GJ[:, 1, 2] * (fy * yc / pz**2))
    # (u, v) and depth
    gp[0] += g[0] * fx / pz
    gp[1] += g[1] * fy / pz
    # the blended depth channel carries p_z, or 1 / p_z for an inverse-depth camera
    dval_dpz = -1.0 / pz**2 if pre.get('_inverse', False) else 1.0
    gp[2] += -g[0] * fx * px / pz**2 - g[1] * fy * py / pz**2 + g[9] * dval_dpz
    gmu = W.T @ gp

    # Sigma = M M^T, M = R S
    GM = (GSig + np.transpose(GSig, (0, 2, 1))) @ M
    scale = pre['_scale']
    GR = GM * scale.T[:, None, :]
    Gscale = np.einsum('nij,nij->nj', GM, R).T
    direct = pre['_direct']
    gs = Gscale if direct else Gscale * scale
    dR = _dR_dq(pre['_qn'])
    Gqn = np.einsum('nij,nijk->kn', GR, dR)
    qn = pre['_qn']
    gq = (Gqn - qn * np.sum(qn * Gqn, axis=0)) / pre['_qnorm']

    o = pre['_opacity']
    z = lambda x: np.where(vis, x, 0.0)
    inter = dict(gp=z(gp), GS2=np.where(vis[:, None, None], GS2, 0.0), gdir=np.zeros((3, N)))
    if direct:
        res = dict(means=z(gmu), log_scales=z(gs), quats=z(gq), opacity_logits=z(g[5]),
                   sh=np.where(vis[None, None], g[6:9][None], 0.0))
        return (res, inter) if intermediates else res
    gom = g[5] * o * (1.0 - o)

    # SH colour
    grgb = np.where(pre['_rgb_raw'] < 0.0, 0.0, g[6:9])
    Y = pre['_Y']
    gsh = grgb[None] * Y[:, None, :]
    dY = _sh.basis_grad(pre['_dirs'], sh_degree)           # [K,3(xyz),N]
    gdir = np.einsum('kcn,kdn,cn->dn', pre['_sh'], dY, grgb)
    dirs = pre['_dirs']
    gd = (gdir - dirs * np.sum(dirs * gdir, axis=0)) / pre['_dnorm']
    gmu = gmu + gd
    inter['gdir'] = z(gd)

    res = dict(means=z(gmu), log_scales=z(gs), quats=z(gq), opacity_logits=z(gom),
               sh=np.where(vis[None, None], gsh, 0.0))
    return (res, inter) if intermediates else res
