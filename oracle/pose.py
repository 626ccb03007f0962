"""Camera pose gradient for global pose refinement (Sec. 2.5:
a global correction {Delta R, Delta t} of each camera, refined by gradient
and applied at intervals). Test infrastructure only.

Reading: the correction acts on the world-to-camera transform from the
left, p' = exp([omega]x) p + delta for the camera-space point p = R mu + t,
i.e. R' = exp([omega]x) R and t' = exp([omega]x) t + delta. The gradient at
omega = delta = 0 follows the camera through every quantity the forward
takes from it, holding the tile sets and blend decisions fixed:
  * the camera-space mean: dp'/domega = [omega]x p, dp'/ddelta = I;
  * the camera-space covariance Sigma_c = R Sigma R^T, rotated to
    exp([omega]x) Sigma_c exp([omega]x)^T (delta does not change it);
  * the view direction (mu - campos) = R'^T (p' - t') + ..., which in the
    world frame moves only with delta: d(mu - campos)/ddelta = R^T.
So, summed over the Gaussians,
  dL/ddelta   = sum_i (g_p,i + R g_dir,i)
  dL/domega_k = sum_i (p_i x g_p,i)_k + tr(G_c,i (E_k Sigma_c,i - Sigma_c,i E_k))
with g_p = dL/dp, g_dir = dL/d(mu - campos), G_c = J^T (dL/dSigma') J and
E_k = [e_k]x.
"""
from __future__ import annotations

import numpy as np

from . import backward as _bwd


def skew(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def rodrigues(omega):
    """exp([omega]x) by Rodrigues' formula."""
    omega = np.asarray(omega, np.float64)
    th = float(np.linalg.norm(omega))
    K = skew(omega)
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th**2 * (K @ K)


def apply_pose(cam, omega, delta):
    """A copy of `cam` with R' = exp([omega]x) R, t' = exp([omega]x) t + delta."""
    import copy

    Q = rodrigues(omega)
    c = copy.copy(cam)
    c.R = Q @ np.asarray(cam.R, np.float64).reshape(3, 3)
    c.t = Q @ np.asarray(cam.t, np.float64).reshape(3) + np.asarray(delta, np.float64)
    return c


def pose_gradient(pre, grad2d, sh_degree, cam):
    """dL/d(omega, delta) [6] from the image-space gradients grad2d[10, N]."""
    _, it = _bwd.preprocess_backward(pre, grad2d, sh_degree, cam, intermediates=True)
    gp, GS2, gdir = it['gp'], it['GS2'], it['gdir']
    W = pre['_W']
    p = pre['_p']
    J = pre['_J']                                         # [N, 2, 3]
    Sc = W @ pre['_Sigma'] @ W.T                          # [N, 3, 3] camera-space covariance
    Gc = np.transpose(J, (0, 2, 1)) @ GS2 @ J             # [N, 3, 3]
    d_delta = np.sum(gp + W @ gdir, axis=1)
    d_omega = np.sum(np.cross(p.T, gp.T), axis=0)
    for k in range(3):
        E = skew(np.eye(3)[k])
        d_omega[k] += np.sum(Gc * (E @ Sc - Sc @ E).transpose(0, 2, 1))
    return np.concatenate([d_omega, d_delta])
