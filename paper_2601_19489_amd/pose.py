"""Global pose refinement (Sec. 2.5): a correction {Delta R,
Delta t} per training camera, refined by gradient. Each training step adds
the view's camera gradient (gs_pose_grad, from the image-space gradients
the backward left in grad2d) to a per-view device accumulator; every
`every` steps the accumulated gradients are applied with one Adam step per
view on (omega, delta) and the cameras are updated:
R <- exp([omega]x) R, t <- exp([omega]x) t + delta.

The six numbers per view live on the host between applications; updating
a camera is host bookkeeping on a 3 x 3 matrix.
"""
from __future__ import annotations

import copy
import math
from typing import Sequence

import numpy as np
import torch

from . import _lib


def rotation_from_vector(w) -> np.ndarray:
    """exp([w]x) (Rodrigues)."""
    w = np.asarray(w, np.float64)
    th = math.sqrt(float(w @ w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + (math.sin(th) / th) * K + ((1.0 - math.cos(th)) / (th * th)) * (K @ K)


def corrected(cam, omega, delta):
    """Copy of `cam` with the left correction applied."""
    Q = rotation_from_vector(omega)
    c = copy.copy(cam)
    c.R = Q @ np.asarray(cam.R, np.float64).reshape(3, 3)
    c.t = Q @ np.asarray(cam.t, np.float64).reshape(3) + np.asarray(delta, np.float64)
    return c


class PoseRefiner:
    def __init__(self, cams: Sequence, lr_rot=2e-4, lr_trans=5e-4, every=300,
                 betas=(0.9, 0.999), eps=1e-12, device='cuda'):
        self.cams = [copy.copy(c) for c in cams]
        self.every = int(every)
        self.lr = np.array([lr_rot] * 3 + [lr_trans] * 3)
        self.b1, self.b2 = betas
        self.eps = eps
        V = len(cams)
        self.acc = torch.zeros((V, 6), dtype=torch.float64, device=device)
        self.m = np.zeros((V, 6))
        self.v = np.zeros((V, 6))
        self.t = np.zeros(V, np.int64)

    def camera(self, v) -> _lib.GsCamera:
        return _lib.camera(self.cams[v])

    def accumulate(self, v, g: _lib.GsGaussians, n, sh_degree, grad2d, stream=None):
        """Add view v's camera gradient (grad2d from this step's backward)."""
        _lib.gs_pose_grad(g, n, sh_degree, self.camera(v), grad2d, self.acc[v], stream)

    def step(self, s):
        """Apply the accumulated gradients every `every` steps."""
        if self.every > 0 and s % self.every == 0:
            self.apply()

    def apply(self):
        grads = self.acc.cpu().numpy()
        for v in range(len(self.cams)):
            g = grads[v]
            if not np.any(g):
                continue
            self.t[v] += 1
            self.m[v] = self.b1 * self.m[v] + (1 - self.b1) * g
            self.v[v] = self.b2 * self.v[v] + (1 - self.b2) * g * g
            mh = self.m[v] / (1 - self.b1 ** self.t[v])
            vh = self.v[v] / (1 - self.b2 ** self.t[v])
            upd = -self.lr * mh / (np.sqrt(vh) + self.eps)
            self.cams[v] = corrected(self.cams[v], upd[:3], upd[3:])
        self.acc.zero_()
