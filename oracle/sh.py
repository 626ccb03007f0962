"""Real spherical harmonics up to degree 3, FP64 (oracle).

The paper inherits view-dependent colour from the 3DGS formulation it builds
on (Sec. 2.1 names the GS-like methods it follows). Colour is
rgb = max(0, sum_lm k_lm * Y_lm(dir) + 0.5) with dir the unit vector from
the camera centre to the Gaussian mean.

Basis: orthonormal real SH on the unit sphere written as Cartesian
polynomials of the unit vector (x, y, z), ordered m = -l..l within degree l
(coefficient index l*l + l + m), times the sign (-1)^m (Condon-Shortley
phase). The constants are the textbook normalisations, e.g.
Y_00 = 1/(2 sqrt(pi)), Y_1m = sqrt(3/(4 pi)) * (y, z, x).
"""
from __future__ import annotations

import math

import numpy as np

_S = math.sqrt
_PI = math.pi


def _basis_terms(x, y, z):
    """List of (Y_lm values) for l <= 3, each an array like x (no sign)."""
    xx, yy, zz = x * x, y * y, z * z
    return [
        # l = 0
        0.5 * _S(1.0 / _PI) * np.ones_like(x),
        # l = 1: m = -1, 0, 1
        _S(3.0 / (4.0 * _PI)) * y,
        _S(3.0 / (4.0 * _PI)) * z,
        _S(3.0 / (4.0 * _PI)) * x,
        # l = 2: m = -2 .. 2
        0.5 * _S(15.0 / _PI) * x * y,
        0.5 * _S(15.0 / _PI) * y * z,
        0.25 * _S(5.0 / _PI) * (2.0 * zz - xx - yy),
        0.5 * _S(15.0 / _PI) * x * z,
        0.25 * _S(15.0 / _PI) * (xx - yy),
        # l = 3: m = -3 .. 3
        0.25 * _S(35.0 / (2.0 * _PI)) * y * (3.0 * xx - yy),
        0.5 * _S(105.0 / _PI) * x * y * z,
        0.25 * _S(21.0 / (2.0 * _PI)) * y * (4.0 * zz - xx - yy),
        0.25 * _S(7.0 / _PI) * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
        0.25 * _S(21.0 / (2.0 * _PI)) * x * (4.0 * zz - xx - yy),
        0.25 * _S(105.0 / _PI) * z * (xx - yy),
        0.25 * _S(35.0 / (2.0 * _PI)) * x * (xx - 3.0 * yy),
    ]


def _m_of(k):
    l = int(math.isqrt(k))
    return k - l * l - l


def basis(dirs, degree):
    """Y[k, ...] for k < (degree+1)^2 at unit vectors dirs[3, ...]."""
    x, y, z = dirs
    terms = _basis_terms(x, y, z)
    K = (degree + 1) ** 2
    return np.stack([(-1.0) ** _m_of(k) * terms[k] for k in range(K)])


def basis_grad(dirs, degree, eps=None):
    """dY[k, 3, ...]: gradient of each polynomial w.r.t. (x, y, z).

    Written out by differentiating the polynomials above term by term.
    """
    x, y, z = dirs
    o = np.zeros_like(x)
    one = np.ones_like(x)
    xx, yy, zz = x * x, y * y, z * z
    c1 = _S(3.0 / (4.0 * _PI))
    a2 = 0.5 * _S(15.0 / _PI)
    b2 = 0.25 * _S(5.0 / _PI)
    d2 = 0.25 * _S(15.0 / _PI)
    a3 = 0.25 * _S(35.0 / (2.0 * _PI))
    b3 = 0.5 * _S(105.0 / _PI)
    c3 = 0.25 * _S(21.0 / (2.0 * _PI))
    e3 = 0.25 * _S(7.0 / _PI)
    f3 = 0.25 * _S(105.0 / _PI)
    g = [
        (o, o, o),
        (o, c1 * one, o),
        (o, o, c1 * one),
        (c1 * one, o, o),
        (a2 * y, a2 * x, o),
        (o, a2 * z, a2 * y),
        (b2 * (-2.0 * x), b2 * (-2.0 * y), b2 * (4.0 * z)),
        (a2 * z, o, a2 * x),
        (d2 * (2.0 * x), d2 * (-2.0 * y), o),
        (a3 * (6.0 * x * y), a3 * (3.0 * xx - 3.0 * yy), o),
        (b3 * y * z, b3 * x * z, b3 * x * y),
        (c3 * (-2.0 * x * y), c3 * (4.0 * zz - xx - 3.0 * yy), c3 * (8.0 * y * z)),
        (e3 * (-6.0 * x * z), e3 * (-6.0 * y * z), e3 * (6.0 * zz - 3.0 * xx - 3.0 * yy)),
        (c3 * (4.0 * zz - 3.0 * xx - yy), c3 * (-2.0 * x * y), c3 * (8.0 * x * z)),
        (f3 * (2.0 * x * z), f3 * (-2.0 * y * z), f3 * (xx - yy)),
        (a3 * (3.0 * xx - 3.0 * yy), a3 * (-6.0 * x * y), o),
    ]
    K = (degree + 1) ** 2
    return np.stack([(-1.0) ** _m_of(k) * np.stack(g[k]) for k in range(K)])
