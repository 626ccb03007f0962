"""Adam update, FP64 (oracle).

The paper does not name its optimiser; the 3DGS formulation it builds on
trains with Adam (Kingma and Ba 2015). One step t >= 1 with bias correction:
    m = b1 m + (1 - b1) g
    v = b2 v + (1 - b2) g^2
    p = p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
