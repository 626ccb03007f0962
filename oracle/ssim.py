"""Photometric loss of Eq. 5 and the pruning score of Eq. 6 (Sec. 3.2,
final round: multi-view score-guided densification and pruning). Test
infrastructure only.

Eq. 5, per view j: E^j = (1 - lambda) L1^j + lambda (1 - SSIM^j).
Readings (the paper gives neither lambda nor the SSIM details): lambda = 0.2
and the SSIM of 3DGS training: per colour channel, local statistics under an
11 x 11 Gaussian window (sigma 1.5, weights normalised to sum 1) with zero
padding outside the image,
    mu_x = w * x, sigma_x^2 = w * x^2 - mu_x^2, sigma_xy = w * (x y) - mu_x mu_y,
    S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
C1 = 0.01^2, C2 = 0.03^2 (data range 1); SSIM^j = the mean of S over channels
and pixels; L1^j = mean |x - y| over channels and pixels.

Eq. 6: s_i^- = normalize(sum_j sum_{(u,v)} M^j(u,v) E^j), the inner sum over
the masked pixels of view j at which Gaussian i is blended (as for Eq. 4), so
s_i^- = normalize(sum_j E^j count_ij). normalize = min-max over the
Gaussians; Gaussian i is pruned when the normalised score exceeds the
threshold, decided as (s_i - min) > thr (max - min) (no Gaussian is pruned
when max = min).

Everything here is FP64; the window correlation is written out as a sum over
the 121 offsets.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2


def window_1d():
    r = np.arange(WINDOW) - WINDOW // 2
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def _filter(img):
    """Zero-padded correlation of a [H, W] map with the 11 x 11 window."""
    g = window_1d()
    w2 = np.outer(g, g)
    H, W = img.shape
    h = WINDOW // 2
    pad = np.zeros((H + 2 * h, W + 2 * h))
    pad[h:h + H, h:h + W] = img
    out = np.zeros((H, W))
    for dy in range(WINDOW):
        for dx in range(WINDOW):
            out += w2[dy, dx] * pad[dy:dy + H, dx:dx + W]
    return out


def _stats(x, y):
    mx, my = _filter(x), _filter(y)
    sxx, syy, sxy = _filter(x * x), _filter(y * y), _filter(x * y)
    return mx, my, sxx, syy, sxy


def ssim_map(image, target):
    """S per channel and pixel [C, H, W]."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    out = np.empty_like(x)
    for c in range(x.shape[0]):
        mx, my, sxx, syy, sxy = _stats(x[c], y[c])
        vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
        num = (2 * mx * my + C1) * (2 * cxy + C2)
        den = (mx * mx + my * my + C1) * (vx + vy + C2)
        out[c] = num / den
    return out


def ssim(image, target):
    return float(np.mean(ssim_map(image, target)))


def ssim_grad(image, target):
    """d SSIM / d image [C, H, W] (SSIM = mean of the map), by the chain rule
    through the five window statistics: with S = f(mu_x, mu_y, E_xx, E_yy,
    E_xy) and E the raw second moments, dS(p)/dx(q) = w(p - q) [f_mu_x(p) +
    2 x(q) f_E_xx(p) + y(q) f_E_xy(p)], and the sum over p is a second
    zero-padded correlation (the window is symmetric)."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    n = x.size
    g = np.empty_like(x)
    for c in range(x.shape[0]):
        mx, my, sxx, syy, sxy = _stats(x[c], y[c])
        vx, vy, cxy = sxx - mx * mx, syy - my * my, sxy - mx * my
        A1 = 2 * mx * my + C1
        A2 = 2 * cxy + C2
        B1 = mx * mx + my * my + C1
        B2 = vx + vy + C2
        S = A1 * A2 / (B1 * B2)
        # partials of S in (mu_x, var_x, cov_xy), then in the raw moments
        dS_dmx = 2 * my * A2 / (B1 * B2) - 2 * mx * S / B1
        dS_dvx = -S / B2
        dS_dcxy = 2 * A1 / (B1 * B2)
        f_mx = dS_dmx - 2 * mx * dS_dvx - my * dS_dcxy   # through var_x and cov_xy
        f_exx = dS_dvx
        f_exy = dS_dcxy
        g[c] = _filter(f_mx) + 2 * x[c] * _filter(f_exx) + y[c] * _filter(f_exy)
    return g / n


def photo_loss(image, target, lam=LAMBDA):
    """Eq. 5: (E, L1, SSIM)."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    l1 = float(np.mean(np.abs(x - y)))
    s = ssim(x, y)
    return (1 - lam) * l1 + lam * (1 - s), l1, s


def photo_loss_grad(image, target, lam=LAMBDA):
    """dE/dimage: (1 - lambda) sign(x - y) / n - lambda dSSIM/dx."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    return (1 - lam) * np.sign(x - y) / x.size - lam * ssim_grad(x, y)


def prune_score(counts, errors):
    """Eq. 6 before normalisation: sum_j E^j count_ij. counts [K, N] (the
    Eq. 4 counts of each view), errors [K] (E^j)."""
    return np.einsum('kn,k->n', np.asarray(counts, np.float64), np.asarray(errors, np.float64))


def prune_mask(score, threshold):
    """Normalised score above the threshold: (s - min) > thr (max - min)."""
    s = np.asarray(score, np.float64)
    if s.size == 0:
        return np.zeros(0, bool)
    lo, hi = s.min(), s.max()
    return (s - lo) > threshold * (hi - lo)
