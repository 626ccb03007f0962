"""The per-splat band of the skip decision (Sec. 2.1, Eq. 1: a pixel skips
a splat when Q > t). The forward and backward evaluate Q in FP32 in the
order dx * (a dx + 2 b dy) + (c dy) dy and decide from its sign against t
unless |q32 - t| is within the splat's band, where FP64 decides. The band is
1e-6 (sqrt(ac) + |b|)^2 / (ac - b^2) t, from the first-order bound
|q32 - Q| <= 5 u (1 + r) / (1 - r) Q, r = |b| / sqrt(ac), u = 2^-24.

These host tests restate that arithmetic in numpy (FP32 steps, the fused
multiply-adds rounded once from their exact FP64 value) and check, over
random conics up to a 10^4 eigenvalue ratio with pixel centres placed next
to the Q = t ellipse: the error never exceeds the first-order bound, and no
FP32 decision taken outside the band differs from the FP64 one."""
import numpy as np

F32 = np.float32
U = 2.0 ** -24


def _fma32(a, b, c):
    # a * b is exact in FP64 for FP32 operands; one rounding of the sum to FP32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _band(a, b, c, t):
    ac = a.astype(np.float64) * c.astype(np.float64)
    det = ac - b.astype(np.float64) ** 2
    with np.errstate(divide='ignore', invalid='ignore'):  # masked below
        sac = np.sqrt(ac.astype(F32))
        bb = np.abs(b)
        num = ((sac + bb) * (sac + bb)).astype(F32)
        band = ((F32(1e-6) * (num / det.astype(F32))).astype(F32) * t).astype(F32)
    ok = (a > 0) & (det > 0) & (t > 1e-20) & (ac > 1e-30) & (ac < 1e30)
    return np.where(ok, band, np.inf).astype(F32), ok


def _case(seed, n=400_000, log_std=(-1.0, 3.6)):
    rng = np.random.default_rng(seed)
    s1 = np.exp(rng.uniform(*log_std, n))
    s2 = np.exp(rng.uniform(*log_std, n))
    th = rng.uniform(0, np.pi, n)
    cs, sn = np.cos(th), np.sin(th)
    a = (cs ** 2 / s1 ** 2 + sn ** 2 / s2 ** 2).astype(F32)
    c = (sn ** 2 / s1 ** 2 + cs ** 2 / s2 ** 2).astype(F32)
    b = (cs * sn * (1 / s1 ** 2 - 1 / s2 ** 2)).astype(F32)
    u = rng.uniform(0, 1600, n).astype(F32)
    v = rng.uniform(0, 1066, n).astype(F32)
    t = rng.uniform(0.01, 11.0, n).astype(F32)
    ad, bd, cd = (x.astype(np.float64) for x in (a, b, c))
    phi = rng.uniform(0, 2 * np.pi, n)
    ex, ey = np.cos(phi), np.sin(phi)
    qd = np.maximum(ad * ex ** 2 + 2 * bd * ex * ey + cd * ey ** 2, 1e-300)
    rad = np.sqrt(t / qd) * rng.uniform(0.999, 1.001, n)
    px = (np.floor(u + rad * ex) + 0.5).astype(F32)
    py = (np.floor(v + rad * ey) + 0.5).astype(F32)
    dx = (px - u).astype(F32)
    dy = (py - v).astype(F32)
    s1_ = (a * dx).astype(F32)
    td = ((c * dy).astype(F32) * dy).astype(F32)
    q32 = _fma32(dx, _fma32((b + b).astype(F32), dy, s1_), td)
    Dx = px.astype(np.float64) - u.astype(np.float64)
    Dy = py.astype(np.float64) - v.astype(np.float64)
    Q = Dx * (ad * Dx + 2.0 * (bd * Dy)) + Dy * (cd * Dy)
    return dict(a=a, b=b, c=c, t=t, q32=q32, Q=Q)


def test_fp32_error_within_first_order_bound():
    for seed in range(3):
        k = _case(seed)
        ad, bd, cd = (k[x].astype(np.float64) for x in 'abc')
        pd = (ad > 0) & (ad * cd - bd * bd > 0) & (k['Q'] > 0)
        r = np.abs(bd) / np.sqrt(ad * cd)
        bound = 5 * U * (1 + r) / (1 - r) * k['Q']
        err = np.abs(k['q32'].astype(np.float64) - k['Q'])
        assert pd.mean() > 0.99
        assert np.all(err[pd] <= bound[pd]), float(np.max(err[pd] / bound[pd]))


def test_decisions_outside_band_equal_fp64():
    inside = 0
    for seed in range(3, 6):
        k = _case(seed)
        band, ok = _band(k['a'], k['b'], k['c'], k['t'])
        assert ok.mean() > 0.99
        diff = (k['q32'] - k['t']).astype(F32)
        outside = np.abs(diff) > band
        fp64_skip = k['Q'] > k['t'].astype(np.float64)
        assert np.array_equal((diff > 0)[outside], fp64_skip[outside])
        inside += int((~outside).sum())
    # the samples sit within 0.1% of the ellipse: some fall inside the band
    assert inside > 0


def test_band_degenerate_conics_always_fp64():
    a = np.array([1.0, -1.0, 1.0, 1.0, 1e-20], F32)
    b = np.array([1.0, 0.0, 0.0, 0.0, 0.0], F32)  # ac = b^2; negative a; ...
    c = np.array([1.0, -1.0, 1.0, 1.0, 1e-20], F32)
    t = np.array([1.0, 1.0, -1.0, 0.0, 1.0], F32)  # ...; t < 0; t = 0; ac < 1e-30
    band, ok = _band(a, b, c, t)
    assert not ok.any() and np.all(np.isinf(band))
