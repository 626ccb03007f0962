"""The tile walk's quotients (Sec. 2.1, Eq. 1-2) are computed without a
division per column: a quotient by the tile size is a product with its
exact reciprocal, and x / c comes from rc = RN(1 / c) as q = RN(x rc),
r = x - c q (exact, one FMA), RN(q + r rc). These tests pin that arithmetic
with exact rational arithmetic on the CPU: the remainder is representable,
the result equals the correctly rounded quotient, for random operands over
the exponent range the walk can meet, for operands whose quotient lies next
to a rounding midpoint, and for divisors with all-ones significands."""
import math
import random
from fractions import Fraction

import numpy as np


def _rn(fr):
    """Round a rational to the nearest double (ties to even)."""
    return float(fr)  # int / int true division in CPython rounds correctly


def _fast_quotient(x, c):
    rc = 1.0 / c
    q = x * rc
    r_exact = Fraction(x) - Fraction(c) * Fraction(q)
    r = _rn(r_exact)
    assert Fraction(r) == r_exact, (x, c)  # the FMA remainder is exact
    return _rn(Fraction(q) + Fraction(r) * Fraction(rc))


def _f32(v):
    return float(np.float32(v))


def test_random_operands_over_the_walk_range():
    rng = random.Random(7)
    for _ in range(20000):
        # c: an FP32 value (a record field), numerators over +-2^-500..2^400
        c = _f32(rng.uniform(1.0, 2.0) * 2.0 ** rng.randint(-149, 127))
        if c == 0.0:
            continue
        c = -c if rng.random() < 0.5 else c
        x = rng.uniform(1.0, 2.0) * 2.0 ** rng.randint(-500, 400)
        x = -x if rng.random() < 0.5 else x
        assert _fast_quotient(x, c) == x / c, (x, c)


def test_quotients_next_to_rounding_midpoints():
    rng = random.Random(11)
    n = 0
    for _ in range(20000):
        c = _f32(rng.uniform(1.0, 2.0) * 2.0 ** rng.randint(-60, 60))
        q0 = rng.uniform(1.0, 2.0) * 2.0 ** rng.randint(-200, 200)
        mid = Fraction(q0) + Fraction(math.ulp(q0)) / 2
        x = _rn(Fraction(c) * mid)  # x / c within a few ulp of the midpoint
        for xx in (x, math.nextafter(x, math.inf), math.nextafter(x, -math.inf)):
            assert _fast_quotient(xx, c) == xx / c, (xx, c)
            n += 1
    assert n == 60000


def test_all_ones_divisors_and_exact_quotients():
    rng = random.Random(13)
    ones = [_f32((2.0 - 2.0 ** -23) * 2.0 ** e) for e in range(-100, 100)]
    for c in ones + [1.0, 3.0, _f32(1.0 / 3.0), 1.5, 0.75]:
        for _ in range(100):
            x = rng.uniform(-1e6, 1e6)
            assert _fast_quotient(x, c) == x / c, (x, c)
            k = float(rng.randint(-2 ** 20, 2 ** 20))
            assert _fast_quotient(k * c, c) == (k * c) / c, (k, c)  # exact quotients


def test_tile_reciprocal_products_equal_quotients():
    rng = random.Random(17)
    for T in (8.0, 16.0, 32.0):
        rT = math.ldexp(1.0, -int(math.log2(T)))
        assert rT * T == 1.0
        for _ in range(20000):
            x = rng.uniform(-1.0, 1.0) * 2.0 ** rng.randint(-1074, 1000)
            assert x * rT == x / T, (x, T)
        for x in (0.0, -0.0, 5e-324, -5e-324, 2.0 ** -1022, 1.7976931348623157e308):
            assert math.copysign(1.0, x * rT) == math.copysign(1.0, x / T)
            assert x * rT == x / T
