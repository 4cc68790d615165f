"""The series logarithm of the pair moments (gd_physics.hpp, log_s and
log1p_s), its steps evaluated on the host: ln y = e ln 2 + 2 atanh(s) with
y = m 2^e, m in [1/sqrt 2, sqrt 2), s = (m - 1)/(m + 1), the atanh series to
s^18/19 in Horner form with fused multiply-adds, and ln(1 + x) = ln u +
(x - (u - 1))/u for u = 1 + x rounded.  Checked against the library log1p
within 3 ulp over the ranges the moments meet: x = N_coll psi > 0 (sticking)
from 1e-20 to 1e30, and -0.1 <= x < 0 (erosion remnants)."""
import math
from fractions import Fraction

import numpy as np


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _log_s(y):
    m, e = math.frexp(y)
    if m < 0.70710678118654752:
        m, e = m + m, e - 1
    f = m - 1.0
    s = f / (2.0 + f)
    s2 = s * s
    p = 1.0 / 19.0
    for k in (17, 15, 13, 11, 9, 7, 5, 3):
        p = _fma(p, s2, 1.0 / k)
    p = _fma(p, s2, 1.0)
    return _fma(float(e), 0.69314718055994530942, (s + s) * p)


def _log1p_s(x):
    u = 1.0 + x
    if u == 1.0:
        return x
    return _log_s(u) + (x - (u - 1.0)) / u


def _ulps(got, want):
    return abs(got - want) / math.ulp(want)


def test_series_log1p_within_3_ulp():
    rng = np.random.default_rng(3)
    xs = list(10.0 ** rng.uniform(-20, 30, 4000)) + list(-0.1 * rng.uniform(1e-9, 1.0, 2000)) + [1.0, 0.5, 1e-6]
    worst = max(_ulps(_log1p_s(float(x)), math.log1p(float(x))) for x in xs)
    assert worst <= 3.0, worst


def test_series_log_within_3_ulp():
    rng = np.random.default_rng(4)
    ys = list(10.0 ** rng.uniform(-30, 30, 4000)) + [1.0 - 2.0 ** -52, 1.0 + 2.0 ** -52, 0.7071067811865475, 1.4142135623730951]
    worst = max(_ulps(_log_s(float(y)), math.log(float(y))) for y in ys if math.log(float(y)) != 0.0)
    assert worst <= 3.0, worst
    assert _log_s(1.0) == 0.0
