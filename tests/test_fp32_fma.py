"""Pins of the FP32 device-rule model (tests/fp32_fma.py) on the CPU.

fma32 must be the correctly rounded float32 fused multiply-add: checked
against exact rational arithmetic (Python fractions, rounded to the nearest
float32, ties to even) on random operands and on a crafted operand triple
whose FP64 sum lands on an FP32 midpoint (where rounding twice is wrong).
step32 in FP64-exact settings reduces to the oracle's update: with every
operand a small integer multiple of a power of two, no rounding happens and
the FP32 step equals the FP64 oracle step exactly.
"""

import math
from fractions import Fraction

import numpy as np

import oracle
from tests import fp32_fma


def round_f32(x: Fraction) -> np.float32:
    """Nearest float32 to an exact rational (ties to even); finite normal range only."""
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    # fix e so that 2^e <= a < 2^(e+1)
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = a / Fraction(2) ** (e - 23)        # in [2^23, 2^24)
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return np.float32(sign * float(Fraction(n) * Fraction(2) ** (e - 23)))


def exact_fma(c, d, f):
    return round_f32(Fraction(float(c)) * Fraction(float(d)) + Fraction(float(f)))


def test_fma32_matches_exact_rounding_on_random_operands():
    rng = np.random.default_rng(7)
    n = 4000
    c = rng.uniform(0.1, 0.6, n).astype(np.float32)
    d = (rng.standard_normal(n) * np.exp2(rng.integers(-12, 3, n))).astype(np.float32)
    f = rng.uniform(-2, 2, n).astype(np.float32)
    got = fp32_fma.fma32(c, d, f)
    ref = np.array([exact_fma(*t) for t in zip(c, d, f)], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # the model differs from the separately rounded c * d + f somewhere (it is a real FMA)
    assert np.any(got != (c * d + f))


def test_fma32_corrects_double_rounding():
    # c d = 2^-24 (1 + 2^-18)(1 - 2^-18) = 2^-24 - 2^-60, f = 1 + 2^-23: the exact sum lies just
    # below the midpoint 1 + 2^-23 + 2^-24, its FP64 rounding lies on it, and nearest-even from
    # there would give 1 + 2^-22; the correct FP32 result is 1 + 2^-23.
    c = np.float32(2.0 ** -24 * (1 + 2.0 ** -18))
    d = np.float32(1 - 2.0 ** -18)
    f = np.float32(1 + 2.0 ** -23)
    s64 = float(c) * float(d) + float(f)
    assert np.float32(s64) == np.float32(1 + 2.0 ** -22)   # what rounding twice gives
    assert exact_fma(c, d, f) == np.float32(1 + 2.0 ** -23)
    assert fp32_fma.fma32(c, d, f) == np.float32(1 + 2.0 ** -23)
    # and just above a midpoint whose even neighbour is below: c d = -(2^-24 - 2^-60),
    # f = 1 + 2^-23, exact sum 1 + 2^-24 + 2^-60, FP64 sum 1 + 2^-24 (nearest even: 1.0);
    # the correct FP32 result rounds up to 1 + 2^-23
    c2 = np.float32(-(2.0 ** -24) * (1 + 2.0 ** -18))
    d2 = np.float32(1 - 2.0 ** -18)
    f2 = np.float32(1 + 2.0 ** -23)
    assert np.float32(float(c2) * float(d2) + float(f2)) == np.float32(1.0)
    assert exact_fma(c2, d2, f2) == np.float32(1 + 2.0 ** -23)
    assert fp32_fma.fma32(c2, d2, f2) == np.float32(1 + 2.0 ** -23)
    f3 = np.float32(1 + 2.0 ** -23)
    c3 = np.float32(2.0 ** -24 * (1 + 2.0 ** -18))
    d3 = np.float32(1 + 2.0 ** -18)                   # c d = 2^-24 + 2^-41 + 2^-60: no midpoint
    assert fp32_fma.fma32(c3, d3, f3) == exact_fma(c3, d3, f3)


def test_step32_equals_the_oracle_when_nothing_rounds(oracle_mod):
    # fields are multiples of 2^-4 in [-4, 4] and the coefficients 2^-2: every difference,
    # product and sum of four steps is exact in FP32 (checked: the FP64 result is FP32
    # representable), so the FP32 model and the FP64 oracle must agree bit for bit (a wrong
    # index, sign or operand order would show)
    nx, ny, nz = 7, 6, 5
    rng = np.random.default_rng(3)
    shapes = oracle.shapes(nx, ny, nz)
    init = [rng.integers(-64, 65, shp).astype(np.float64) / 16 for shp in shapes.values()]
    ref = oracle.make_state(init[:3], init[3:])
    ce = oracle.coef_e(nx, ny, nz, 1.0, 0.25)
    ch = oracle.coef_h(nx, ny, nz, 1.0, 0.25)
    got = [a.astype(np.float32) for a in ref]
    steps = 4
    oracle.run(ref, ce, ch, steps)
    assert all(np.array_equal(r.astype(np.float32).astype(np.float64), r) for r in ref)
    ce32 = [a.astype(np.float32) for a in ce]
    ch32 = [a.astype(np.float32) for a in ch]
    for _ in range(steps):
        fp32_fma.step32(got, ce32, ch32)
    for g, r in zip(got, ref):
        assert np.array_equal(g.astype(np.float64), r)
