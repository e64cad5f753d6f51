"""The FP64 division shortcuts of the stage kernels give IEEE quotients.

Two places in the kernels replace a division by something that must equal
it bit for bit (the oracle divides plainly):
  * divide(): the hardware's double division sequence without its operand
    scaling and special-value fix-up -- the hardware reciprocal r0 of y, two
    Newton steps r += r (1 - y r), q = x r, one residual correction
    q += r (x - y q), every step a fused multiply-add -- used where y and x
    lie in the checked range of the WENO-IS weights (and of the cut-off
    weights' share test), sharing one reciprocal among the quotients by the
    same denominator;
  * star_zeros(): the signed zero 0 * (num / den) of eq. (14)'s discarded
    star state, formed as (0 * num) * den without the division.
With the hardware reciprocal, divide() runs the very instructions of the
hardware division except the scaling (v_div_scale) and the fix-up
(v_div_fixup), so it returns the hardware quotient whenever those two are
identities.  Checked here without a GPU:
  * the stated ranges lie where the documented scaling conditions of
    v_div_scale_f64 never hold and the fix-up returns its input;
  * replayed with exact rounding from the correctly rounded reciprocal, the
    sequence gives the correctly rounded quotient across those ranges
    (including all-ones mantissas, where a reciprocal one unit off makes the
    Newton steps stall -- the hardware reciprocal is what avoids that, and
    the GPU parity tests compare the resulting quotients with the oracle's);
  * the signed-zero rule of star_zeros().
"""
import math
import random
from fractions import Fraction

import pytest


def _rn(v: Fraction) -> float:
    return float(v)  # int / int true division: correctly rounded, ties to even


def _fma(a, b, c):
    return _rn(Fraction(a) * Fraction(b) + Fraction(c))


def _mul(a, b):
    return _rn(Fraction(a) * Fraction(b))


def _sequence(x, y, delta):
    r = _rn(Fraction(1) / Fraction(y) * (1 + Fraction(delta)))
    e = _fma(-y, r, 1.0)
    r = _fma(r, e, r)
    e = _fma(-y, r, 1.0)
    r = _fma(r, e, r)
    q = _mul(x, r)
    rem = _fma(-y, q, x)
    return _fma(rem, r, q)


def _rand(rs, lo_exp, hi_exp):
    m = rs.uniform(1.0, 2.0)
    return math.copysign(math.ldexp(m, rs.randint(lo_exp, hi_exp)), rs.choice((-1.0, 1.0)))


def _biased_exp(v):
    return 0 if v == 0.0 else max(0, math.frexp(abs(v))[1] + 1022)


def _div_scale_acts(x, y):
    """The conditions under which v_div_scale_f64 scales an operand (or
    returns NaN), as the CDNA instruction set documents them: a zero
    operand; numerator and denominator exponents 768 or more apart; a
    denormal denominator, reciprocal or quotient; a numerator exponent at
    most 53 (biased)."""
    if x == 0.0 or y == 0.0:
        return True
    tiny = 2.0 ** -1022
    return (_biased_exp(x) - _biased_exp(y) >= 768 or abs(y) < tiny or 1.0 / abs(y) < tiny
            or abs(x / y) < tiny or _biased_exp(x) <= 53)


def _cases(rs):
    cases = []
    # generic operands: y in [2^-100, 2^100], x in [2^-600, 2^600]
    for _ in range(600):
        cases.append((_rand(rs, -600, 599), _rand(rs, -100, 99)))
    for ex in (-600, 599):
        for ey in (-100, 99):
            for mx in (1.0, 2.0 - 2.0 ** -52):
                for my in (1.0, 2.0 - 2.0 ** -52):
                    cases.append((math.ldexp(mx, ex), math.ldexp(my, ey)))
    # WENO-IS weights, in the range the kernel checks (epsilon in
    # [2^-200, 2^100], indicators summing to at most 2^200, tau zero or at
    # least 2^-700): tau / (beta + eps) with tau in [2^-700, 2^200] and
    # beta + eps in [2^-200, 2^201]; then alpha_k / sum(alpha) with
    # alpha_k = d_k (1 + ratios) in [0.1, 2^801] and alpha_k <= sum
    for _ in range(300):
        cases.append((abs(_rand(rs, -700, 199)), abs(_rand(rs, -200, 200))))
    for _ in range(300):
        s = abs(_rand(rs, -4, 800))
        a = s * rs.uniform(0.0, 1.0)
        if a >= 0.1:
            cases.append((a, s))
    # cut-off weights' share test in the same checked range: the shares
    # t_k = g_k / g_max with 1 <= g_k <= g_max <= 2^801 (g = 1 + ratios),
    # among them t = 1 exactly
    for _ in range(300):
        gm = abs(_rand(rs, 0, 800))
        g = max(1.0, gm * rs.uniform(0.0, 1.0))
        cases.append((g, gm))
    for gm in (1.0, math.ldexp(2.0 - 2.0 ** -52, 800), math.ldexp(1.0, 800), 3.0):
        cases += [(gm, gm), (1.0, gm)]
    # reciprocals with all-ones or power-of-two mantissas, quotients next to
    # a power of two
    for e in (-100, -37, 0, 51, 99):
        for y in (math.ldexp(2.0 - 2.0 ** -52, e), math.ldexp(1.0, e),
                  math.ldexp(1.0 + 2.0 ** -52, e)):
            for x in (y, -y, math.nextafter(y, 0.0), math.nextafter(y, math.inf),
                      math.ldexp(3.0, 17), _rand(rs, -600, 599)):
                cases.append((x, y))
    return cases


def test_stated_ranges_need_no_operand_scaling():
    rs = random.Random(1707)
    for x, y in _cases(rs):
        assert not _div_scale_acts(x, y), (x, y)
    # and the range tests are tight enough to exclude the scaling cases
    assert _div_scale_acts(2.0 ** -1000, 1.0) and _div_scale_acts(2.0 ** 800, 2.0 ** -100)
    assert _div_scale_acts(1.0, 2.0 ** 1023)


def test_unscaled_sequence_is_correctly_rounded():
    rs = random.Random(11)
    for x, y in _cases(rs):
        want = x / y
        got = _sequence(x, y, 0.0)
        assert got == want and math.copysign(1, got) == math.copysign(1, want), (x, y)


def test_signed_zero_of_a_discarded_star_state():
    rs = random.Random(3)
    vals = [0.0, -0.0, 1.0, -1.0, 1e-300, -1e300, 5e-324, -5e-324]
    vals += [_rand(rs, -900, 900) for _ in range(40)]
    for num in vals:
        for den in vals:
            if den == 0.0:
                continue
            q = num / den
            if math.isinf(q):
                continue  # 0 * inf is NaN: outside the finite states the kernels see
            a = 0.0 * q
            b = (0.0 * num) * den
            assert a == 0.0 and b == 0.0
            assert math.copysign(1, a) == math.copysign(1, b), (num, den)
