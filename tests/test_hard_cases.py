"""The hardest operands of tests/golden/hard_cases.txt (used by the GPU test
of the refined division, reciprocal and square root) are what they claim to
be: their exact results lie within a few units of 2^-106 (relative) of a
rounding midpoint, checked in exact rational arithmetic."""
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def _cases():
    out = []
    with open(os.path.join(HERE, "golden", "hard_cases.txt")) as f:
        for line in f:
            if not line.startswith("#"):
                p = line.split()
                out.append((p[0], [int(x) for x in p[1:]]))
    return out


def _midpoint_distance(z):
    """Distance of a positive rational z from the nearest midpoint of two
    consecutive doubles, relative to z's ulp."""
    e = 0
    while z >= 2:
        z /= 2
        e += 1
    while z < 1:
        z *= 2
        e -= 1
    scaled = z * 2 ** 52                   # significand in units of the ulp
    frac = scaled - (scaled.numerator // scaled.denominator)
    return abs(frac - Fraction(1, 2))


def test_hard_cases_lie_next_to_midpoints():
    cases = _cases()
    kinds = {k for k, _ in cases}
    assert kinds == {"rcp", "div", "sqrt"}
    for kind, v in cases:
        if kind == "rcp":
            assert 2 ** 52 <= v[0] < 2 ** 53
            z = Fraction(2 ** 52, v[0])
            assert _midpoint_distance(z) <= Fraction(12, 2 ** 52), v
        elif kind == "div":
            A, B = v
            assert 2 ** 52 <= A < 2 ** 53 and 2 ** 52 <= B < 2 ** 53
            assert _midpoint_distance(Fraction(A, B)) <= Fraction(6, 2 ** 52), v
        else:
            U = v[0]
            assert 2 ** 52 <= U < 2 ** 54 and (U < 2 ** 53 or U % 2 == 0)
            # sqrt(u) near a midpoint m: compare u with m^2 exactly, where m
            # is the midpoint nearest to the double-precision root
            import math
            s_units = math.isqrt(U * 2 ** 52)            # floor(sqrt(u) 2^52)
            m = Fraction(2 * s_units + 1, 2 ** 53)       # midpoint above floor
            u = Fraction(U, 2 ** 52)
            assert abs(u - m * m) <= Fraction(200, 2 ** 106), v
