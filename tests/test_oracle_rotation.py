"""Pins for the oracle's rotation formulas, eqs. (4.3)-(4.6), Section 4.3.1.

The checks use properties the paper and the mathematics fix, not the
formulas themselves: the 2x2 transformation must diagonalise the pivot Gram
matrix, eq. (2.4), evaluated in exact rational arithmetic; the cot/coth
double-angle identities at the short-cut thresholds; and the mean
departures from (J-)orthogonality of Table B.1 (Appendix B).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table_b1.txt")
EPS = 2.0 ** -53


def _golden_b1():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _offdiag_exact(hpp, hqq, hpq, tn, cs, t):
    """Off-diagonal of Vhat^T Hhat Vhat in exact arithmetic, where Vhat is
    cs [[1, tn], [-tn, 1]] (trig, eq. 4.1) or cs [[1, tn], [tn, 1]]
    (hyperbolic, eq. 4.2)."""
    F = Fraction
    a, b, c = F(hpp), F(hqq), F(hpq)
    tn_, cs_ = F(tn), F(cs)
    v21 = -tn_ if t > 0 else tn_
    # columns of Vhat: (1, v21) and (tn, 1), scaled by cs
    x = (F(1), v21)
    y = (tn_, F(1))
    off = x[0] * (a * y[0] + c * y[1]) + x[1] * (c * y[0] + b * y[1])
    return float(off * cs_ * cs_)


@pytest.mark.parametrize("t", [1, -1])
def test_rotation_diagonalises_pivot_matrix(t):
    """eq. (2.4): the transformation diagonalises the 2x2 pivot matrix."""
    g = np.random.default_rng(11)
    for _ in range(400):
        X = g.standard_normal((8, 2)) * (10.0 ** g.uniform(-3, 3, size=2))
        if t < 0:
            # keep the hyperbolic problem away from |coth 2phi| ~ 1
            X[:, 1] *= 0.3
        hpp, hqq, hpq = float(X[:, 0] @ X[:, 0]), float(X[:, 1] @ X[:, 1]), float(X[:, 0] @ X[:, 1])
        tn, cs, clamped = oracle.rotation(hpp, hqq, hpq, t)
        assert not clamped
        off = _offdiag_exact(hpp, hqq, hpq, tn, cs, t)
        scale = np.sqrt(hpp * hqq) * cs * cs
        assert abs(off) <= 8 * EPS * max(scale, abs(hpq)), (hpp, hqq, hpq, off)


def test_trig_sign_convention():
    """h_pp' = h_pp - tn h_pq for the trigonometric rotation (4.1): the
    larger diagonal element stays larger after the rotation when h_pp >
    h_qq, which pins the direction of the rotation."""
    g = np.random.default_rng(3)
    for _ in range(200):
        hpp, hqq = g.uniform(1, 2), g.uniform(0, 1)
        hpq = g.uniform(-0.4, 0.4) * np.sqrt(hpp * hqq)
        tn, cs, _ = oracle.rotation(hpp, hqq, hpq, 1)
        lam = np.linalg.eigvalsh(np.array([[hpp, hpq], [hpq, hqq]]))
        F = Fraction
        c2 = F(cs) ** 2
        new_pp = c2 * (F(hpp) - 2 * F(tn) * F(hpq) + F(tn) ** 2 * F(hqq))
        assert abs(float(new_pp) - lam[1]) <= 1e-14 * lam[1]


def test_trig_short_cut_small_cot():
    """|cot 2phi| < sqrt(eps): |cot phi| = |cot 2phi| + 1, so tan phi ~ 1
    (a rotation by ~pi/4); the identity cot 2phi = (1 - tan^2)/(2 tan)."""
    hpq = 1.0
    for h in [0.0, 1e-12, -1e-12, 1e-9]:
        hpp = 1.0
        hqq = hpp + h
        tn, cs, _ = oracle.rotation(hpp, hqq, hpq, 1)
        ct2 = (hqq - hpp) / 2.0
        assert abs((1 - tn * tn) / (2 * tn) - ct2) <= 4 * EPS
        assert abs(cs - 1 / np.sqrt(1 + tn * tn)) <= 4 * EPS


def test_short_cut_large_cot():
    """|ct 2phi| >= sqrt(2/eps) = 2^27: |ct phi| = 2|ct 2phi| and cs = 1."""
    for t in (1, -1):
        hpq = 1e-20
        hpp, hqq = 1.0, 0.5
        tn, cs, _ = oracle.rotation(hpp, hqq, hpq, t)
        ct2 = t * (hqq - t * hpp) / (2 * hpq)
        assert cs == 1.0
        assert tn == np.sign(ct2) / (2 * abs(ct2))


def test_hyperbolic_coth_substitution():
    """|coth 2phi| numerically 1 is replaced by 5/4, i.e. tanh phi = 1/2
    (coth 2phi = (1 + tanh^2)/(2 tanh)), cosh phi = 2/sqrt(3)."""
    tn, cs, clamped = oracle.rotation(1.0, 1.0, 1.0, -1)
    assert clamped
    assert tn == -0.5
    assert abs(cs - 2 / np.sqrt(3)) <= 2 * EPS * cs
    tn, cs, clamped = oracle.rotation(1.0, 1.0, -1.0, -1)
    assert clamped and tn == 0.5


def _mean_departure(t, exps, per_exp, seed):
    g = np.random.default_rng(seed)
    means = []
    for e in exps:
        mant = g.integers(0, 2 ** 52, size=per_exp, dtype=np.uint64)
        x = np.ldexp(1.0 + mant.astype(np.float64) / 2.0 ** 52, e)
        tn, cs = oracle.rot_params(x, t)
        d = np.empty(per_exp)
        for k in range(per_exp):
            a, c = Fraction(float(tn[k])), Fraction(float(cs[k]))
            d[k] = abs(float(c * c * (1 + t * a * a) - 1))
        means.append(d.mean())
    return float(np.mean(means))


def test_table_b1_mean_departures():
    """Appendix B, Table B.1: mean departures d_t (cos_2) and d_h (cosh_2)
    over random |ct 2phi| of each binary exponent, evaluated exactly.
    Reading: the hyperbolic experiment uses exponents 0..53 (|coth 2phi| is
    at least 1); the trigonometric one -53..53.  Fewer samples than the
    paper's 2^24 per exponent, hence the tolerance."""
    ref = _golden_b1()
    d_t = _mean_departure(1, range(-53, 54), 384, 5)
    d_h = _mean_departure(-1, range(0, 54), 512, 6)
    assert abs(d_t - ref["d_t_cos2"]) <= 0.04 * ref["d_t_cos2"], d_t
    assert abs(d_h - ref["d_h_cosh2"]) <= 0.04 * ref["d_h_cosh2"], d_h
    # the cosh_1 figure is clearly different: the test separates the two
    assert abs(d_h - ref["d_h_cosh1"]) > 0.08 * ref["d_h_cosh1"]
