"""Pins for the oracle's DRDSSQ (Appendix A) and DDRJAC method (Section 4.3.1).

DRDSSQ is checked against what the mathematics fixes: the safe bounds
against their defining inequalities in exact rational arithmetic and
against closed forms worked out by hand, the sum of squares against its
exact rational value within the error bound of a sum of n positive terms,
vectors whose norm is exact (2^k times a perfect-square count of equal
elements, a single element at any magnitude, subnormals included), the
partition of Appendix A on inputs that must use each partial sum, the
common form, and invariance under scaling by powers of two.  DDRJAC is
checked against LAPACK, against the plain x87 extended-precision oracle on
badly graded input (whose squares do not overflow there), and for exact
invariance under scaling by 2^+-700, where every Gram entry of the plain
double method would overflow or underflow.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import rdssq as R
from paper_1401_2720_amd import inputs

EPS = 2.0 ** -53
F_EPS = Fraction(1, 2 ** 53)


# ------------------------------------------------------------ safe bounds

def test_t_lo_closed_form():
    """sqrt(mu / gamma) = 2^-511 (1 - eps)^(-1/2) = 2^-511 (1 + eps/2 + ...)
    lies strictly between 2^-511 and its successor 2^-511 (1 + 2^-52), so
    rounding it up gives the successor."""
    assert R.t_lo() == math.ldexp(1.0 + 2.0 ** -52, -511)


def test_t_hi_closed_form_for_one_element():
    """L = 0: sqrt(nu / (1 + eps)) = 2^512 sqrt((1 - eps) / (1 + eps))
    = 2^512 (1 - eps + eps^2 / 2 + ...), just above 2^512 (1 - eps), the
    predecessor of 2^512; rounding toward zero gives that predecessor."""
    assert R.t_hi(0) == np.nextafter(2.0 ** 512, 0.0)


@pytest.mark.parametrize("L", list(range(0, 64)))
def test_bounds_defining_inequalities(L):
    """t_hi(L)^2 delta_n <= nu < succ(t_hi(L))^2 delta_n and
    t_lo^2 gamma >= mu > pred(t_lo)^2 gamma, exactly."""
    th = R.t_hi(L)
    dn = R.delta_n(L)
    assert Fraction(th) ** 2 * dn <= R.NU
    assert Fraction(float(np.nextafter(th, np.inf))) ** 2 * dn > R.NU
    tl = R.t_lo()
    gamma = 1 - F_EPS
    assert Fraction(tl) ** 2 * gamma >= R.MU
    assert Fraction(float(np.nextafter(tl, 0.0))) ** 2 * gamma < R.MU


def test_table_matches_bounds():
    tab = R.t_hi_table()
    assert tab.shape == (64,)
    assert all(tab[L] == R.t_hi(L) for L in (0, 1, 7, 30, 63))
    assert np.all(np.diff(tab) < 0)


# ------------------------------------------------------------ DRDSSQ

def _value(j, s):
    return Fraction(s) * Fraction(2) ** j


def _wide_vector(g, n, lo=-1074, hi=1020):
    """Elements with exponents uniform over [lo, hi], random signs and
    significands (subnormals included)."""
    e = g.integers(lo, hi + 1, n)
    f = g.uniform(1.0, 2.0, n) * g.choice([-1.0, 1.0], n)
    return np.array([math.ldexp(a, int(b)) for a, b in zip(f, e)])


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 65, 300])
def test_sum_of_squares_against_exact(n):
    """2^j s against the exact rational sum of squares, within the bound of
    a sequential sum of n positive terms plus the two additions of the
    partial sums: relative error <= (n + 4) eps (1 + small)."""
    g = np.random.default_rng(100 + n)
    for trial in range(20):
        if trial % 4 == 0:
            x = g.standard_normal(n)
        elif trial % 4 == 1:
            x = _wide_vector(g, n)
        elif trial % 4 == 2:
            x = _wide_vector(g, n, -1074, -500)
        else:
            x = _wide_vector(g, n, 400, 1023)
        j, s, _ = R.rdssq(x)
        exact = R.exact_ssq(x)
        got = _value(j, s)
        bound = Fraction(n + 4) * F_EPS * Fraction(101, 100)
        assert abs(got - exact) <= bound * exact, (n, trial)


@pytest.mark.parametrize("k", [0, 1, 600, 1000, -600, -1000, -1060, -1074])
def test_exact_norm_of_equal_elements(k):
    """16 elements of 2^k: the norm is 4 2^k exactly, also where the squares
    overflow (k = 1000) or underflow (k <= -600; 2^-1060 and 2^-1074 are
    subnormal)."""
    x = np.full(16, math.ldexp(1.0, k))
    x[::3] *= -1
    assert R.norm(x) == math.ldexp(4.0, k)
    j, s, _ = R.rdssq(x)
    assert _value(j, s) == Fraction(16) * Fraction(2) ** (2 * k)


def test_single_element_norm_is_its_magnitude():
    """sqrt(RN(y^2)) = |y| in binary floating point without under- or
    overflow, and DRDSSQ scales the element into that range: the norm of
    [v] is |v| exactly for any finite v, subnormal or near overflow."""
    g = np.random.default_rng(7)
    vals = list(_wide_vector(g, 400)) + [5e-324, -5e-324, 2.2250738585072014e-308,
                                          1.7976931348623157e308, -1.0, 3.0]
    for v in vals:
        assert R.norm(np.array([v])) == abs(v), v


def test_partitions():
    """The partial sums that Appendix A forms for each range of values."""
    tl, th = R.t_lo(), float(R.t_hi_table()[2])
    assert R.rdssq(np.array([1.0, -2.0, 3.0]))[2] == 2
    assert R.rdssq(np.array([2.0 ** 600, -2.0 ** 700, 2.0 ** 900]))[2] == 4
    assert R.rdssq(np.array([2.0 ** -600, 5e-324, -2.0 ** -700]))[2] == 1
    assert R.rdssq(np.array([2.0 ** 600, 3.0, 2.0 ** -600]))[2] == 7
    assert R.rdssq(np.array([th, tl, 0.0]))[2] == 2      # inclusive bounds
    assert R.rdssq(np.array([np.nextafter(th, np.inf), 1.0, 0.0]))[2] == 6
    assert R.rdssq(np.array([np.nextafter(tl, 0.0), 1.0, 0.0]))[2] == 3
    # elements exactly on the bounds belong to the unscaled sum, and alone
    # their norm is exact (sqrt(RN(v^2)) = |v|)
    for v in (tl, float(R.t_hi_table()[0])):
        j, s, parts = R.rdssq(np.array([v]))
        assert parts == 2 and R.norm(np.array([v])) == v, v
    assert R.rdssq(np.full(16, float(R.t_hi_table()[4])))[2] == 2
    # three partial sums: the value is exact here (each term is a power of
    # two far apart, and the sums are dominated by the largest)
    j, s, _ = R.rdssq(np.array([2.0 ** 600, 3.0, 2.0 ** -600]))
    assert (j, s) == (1200, 1.0)


def test_zero_vector_and_zeros_ignored():
    assert R.rdssq(np.zeros(5)) == (0, 0.0, 0)
    x = np.array([0.0, 2.0 ** -900, 0.0, -2.0 ** -900])
    j, s, parts = R.rdssq(x)
    assert parts == 1 and _value(j, s) == 2 * Fraction(2) ** -1800


def test_common_form():
    g = np.random.default_rng(8)
    for _ in range(200):
        x = _wide_vector(g, int(g.integers(1, 50)))
        j, s, _ = R.rdssq(x)
        assert j % 2 == 0 and 0.5 <= s < 2.0


@pytest.mark.parametrize("k", [300, 700, 1000, -300, -700])
def test_power_of_two_scaling_is_exact(k):
    """Scaling x by 2^k scales the sum of squares by 2^(2k): j moves by 2k
    and s is the same bits, whichever partial sums the scaled vector uses."""
    x = np.random.default_rng(9).standard_normal(100)
    j0, s0, p0 = R.rdssq(x)
    j1, s1, p1 = R.rdssq(x * 2.0 ** k)
    assert p0 == 2 and p1 == (2 if abs(k) < 500 else (4 if k > 0 else 1))
    assert j1 == j0 + 2 * k and s1 == s0


# ------------------------------------------------------------ DDRJAC

def test_ddrjac_against_lapack():
    g = inputs.rng(21)
    for m, n in [(40, 30), (64, 64), (100, 17)]:
        A = inputs.gaussian(m, n, g)
        r = R.gesvj(A)
        s = scipy.linalg.svd(A, compute_uv=False)
        assert r["converged"]
        assert np.max(np.abs(r["S"] - s)) <= 10 * n * EPS * s[0]
        U, S, V = r["U"], r["S"], r["V"]
        assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
        assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
        assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)


def test_ddrjac_agrees_with_plain_method():
    A = inputs.prescribed(80, 60, inputs.logspaced(60, -8.0), inputs.rng(22))
    a = R.gesvj(A)["S"]
    b = oracle.gesvj(A)["S"]
    assert np.max(np.abs(a - b)) <= 10 * 60 * EPS * b[0]


@pytest.mark.parametrize("k", [700, -700])
def test_ddrjac_power_of_two_scaling_is_exact(k):
    """Every step of DDRJAC commutes with an exact scaling of G by 2^k, so
    the result on 2^k G is 2^k times the result on G, bit for bit; on such
    input the plain double method's Gram entries overflow (k = 700) or
    underflow (k = -700)."""
    A = inputs.gaussian(50, 40, inputs.rng(23))
    r0 = R.gesvj(A)
    r1 = R.gesvj(A * 2.0 ** k)
    assert r1["sweeps"] == r0["sweeps"]
    assert np.array_equal(r1["S"], r0["S"] * 2.0 ** k)
    assert np.array_equal(r1["U"], r0["U"]) and np.array_equal(r1["V"], r0["V"])
    with np.errstate(over="ignore", under="ignore"):
        hpp = np.sum((A[:, 0] * 2.0 ** k) ** 2)
    assert hpp == np.inf or hpp < 2.0 ** -1000


@pytest.mark.parametrize("top,bottom", [(900, 100), (-100, -900)])
def test_ddrjac_graded_columns_against_extended_precision(top, bottom):
    """Columns graded over 2^top .. 2^bottom (ratios up to 2^800): the plain
    method in x87 extended precision (whose exponent range holds every
    square) is the reference; DDRJAC in double keeps every sigma to the
    relative accuracy the column scaling allows, where the plain double
    method's squares overflow or underflow."""
    g = np.random.default_rng(24)
    B = g.standard_normal((40, 24))
    d = np.array([math.ldexp(1.0, int(e)) for e in np.linspace(top, bottom, 24).round()])
    A = B * d
    r = R.gesvj(A)
    rx = oracle.gesvj(A, precision="extended")
    sx = rx["S"].astype(np.float64)
    rel = np.abs(r["S"] - sx) / sx
    assert r["converged"]
    assert np.max(rel) <= 64 * EPS * np.linalg.cond(B) * np.sqrt(24)
    with np.errstate(all="ignore"):
        plain = oracle.gesvj(A, max_sweeps=30)["S"]
        assert not np.all(np.abs(plain - sx) <= 1e-12 * sx)


def test_ddrjac_hyperbolic_agrees_with_plain_method():
    A = inputs.gaussian(60, 40, inputs.rng(25))
    a = R.gesvj(A, n_plus=25)
    b = oracle.gesvj(A, n_plus=25)
    assert np.max(np.abs(a["S"] - b["S"]) / b["S"]) <= 1e-12
    a2 = R.gesvj(A * 2.0 ** 650, n_plus=25)
    assert np.array_equal(a2["S"], a["S"] * 2.0 ** 650)


def test_ddrjac_zero_column_and_many():
    A = inputs.gaussian(30, 12, inputs.rng(26))
    A[:, 4] = 0.0
    r = R.gesvj(A)
    assert r["converged"] and r["S"][-1] == 0.0 and np.all(r["U"][:, -1] == 0.0)
    mats = [inputs.gaussian(int(m), int(n), inputs.rng(27 + i)) * 2.0 ** (600 * (-1) ** i)
            for i, (m, n) in enumerate([(10, 8), (33, 20), (64, 64), (5, 1)])]
    many = R.gesvj_many(mats)
    for M, res in zip(mats, many):
        one = R.gesvj(M)
        assert np.array_equal(res["S"], one["S"]) and np.array_equal(res["U"], one["U"])
