"""The refined FP64 operations of the hot path against IEEE on the host.

The rotation formulas (4.3)-(4.6) and the relative orthogonality test of
Section 4.3 assume correctly rounded division and square root, and so does
the Cholesky factorization of Section 4.1.  The kernels compute them from
the hardware reciprocal and reciprocal-square-root seeds: Newton steps and a
residual correction with fused multiply-adds (Markstein's scheme) give a
result within one ulp, and an exact rounding test against its neighbour
makes it the correctly rounded one.  jsvd_diag_refined runs the kernels'
own device functions; here they are compared bit for bit with the host's
IEEE results over the operand ranges in which the kernels call them
(operands and results in [2^-900, 2^900]) on

  * random significands, signed quotients;
  * a grid of edge significands (1, 1 + ulp, 2 - ulp, 1.5 +- ulp, ...);
  * the hardest operands (tests/golden/hard_cases.txt): those whose exact
    reciprocal, quotient or root lies closest to a rounding midpoint, where
    a Newton iteration without the final test does round the wrong way.

The Cholesky's pair (1/sqrt and sqrt of a pivot, after an exact power-of-two
scaling) is checked over the whole positive range, subnormals included: the
root correctly rounded, 1/sqrt within 2 ulps.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _ops(a, b):
    import torch
    import paper_1401_2720_amd as jsvd
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    out = jsvd.diag_refined(torch.from_numpy(np.ascontiguousarray(a)).cuda(),
                            torch.from_numpy(np.ascontiguousarray(b)).cuda())
    return [o.cpu().numpy() for o in out]


EDGE = np.array([1.0, np.nextafter(1.0, 2.0), np.nextafter(2.0, 1.0), 1.5,
                 np.nextafter(1.5, 1.0), np.nextafter(1.5, 2.0), 1.25, 1.75,
                 1.0 + 2.0 ** -51, 2.0 - 2.0 ** -51, 1.0 + 3 * 2.0 ** -52,
                 2.0 - 3 * 2.0 ** -52])


def _significands(count, g):
    return np.concatenate([g.uniform(1.0, 2.0, count),
                           np.tile(EDGE, 200),
                           1.0 + g.integers(0, 2 ** 12, 4000) * 2.0 ** -52,   # next to 1
                           2.0 - g.integers(1, 2 ** 12, 4000) * 2.0 ** -52])  # next to 2


@pytest.mark.parametrize("seed", [1, 2])
def test_division_reciprocal_sqrt_bitwise(seed):
    g = np.random.default_rng(seed)
    sb = _significands(400000, g)
    eb = g.integers(-900, 901, sb.size)
    b = np.ldexp(sb, eb)
    sa = _significands(400000, g)[g.permutation(sb.size)]
    ea = np.clip(eb + g.integers(-600, 601, sb.size), -900, 900)   # a / b stays normal
    a = np.ldexp(sa, ea)
    bs = b * np.where(g.integers(0, 2, b.size) == 1, -1.0, 1.0)
    a_signed = a * np.where(g.integers(0, 2, a.size) == 1, -1.0, 1.0)
    rcp, _, root, _, d = _ops(a, b)
    _, quo, _, _, _ = _ops(a_signed, bs)
    bad = {"rcp": int(np.sum(rcp != 1.0 / b)), "div": int(np.sum(quo != a_signed / bs)),
           "sqrt": int(np.sum(root != np.sqrt(a))), "chol_sqrt": int(np.sum(d != np.sqrt(a)))}
    print(f"mismatches of {a.size}: {bad}", flush=True)
    assert bad == {"rcp": 0, "div": 0, "sqrt": 0, "chol_sqrt": 0}


def test_edge_significand_grid_bitwise():
    """Every pair of the edge significands, at exponents whose quotients stay
    inside the kernels' range, both signs of the quotient."""
    ex = np.array([-450, -300, -1, 0, 1, 300, 449])
    vals = np.concatenate([np.ldexp(EDGE, e) for e in ex])
    a = np.repeat(vals, vals.size)
    b = np.tile(vals, vals.size)
    rcp, quo, root, rs, d = _ops(a, b)
    assert np.array_equal(rcp, 1.0 / b)
    assert np.array_equal(quo, a / b)
    assert np.array_equal(root, np.sqrt(a))
    assert np.array_equal(d, np.sqrt(a))
    _, quo_neg, _, _, _ = _ops(-a, b)
    assert np.array_equal(quo_neg, -a / b)


def _hard_cases():
    rcp, div, sq = [], [], []
    with open(os.path.join(HERE, "golden", "hard_cases.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "rcp":
                rcp.append(int(p[1]))
            elif p[0] == "div":
                div.append((int(p[1]), int(p[2])))
            else:
                sq.append(int(p[1]))
    return rcp, div, sq


def test_hardest_operands_bitwise():
    """Reciprocals, quotients and roots that lie closest to a rounding
    midpoint, at exponents across the kernels' range."""
    rcp_b, div_ab, sq_u = _hard_cases()
    assert len(rcp_b) >= 50 and len(div_ab) >= 300 and len(sq_u) >= 50
    for e in (-800, -301, 0, 299, 800):
        b = np.ldexp(np.array(rcp_b, dtype=np.float64), -52 + e)
        rcp, _, _, _, _ = _ops(np.ones_like(b), b)
        assert np.array_equal(rcp, 1.0 / b), e
        A = np.array([x for x, _ in div_ab], dtype=np.float64)
        B = np.array([y for _, y in div_ab], dtype=np.float64)
        a, b = np.ldexp(A, -52 + e // 2), np.ldexp(B, -52 - e // 2)
        _, quo, _, _, _ = _ops(np.concatenate([a, -a]), np.concatenate([b, b]))
        assert np.array_equal(quo, np.concatenate([a / b, -a / b])), e
        u = np.ldexp(np.array(sq_u, dtype=np.float64), -52 + 2 * (e // 2))
        _, _, root, _, d = _ops(u, np.ones_like(u))
        assert np.array_equal(root, np.sqrt(u)), e
        assert np.array_equal(d, np.sqrt(u)), e


def _ulps(x, ref):
    return np.abs(x.view(np.int64) - ref.view(np.int64))


def test_cholesky_rsqrt_within_two_ulps_whole_range():
    """The Cholesky's 1/sqrt (the pivot row's multiplier) over the whole
    positive range, subnormals included, against 1/sqrt in extended
    precision rounded to double: within 2 ulps; its sqrt correctly rounded."""
    g = np.random.default_rng(5)
    a = np.concatenate([np.ldexp(g.uniform(1.0, 2.0, 200000), g.integers(-1022, 1024, 200000)),
                        g.uniform(0.0, 1.0, 2000) * 2.0 ** -1022,     # subnormal
                        np.array([5e-324, 2.0 ** -1022, np.finfo(np.float64).max])])
    a = a[a > 0]
    _, _, _, rs, d = _ops(a, np.ones_like(a))
    assert np.array_equal(d, np.sqrt(a))
    ref = (1.0 / np.sqrt(a.astype(np.longdouble))).astype(np.float64)
    worst = int(_ulps(rs, ref).max())
    print(f"max ulps of 1/sqrt: {worst}", flush=True)
    assert worst <= 2
