"""The refined FP64 operations of the hot path against IEEE on the host.

The rotation formulas (4.3)-(4.6) and the relative orthogonality test of
Section 4.3 assume correctly rounded division and square root, and so does
the Cholesky factorization of Section 4.1.  The kernels compute them from
the hardware reciprocal and reciprocal-square-root seeds refined by Newton
steps and a residual correction (the fused multiply-add refinements of
Markstein; the coupled root / half-reciprocal iteration for the square
root).  jsvd_diag_refined runs the kernels' own device functions; here they
are compared bit for bit with the host's IEEE results over the operand range
in which the kernels call them ([2^-900, 2^900]), on random significands and
on the significands where such refinements are known to be hardest: 1,
1 + ulp, all ones (2 - ulp), 1.5, and values next to powers of two.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _ops(a, b):
    import torch
    import paper_1401_2720_amd as jsvd
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    out = jsvd.diag_refined(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    return [o.cpu().numpy() for o in out]


def _operands(count, lo, hi, seed):
    g = np.random.default_rng(seed)
    edge = np.array([1.0, np.nextafter(1.0, 2.0), np.nextafter(2.0, 1.0), 1.5,
                     np.nextafter(1.5, 1.0), np.nextafter(1.5, 2.0), 1.25, 1.75,
                     np.nextafter(1.0, 2.0) + 2.0 ** -51, 2.0 - 2.0 ** -51])
    sig = np.concatenate([g.uniform(1.0, 2.0, count),
                          np.tile(edge, 200),
                          1.0 + g.integers(0, 2 ** 12, 4000) * 2.0 ** -52,   # next to 1
                          2.0 - g.integers(1, 2 ** 12, 4000) * 2.0 ** -52])  # next to 2
    ex = g.integers(lo, hi, sig.size)
    return np.ldexp(sig, ex)


def _ulps(x, ref):
    xi = x.view(np.int64)
    ri = ref.view(np.int64)
    return np.abs(xi - ri)


@pytest.mark.parametrize("seed", [1, 2])
def test_division_reciprocal_sqrt_bitwise(seed):
    a = _operands(400000, -900, 900, seed)
    b = _operands(400000, -900, 900, seed + 10)[: a.size]
    g = np.random.default_rng(seed)
    b = b[g.permutation(b.size)]
    rcp, quo, root, rs, d = _ops(a, b)
    bad = {"rcp": int(np.sum(rcp != 1.0 / b)), "div": int(np.sum(quo != a / b)),
           "sqrt": int(np.sum(root != np.sqrt(a))), "chol_sqrt": int(np.sum(d != np.sqrt(a)))}
    print(f"mismatches of {a.size}: {bad}", flush=True)
    assert bad == {"rcp": 0, "div": 0, "sqrt": 0, "chol_sqrt": 0}


def test_edge_significand_grid_bitwise():
    """Every pair of the edge significands, at a few exponents."""
    edge = np.array([1.0, np.nextafter(1.0, 2.0), np.nextafter(2.0, 1.0), 1.5,
                     np.nextafter(1.5, 1.0), np.nextafter(1.5, 2.0), 1.25, 1.75,
                     1.0 + 2.0 ** -51, 2.0 - 2.0 ** -51, 1.0 + 3 * 2.0 ** -52,
                     2.0 - 3 * 2.0 ** -52])
    ex = np.array([-900, -511, -1, 0, 1, 300, 899])
    vals = np.concatenate([np.ldexp(edge, e) for e in ex])
    a = np.repeat(vals, vals.size)
    b = np.tile(vals, vals.size)
    rcp, quo, root, rs, d = _ops(a, b)
    assert np.array_equal(rcp, 1.0 / b)
    assert np.array_equal(quo, a / b)
    assert np.array_equal(root, np.sqrt(a))
    assert np.array_equal(d, np.sqrt(a))


def test_cholesky_rsqrt_within_two_ulps_whole_range():
    """The Cholesky's 1/sqrt (the pivot row's multiplier) over the whole
    positive range, subnormals included, against 1/sqrt in extended
    precision rounded to double: within 2 ulps; its sqrt correctly rounded."""
    g = np.random.default_rng(5)
    a = np.concatenate([np.ldexp(g.uniform(1.0, 2.0, 200000), g.integers(-1022, 1024, 200000)),
                        g.uniform(0.0, 1.0, 2000) * 2.0 ** -1022,     # subnormal
                        np.array([5e-324, 2.0 ** -1022, np.nextafter(2.0 ** 1024, 0.0)])])
    a = a[a > 0]
    _, _, _, rs, d = _ops(a, np.ones_like(a))
    assert np.array_equal(d, np.sqrt(a))
    ref = (1.0 / np.sqrt(a.astype(np.longdouble))).astype(np.float64)
    assert int(_ulps(rs, ref).max()) <= 2
