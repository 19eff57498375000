"""DRDSSQ (Appendix A) and the DDRJAC pairs (Section 4.3.1) on the GPU,
through the C ABI, against the oracle.

  * jsvd_colnorms: the pair (j, s) of each column against the oracle's
    DRDSSQ and against the exact rational sum of squares, within the error
    bound of the two summation orders; bit for bit where the result is
    exact (equal powers of two, single elements at any magnitude); zero,
    NaN and ragged cases; lengths across the workgroup's tile;
  * the batched SVD with opts.scaled = 2: every problem solved with DDRJAC
    pairs, against the oracle's DDRJAC method, on well-scaled problems, on
    problems scaled by 2^+-700 (every square of the plain method overflows
    or underflows) and on problems whose columns are graded over 2^800; the
    SVD invariants; a NaN problem reported alone.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import rdssq as R
from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _say(msg):
    print(msg, flush=True)


def _gpu_colnorms(A):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    ex, ss, nr = jsvd.colnorms(torch.from_numpy(np.asfortranarray(A)).cuda())
    torch.cuda.synchronize()
    return ex.cpu().numpy(), ss.cpu().numpy(), nr.cpu().numpy()


def _wide(g, m, n, lo=-1074, hi=1020):
    e = g.integers(lo, hi + 1, (m, n))
    f = g.uniform(1.0, 2.0, (m, n)) * g.choice([-1.0, 1.0], (m, n))
    return np.ldexp(f, e)


@pytest.mark.parametrize("m", [1, 7, 255, 256, 257, 300, 4097])
def test_colnorms_against_oracle_and_exact(m):
    _say(f"colnorms m={m}")
    g = np.random.default_rng(500 + m)
    cols = [g.standard_normal((m, 4)), _wide(g, m, 4), _wide(g, m, 4, -1074, -500),
            _wide(g, m, 4, 400, 1023), np.ldexp(g.standard_normal((m, 4)), 700)]
    A = np.hstack(cols)
    ex, ss, nr = _gpu_colnorms(A)
    # the device sums ceil(m / 256) terms per thread, then a tree of depth 8,
    # then at most two additions of partial sums; the oracle sums in order
    k_gpu = math.ceil(m / 256) + 8 + 4
    for c in range(A.shape[1]):
        x = A[:, c]
        j0, s0, _ = R.rdssq(x)
        assert ex[c] % 2 == 0 and 0.5 <= ss[c] < 2.0
        got = Fraction(float(ss[c])) * Fraction(2) ** int(ex[c])
        if m <= 300:
            exact = R.exact_ssq(x)
            assert abs(got - exact) <= Fraction(k_gpu) * Fraction(101, 100) * R.EPS * exact, c
        ref = Fraction(s0) * Fraction(2) ** j0
        assert abs(got - ref) <= Fraction(k_gpu + m + 4) * Fraction(101, 100) * R.EPS * ref, c
        with np.errstate(over="ignore"):
            assert nr[c] == np.ldexp(np.sqrt(ss[c]), int(ex[c]) // 2)


def test_colnorms_exact_cases():
    """Bit for bit where the result is exact: 16 elements of 2^k (norm 4 2^k,
    squares overflowing or subnormal), a single row (norm |v| for any v),
    a zero column; NaN for a column holding a NaN or an infinity."""
    _say("colnorms exact cases")
    ks = [0, 600, 1000, -600, -1000, -1060, -1074]
    A = np.column_stack([np.full(16, math.ldexp(1.0, k)) for k in ks] + [np.zeros(16)])
    ex, ss, nr = _gpu_colnorms(A)
    for c, k in enumerate(ks):
        assert nr[c] == math.ldexp(4.0, k)
        j0, s0, _ = R.rdssq(A[:, c])
        assert (int(ex[c]), float(ss[c])) == (j0, s0)
    assert ex[-1] == 0 and ss[-1] == 0.0 and nr[-1] == 0.0
    g = np.random.default_rng(501)
    row = _wide(g, 1, 300)
    row[0, :4] = [5e-324, -5e-324, 1.7976931348623157e308, -2.2250738585072014e-308]
    ex, ss, nr = _gpu_colnorms(row)
    assert np.array_equal(nr, np.abs(row[0]))
    B = g.standard_normal((40, 3))
    B[5, 0] = np.nan
    B[7, 1] = np.inf
    ex, ss, nr = _gpu_colnorms(B)
    assert np.isnan(ss[0]) and np.isnan(ss[1]) and np.isfinite(ss[2])


# ----------------------------------------------------------- batched DDRJAC

def _solve_batch(mats, scaled):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    batch = jsvd.Batch(mats)
    jsvd.gesvd_batched(batch, scaled=scaled)
    torch.cuda.synchronize()
    return [batch.results(i) for i in range(len(mats))], batch.status.cpu().numpy()


def _check_problem(A, U, S, V, ref, rel_tol):
    n = S.shape[0]
    assert np.all(np.diff(S) <= 0)
    pos = ref > 0
    assert np.max(np.abs(S[pos] - ref[pos]) / ref[pos]) <= rel_tol
    assert np.all(S[~pos] == 0)
    k = int(np.sum(pos))
    assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-13 * n
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    # columnwise residual relative to the column's norm (the scales differ)
    Rm = A - (U * S) @ V.T
    cn = np.array([R.norm(A[:, j]) for j in range(n)])
    rn = np.array([R.norm(Rm[:, j]) for j in range(n)])
    assert np.max(rn / np.where(cn > 0, cn, 1.0)) <= 1e-13 * n


SIZES = [(20, 12), (32, 32), (60, 40), (100, 64), (150, 96), (192, 128), (300, 80), (256, 256)]


@pytest.mark.parametrize("scale", ["unit", "big", "small", "graded"])
def test_batched_ddrjac_against_oracle(scale):
    _say(f"batched ddrjac scale={scale}")
    g = inputs.rng(600)
    mats = []
    for i, (m, n) in enumerate(SIZES):
        B = inputs.gaussian(m, n, g)
        if scale == "big":
            B = np.ldexp(B, 700)
        elif scale == "small":
            B = np.ldexp(B, -700)
        elif scale == "graded":
            e = np.linspace(400, -400, n).round().astype(int)
            B = np.ldexp(B, e[None, :])
        mats.append(B)
    res, status = _solve_batch(mats, "on")
    assert np.all(status == 0), status
    refs = R.gesvj_many(mats)
    for A, (U, S, V), ref in zip(mats, res, refs):
        _check_problem(A, U, S, V, ref["S"], 1e-12 if scale != "graded" else 1e-11)
    if scale == "big":
        # exact scaling: the results are those of the unit problems times 2^700
        res1, _ = _solve_batch([np.ldexp(A, -700) for A in mats], "on")
        for (U, S, V), (U1, S1, V1) in zip(res, res1):
            assert np.array_equal(S, np.ldexp(S1, 700)) and np.array_equal(U, U1)
            assert np.array_equal(V, V1)


def test_batched_ddrjac_matches_plain_on_well_scaled():
    _say("batched ddrjac vs plain")
    g = inputs.rng(601)
    mats = [inputs.gaussian(m, n, g) for m, n in SIZES]
    a, sa = _solve_batch(mats, "on")
    b, sb = _solve_batch(mats, "off")
    assert np.all(sa == 0) and np.all(sb == 0)
    for (U, S, V), (U2, S2, V2) in zip(a, b):
        assert np.max(np.abs(S - S2)) <= 1e-13 * S[0] * S.shape[0]


def test_batched_ddrjac_nan_problem_reported_alone():
    _say("batched ddrjac nan")
    g = inputs.rng(602)
    mats = [inputs.gaussian(40, 30, g) for _ in range(3)]
    mats[1][4, 2] = np.nan
    res, status = _solve_batch(mats, "on")
    assert status[1] == 3 and status[0] == 0 and status[2] == 0
    refs = R.gesvj_many([mats[0], mats[2]])
    for (U, S, V), ref in zip([res[0], res[2]], refs):
        assert np.max(np.abs(S - ref["S"]) / ref["S"]) <= 1e-12
