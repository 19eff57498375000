"""The library's DRDSSQ bounds (a host-only call, no device needed) against
the oracle's exact rational ones, for every ceil(lg n) the library accepts;
and its argument checks."""
import ctypes

import pytest

from oracle import rdssq as R


def test_bounds_match_exact_rational_bounds():
    import paper_1401_2720_amd as jsvd
    tl = R.t_lo()
    for lg in range(64):
        lo, hi = jsvd.rdssq_bounds(lg)
        assert lo == tl, lg
        assert hi == R.t_hi(lg), lg


def test_bounds_argument_checks():
    from paper_1401_2720_amd import _binding as B
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert B.lib().jsvd_rdssq_bounds(-1, ctypes.byref(lo), ctypes.byref(hi)) == -1
    assert B.lib().jsvd_rdssq_bounds(64, ctypes.byref(lo), ctypes.byref(hi)) == -1
    assert B.lib().jsvd_rdssq_bounds(3, None, ctypes.byref(hi)) == -2
    with pytest.raises(B.JsvdError):
        B.rdssq_bounds(70)
