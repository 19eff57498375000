"""DRDSSQ (Appendix A) and the DDRJAC one-sided Jacobi method (Section 4.3.1):
test infrastructure only, like the rest of ``oracle``.

A DRDSSQ result is a pair (j, s) standing for the sum of squares 2^j s, in
the common form of Appendix A (j even, 0.5 <= s < 2; (0, 0) for a zero
vector); the norm is 2^(j/2) sqrt(s).

The safe bounds of Appendix A, rounded inwards to doubles, are computed here
exactly in rational arithmetic:

    t_lo    = RU(sqrt(mu / gamma)),          mu = 2^-1022, gamma = 1 - eps,
    t_hi(L) = RZ(sqrt(nu / delta_n)),        nu = the largest double,
              delta_n = 2^L delta^(1 + L),  delta = 1 + eps, L = ceil(lg n),

with eps = 2^-53.  The C side (``jsvd_oracle.c``) takes them as arguments.
"""
import ctypes
import math
from fractions import Fraction

import numpy as np

from . import _load, final_order

EPS = Fraction(1, 2 ** 53)
MU = Fraction(1, 2 ** 1022)
NU = Fraction((2 ** 53 - 1) * 2 ** 971)
MAX_LG = 63  # table of t_hi for L = 0 .. MAX_LG

_i32, _i64 = ctypes.c_int32, ctypes.c_int64
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(_i32)
_pi64 = ctypes.POINTER(_i64)


def _sqrt_to_double(x, up):
    """The largest double <= sqrt(x) (up=False) or the smallest >= sqrt(x)
    (up=True), for a positive rational x whose root is a normal double."""
    # sqrt(x) = D 2^e with D an integer in [2^52, 2^53]: pick e from the bit
    # lengths, then D = floor or ceil of sqrt(x / 2^(2e)) by integer roots.
    lg = (x.numerator.bit_length() - x.denominator.bit_length()) // 2
    e = lg - 52
    while True:
        y = x / Fraction(2) ** (2 * e)
        if up:
            c = math.ceil(y)
            D = math.isqrt(c - 1) + 1
        else:
            D = math.isqrt(math.floor(y))
        if D >= 2 ** 53 and not (up and D == 2 ** 53):
            e += 1
        elif D < 2 ** 52:
            e -= 1
        else:
            return math.ldexp(D, e)


def t_lo():
    """RU(sqrt(mu / gamma))."""
    return _sqrt_to_double(MU / (1 - EPS), up=True)


def delta_n(L):
    return Fraction(2) ** L * (1 + EPS) ** (1 + L)


def t_hi(L):
    """RZ(sqrt(nu / delta_n)) for ceil(lg n) = L."""
    return _sqrt_to_double(NU / delta_n(L), up=False)


_TABLE = None


def t_hi_table():
    global _TABLE
    if _TABLE is None:
        _TABLE = np.array([t_hi(L) for L in range(MAX_LG + 1)], dtype=np.float64)
    return _TABLE


def ceil_lg(n):
    return max(0, (int(n) - 1).bit_length())


def _lib():
    lib, _, _ = _load("double")
    if not getattr(lib, "_rdssq_ready", False):
        lib.orc_rdssq.restype = None
        lib.orc_rdssq.argtypes = [_i64, _pd, _i64, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_int), _pd, ctypes.POINTER(ctypes.c_int)]
        lib.orc_gesvj_ddrjac.restype = ctypes.c_int
        lib.orc_gesvj_ddrjac.argtypes = [_i64, _i64, _pd, _i64, _pd, _i64, _i64, _i32, _pi64,
                                         ctypes.c_double, ctypes.c_double]
        lib.orc_colnorms_rdssq.restype = None
        lib.orc_colnorms_rdssq.argtypes = [_i64, _i64, _pd, _i64, _pd, _pi32, _pd,
                                           ctypes.c_double, ctypes.c_double]
        lib.orc_gesvj_many_ddrjac.restype = None
        lib.orc_gesvj_many_ddrjac.argtypes = [_i64, _pi32, _pi32, _pi64, _pi64, _pi64, _pd, _pd,
                                              _pd, _i32, _pi32, _pi32, ctypes.c_double, _pd]
        lib._rdssq_ready = True
    return lib


def rdssq(x):
    """DRDSSQ of the vector x: (j, s, parts), the sum of squares 2^j s in
    the common form and the mask of partial sums formed (1: elements below
    t_lo, scaled up; 2: unscaled; 4: above t_hi, scaled down)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    n = x.size
    j, parts = ctypes.c_int(), ctypes.c_int()
    s = ctypes.c_double()
    _lib().orc_rdssq(n, x.ctypes.data_as(_pd), 1, t_lo(), float(t_hi_table()[ceil_lg(n)]),
                     ctypes.byref(j), ctypes.byref(s), ctypes.byref(parts))
    return j.value, s.value, parts.value


def norm(x):
    """||x||_2 from DRDSSQ, 2^(j/2) sqrt(s), as a double."""
    j, s, _ = rdssq(x)
    return math.ldexp(math.sqrt(s), j // 2) if s > 0 else 0.0


def exact_ssq(x):
    """sum x_i^2 in exact rational arithmetic."""
    return sum((Fraction(float(v)) ** 2 for v in np.asarray(x, dtype=np.float64).ravel()),
               Fraction(0))


def gesvj(A, n_plus=None, max_sweeps=100, want_v=True, sort=True):
    """The row-cyclic one-sided Jacobi (H)SVD with DDRJAC pairs (DRDSSQ
    norms, the cosine of the angle from scaled columns, ct 2phi from the
    norm ratio) and DRDSSQ singular values.  Same result layout as
    ``oracle.gesvj``, plus the DRDSSQ pairs of the final columns
    (``exps``, ``ssq``) in the output order."""
    lib = _lib()
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("oracle expects m >= n")
    G = np.asfortranarray(A.copy())
    V = np.zeros((n, n), order="F") if want_v else None
    stats = np.zeros(5, dtype=np.int64)
    npl = n if n_plus is None else int(n_plus)
    th = float(t_hi_table()[ceil_lg(m)])
    lib.orc_gesvj_ddrjac(m, n, G.ctypes.data_as(_pd), m,
                         V.ctypes.data_as(_pd) if want_v else _pd(), n, npl, max_sweeps,
                         stats.ctypes.data_as(_pi64), t_lo(), th)
    S = np.zeros(n)
    ex = np.zeros(n, dtype=np.int32)
    ss = np.zeros(n)
    lib.orc_colnorms_rdssq(m, n, G.ctypes.data_as(_pd), m, S.ctypes.data_as(_pd),
                           ex.ctypes.data_as(_pi32), ss.ctypes.data_as(_pd), t_lo(), th)
    U = G
    if sort:
        # order by the exact norms 2^(j/2) sqrt(s) (S itself may overflow)
        key = _order_key(ex, ss)
        perm = final_order(key, None if n_plus is None else npl)
        S, U, ex, ss = S[perm], U[:, perm], ex[perm], ss[perm]
        if want_v:
            V = V[:, perm]
    return dict(U=U, S=S, V=V, exps=ex, ssq=ss, sweeps=int(stats[0]), rotations=int(stats[1]),
                proper=int(stats[2]), clamps=int(stats[3]), converged=bool(stats[4]))


def _order_key(ex, ss):
    """Keys that order like the norms 2^(j/2) sqrt(s): the rank of (j, s) in
    lexicographic order (the common form makes it the order of the norms),
    a zero column lowest, equal pairs equal keys."""
    ex = np.where(np.asarray(ss) > 0, np.asarray(ex, dtype=np.int64), np.iinfo(np.int64).min)
    ss = np.asarray(ss, dtype=np.float64)
    order = np.lexsort((ss, ex))
    key = np.zeros(len(ss))
    rank, prev = 0, None
    for i in order:
        cur = (int(ex[i]), float(ss[i]))
        if prev is not None and cur != prev:
            rank += 1
        key[i] = rank
        prev = cur
    return key


def gesvj_many(mats, max_sweeps=100, want_v=True):
    """``oracle.gesvj_many`` with DDRJAC pairs and DRDSSQ norms."""
    lib = _lib()
    count = len(mats)
    ms = np.array([a.shape[0] for a in mats], dtype=np.int32)
    ns = np.array([a.shape[1] for a in mats], dtype=np.int32)
    a_off = np.zeros(count, dtype=np.int64)
    s_off = np.zeros(count, dtype=np.int64)
    v_off = np.zeros(count, dtype=np.int64)
    if count:
        a_off[1:] = np.cumsum(ms.astype(np.int64) * ns)[:-1]
        s_off[1:] = np.cumsum(ns.astype(np.int64))[:-1]
        v_off[1:] = np.cumsum(ns.astype(np.int64) * ns)[:-1]
    A = np.concatenate([np.asarray(a, dtype=np.float64).ravel(order="F") for a in mats]) \
        if count else np.zeros(0)
    S = np.zeros(int(ns.sum()))
    V = np.zeros(int((ns.astype(np.int64) ** 2).sum())) if want_v else None
    sweeps = np.zeros(count, dtype=np.int32)
    status = np.zeros(count, dtype=np.int32)
    tab = t_hi_table()
    lib.orc_gesvj_many_ddrjac(
        count, ms.ctypes.data_as(_pi32), ns.ctypes.data_as(_pi32), a_off.ctypes.data_as(_pi64),
        s_off.ctypes.data_as(_pi64), v_off.ctypes.data_as(_pi64), A.ctypes.data_as(_pd),
        S.ctypes.data_as(_pd), V.ctypes.data_as(_pd) if want_v else _pd(), max_sweeps,
        sweeps.ctypes.data_as(_pi32), status.ctypes.data_as(_pi32), t_lo(),
        tab.ctypes.data_as(_pd))
    out = []
    for i in range(count):
        m, n = int(ms[i]), int(ns[i])
        U = A[a_off[i]:a_off[i] + m * n].reshape((m, n), order="F")
        s = S[s_off[i]:s_off[i] + n]
        perm = final_order(s)
        Vi = V[v_off[i]:v_off[i] + n * n].reshape((n, n), order="F")[:, perm] if want_v else None
        out.append(dict(U=U[:, perm], S=s[perm], V=Vi, sweeps=int(sweeps[i]),
                        converged=status[i] == 0))
    return out
