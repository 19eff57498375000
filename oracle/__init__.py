"""Oracle for the one-sided Jacobi (H)SVD: test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library in ``paper_1401_2720_amd``; the two meet only through the seeded
input generators.

Contents
  * ``gesvj``        -- cyclic one-sided Jacobi SVD / hyperbolic SVD (C, fp64
                        or x87 extended), with the final ordering applied.
  * ``rotation``     -- rotation parameters of eqs. (4.3)-(4.6).
  * ``rot_params``   -- eqs. (4.4)-(4.6) from |ct 2phi| (Appendix B).
  * ``gesvj_many``   -- many independent small problems (OpenMP).
  * ``strategy``     -- the closest parallel strategies of Section 3.
  * ``adjoint``      -- the SVD adjoint (reverse-mode derivative).
  * ``rdssq``        -- DRDSSQ, the overflow-safe sum of squares of
                        Appendix A, and the one-sided Jacobi method with
                        DDRJAC pairs (Section 4.3.1) built on it.

Final ordering (the paper fixes none; reading used): ordinary SVD -- singular
values non-increasing, ties kept in column order; hyperbolic SVD -- J stays
partitioned, the positive part by non-increasing sigma and the negative part
by non-decreasing sigma, so that lambda_i = j_i sigma_i^2 is non-increasing
(Section 4.3, subphase 5, keeps that order locally).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIBS = {}
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def _load(precision="double"):
    if precision in _LIBS:
        return _LIBS[precision]
    path = _build.LIBS[precision]
    if not os.path.exists(path):
        _build.build()
    lib = ctypes.CDLL(path)
    sfx = "_ld" if precision == "extended" else ""
    real = ctypes.c_longdouble if precision == "extended" else ctypes.c_double
    preal = ctypes.POINTER(real)
    f = getattr(lib, "orc_gesvj" + sfx)
    f.restype = ctypes.c_int
    f.argtypes = [_i64, _i64, preal, _i64, preal, _i64, _i64, _i32, ctypes.POINTER(_i64)]
    f = getattr(lib, "orc_gesvj_rr" + sfx)
    f.restype = ctypes.c_int
    f.argtypes = [_i64, _i64, preal, _i64, preal, _i64, _i64, _i32, _i64, ctypes.POINTER(_i64)]
    f = getattr(lib, "orc_colnorms" + sfx)
    f.restype = None
    f.argtypes = [_i64, _i64, preal, _i64, preal]
    f = getattr(lib, "orc_rotation" + sfx)
    f.restype = ctypes.c_int
    f.argtypes = [real, real, real, ctypes.c_int, preal, preal]
    f = getattr(lib, "orc_rot_params" + sfx)
    f.restype = None
    f.argtypes = [_i64, preal, ctypes.c_int, preal, preal]
    f = getattr(lib, "orc_gesvj_many" + sfx)
    f.restype = None
    pi32 = ctypes.POINTER(_i32)
    pi64 = ctypes.POINTER(_i64)
    f.argtypes = [_i64, pi32, pi32, pi64, pi64, pi64, preal, preal, preal, _i32, pi32, pi32]
    getattr(lib, "orc_num_threads" + sfx).restype = ctypes.c_int
    _LIBS[precision] = (lib, sfx, real)
    return _LIBS[precision]


def _dtype(precision):
    return np.longdouble if precision == "extended" else np.float64


def _ptr(a, real):
    return a.ctypes.data_as(ctypes.POINTER(real))


def final_order(S, n_plus=None):
    """Permutation that puts the computed columns in the output order."""
    n = S.shape[0]
    if n_plus is None or n_plus >= n:
        return np.argsort(-S, kind="stable")
    pos = np.argsort(-S[:n_plus], kind="stable")
    neg = n_plus + np.argsort(S[n_plus:], kind="stable")
    return np.concatenate([pos, neg])


def gesvj(A, n_plus=None, max_sweeps=100, order="row", precision="double",
          want_v=True, sort=True, max_rounds=0):
    """One-sided Jacobi (H)SVD of A (m x n, m >= n).

    n_plus: number of +1 entries of J = diag(I, -I); None = ordinary SVD.
    order: "row" (sequential row-cyclic) or "rr" (parallel round-robin).
    Returns dict(U, S, V, sweeps, rotations, proper, clamps, converged).
    For the hyperbolic SVD, G V = U Sigma with V^T J V = J.
    """
    lib, sfx, real = _load(precision)
    dt = _dtype(precision)
    A = np.asarray(A)
    m, n = A.shape
    if m < n:
        raise ValueError("oracle expects m >= n")
    G = np.asfortranarray(A.astype(dt, copy=True))
    V = np.zeros((n, n), dtype=dt, order="F") if want_v else None
    stats = np.zeros(5, dtype=np.int64)
    npl = n if n_plus is None else int(n_plus)
    vptr = _ptr(V, real) if want_v else ctypes.POINTER(real)()
    if order == "row":
        getattr(lib, "orc_gesvj" + sfx)(m, n, _ptr(G, real), m, vptr, n, npl, max_sweeps,
                                        stats.ctypes.data_as(ctypes.POINTER(_i64)))
    elif order == "rr":
        getattr(lib, "orc_gesvj_rr" + sfx)(m, n, _ptr(G, real), m, vptr, n, npl, max_sweeps,
                                           int(max_rounds),
                                           stats.ctypes.data_as(ctypes.POINTER(_i64)))
    else:
        raise ValueError(order)
    S = np.zeros(n, dtype=dt)
    getattr(lib, "orc_colnorms" + sfx)(m, n, _ptr(G, real), m, _ptr(S, real))
    U = G
    if sort:
        perm = final_order(S, None if n_plus is None else npl)
        S = S[perm]
        U = U[:, perm]
        if want_v:
            V = V[:, perm]
    return dict(U=U, S=S, V=V, sweeps=int(stats[0]), rotations=int(stats[1]),
                proper=int(stats[2]), clamps=int(stats[3]), converged=bool(stats[4]))


def rotation(hpp, hqq, hpq, t, precision="double"):
    """(tn, cs, clamped) from eqs. (4.3)-(4.6); t = +1 trig, -1 hyperbolic."""
    lib, sfx, real = _load(precision)
    tn, cs = real(), real()
    fl = getattr(lib, "orc_rotation" + sfx)(hpp, hqq, hpq, int(t), ctypes.byref(tn),
                                             ctypes.byref(cs))
    return tn.value, cs.value, bool(fl & 1)


def rot_params(abs_ct2, t, precision="double"):
    """Vectorised eqs. (4.4)-(4.6) from |ct 2phi|: returns (tn, cs)."""
    lib, sfx, real = _load(precision)
    a = np.ascontiguousarray(abs_ct2, dtype=_dtype(precision))
    tn = np.empty_like(a)
    cs = np.empty_like(a)
    getattr(lib, "orc_rot_params" + sfx)(a.size, _ptr(a, real), int(t), _ptr(tn, real),
                                          _ptr(cs, real))
    return tn, cs


def gesvj_many(mats, max_sweeps=100, want_v=True):
    """Solve many independent small SVDs (one per OpenMP thread).

    mats: list of (m_i x n_i) arrays.  Returns a list of dict(U, S, V, sweeps,
    converged), each in the final order.
    """
    lib, sfx, real = _load("double")
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
    S = np.zeros(int(ns.sum()), dtype=np.float64)
    V = np.zeros(int((ns.astype(np.int64) ** 2).sum()), dtype=np.float64) if want_v else None
    sweeps = np.zeros(count, dtype=np.int32)
    status = np.zeros(count, dtype=np.int32)
    pi32 = ctypes.POINTER(_i32)
    pi64 = ctypes.POINTER(_i64)
    getattr(lib, "orc_gesvj_many" + sfx)(
        count, ms.ctypes.data_as(pi32), ns.ctypes.data_as(pi32), a_off.ctypes.data_as(pi64),
        s_off.ctypes.data_as(pi64), v_off.ctypes.data_as(pi64), _ptr(A, real), _ptr(S, real),
        _ptr(V, real) if want_v else ctypes.POINTER(real)(), max_sweeps,
        sweeps.ctypes.data_as(pi32), status.ctypes.data_as(pi32))
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


def num_threads():
    """OpenMP threads used by the parallel oracle entry points."""
    lib, sfx, _ = _load("double")
    return int(getattr(lib, "orc_num_threads" + sfx)())
