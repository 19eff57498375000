"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the Jacobi method: it only draws random
matrices of the shapes and spectra of the workloads (numpy PCG64 streams,
fp64, on the host).  The paper's own test matrices (Section 6: Cholesky
factors generated in quadruple precision) are not available; these stand
in for them.

Haar-distributed orthogonal factors come from the QR factorisation of a
Gaussian matrix with the signs of R's diagonal moved into Q, which is what
makes the distribution Haar.
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def orthonormal_columns(m, n, gen):
    """m x n matrix with Haar-distributed orthonormal columns (m >= n)."""
    Q, R = np.linalg.qr(gen.standard_normal((m, n)))
    d = np.sign(np.diag(R))
    d[d == 0] = 1
    return Q * d


def prescribed(m, n, sigma, gen):
    """A = Q1 diag(sigma) Q2^T with Q1 (m x n) and Q2 (n x n) Haar."""
    Q1 = orthonormal_columns(m, n, gen)
    Q2 = orthonormal_columns(n, n, gen)
    return np.asfortranarray((Q1 * np.asarray(sigma)) @ Q2.T)


def logspaced(n, lo_exp):
    """n values log-spaced from 1 down to 10**lo_exp."""
    if n == 1:
        return np.ones(1)
    return 10.0 ** (lo_exp * np.arange(n) / (n - 1))


def gaussian(m, n, gen):
    return np.asfortranarray(gen.standard_normal((m, n)))


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def small_graded(seed=1, n=256):
    """256 x 256, sigma log-spaced 1 .. 1e-6, Haar factors (block width 16)."""
    g = rng(seed)
    return prescribed(n, n, logspaced(n, -6.0), g)


def square_gaussian(seed=2, n=4096):
    """n x n with N(0,1) entries."""
    return gaussian(n, n, rng(seed))


def tall_graded(seed=3, m=8192, n=2048):
    """m x n, sigma log-spaced 1 .. 1e-10, Haar factors."""
    g = rng(seed)
    return prescribed(m, n, logspaced(n, -10.0), g)


def hyperbolic_gaussian(seed=4, n=2048, n_plus=1280):
    """n x n with N(0,1) entries and J = diag(+1 x n_plus, -1 x rest)."""
    A = gaussian(n, n, rng(seed))
    J = np.concatenate([np.ones(n_plus, np.int8), -np.ones(n - n_plus, np.int8)])
    return A, J


def ragged_batch(seed=5, count=10000, n_lo=8, n_hi=128, extra_rows=64,
                 prescribed_count=None):
    """Many uneven small problems packed column-major into one buffer.

    n_i ~ U{n_lo..n_hi}, m_i = n_i + U{0..extra_rows}; a seeded choice of
    20% of the problems (``prescribed_count``) use Q1 diag(logspace(0,-8))
    Q2^T, the rest N(0,1).  Returns dict(m, n, a_off, A, mats) with int32
    sizes, int64 offsets (in elements) and the packed fp64 buffer.
    """
    g = rng(seed)
    n = g.integers(n_lo, n_hi + 1, size=count).astype(np.int32)
    m = (n + g.integers(0, extra_rows + 1, size=count)).astype(np.int32)
    if prescribed_count is None:
        prescribed_count = count // 5
    special = np.zeros(count, bool)
    special[g.choice(count, size=prescribed_count, replace=False)] = True
    mats = []
    for i in range(count):
        if special[i]:
            mats.append(prescribed(int(m[i]), int(n[i]), logspaced(int(n[i]), -8.0), g))
        else:
            mats.append(gaussian(int(m[i]), int(n[i]), g))
    sizes = m.astype(np.int64) * n
    a_off = np.zeros(count, np.int64)
    a_off[1:] = np.cumsum(sizes)[:-1]
    A = np.concatenate([a.ravel(order="F") for a in mats]) if count else np.zeros(0)
    return dict(m=m, n=n, a_off=a_off, A=A, mats=mats, special=special)


def differentiable_set(seed=6, batch=256, n_small=64, n_large=1024, k=8):
    """Well-separated spectra sigma_i = 1 + 0.01 i with Haar factors, and
    N(0,1) loss weights (w per singular value, W per entry)."""
    g = rng(seed)
    sig_s = 1.0 + 0.01 * np.arange(n_small)
    small = np.stack([prescribed(n_small, n_small, sig_s, g) for _ in range(batch)])
    sig_l = 1.0 + 0.01 * np.arange(n_large)
    large = prescribed(n_large, n_large, sig_l, g)
    w_s = g.standard_normal((batch, n_small))
    W_s = g.standard_normal((batch, n_small, n_small))
    w_l = g.standard_normal(n_large)
    W_l = g.standard_normal((n_large, n_large))
    return dict(small=small, large=large, w_small=w_s, W_small=W_s, w_large=w_l,
                W_large=W_l, k=k)
