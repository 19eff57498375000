"""Pins for the oracle's hyperbolic SVD (eq. (2.10); Section 4.3, subphase 4).

G = U Sigma V^{-1} with V^T J V = J, J = diag(I_{n+}, -I).  Checks: the
eigenvalues of G J G^T are j_i sigma_i^2 (the accuracy measure (6.1) of
Section 6) computed in 40-digit arithmetic; the J-orthogonality of V; G V =
U Sigma; the J-weighted trace invariant; and the special cases J = I and
J = -I, which contain no mixed pair and so no hyperbolic rotation.
"""
import mpmath
import numpy as np
import pytest

import oracle

EPS = 2.0 ** -53


def _jvec(n, n_plus):
    return np.concatenate([np.ones(n_plus), -np.ones(n - n_plus)])


def _eig_gjgt(G, j):
    mpmath.mp.dps = 40
    M = mpmath.matrix(G.tolist())
    Jm = mpmath.diag([mpmath.mpf(float(x)) for x in j])
    E = mpmath.eigsy(M * Jm * M.T, eigvals_only=True)
    return np.array([float(e) for e in E])


def test_2x2_hyperbolic_closed_form():
    g = np.random.default_rng(21)
    for _ in range(50):
        G = g.standard_normal((2, 2))
        r = oracle.gesvj(G, n_plus=1)
        lam = np.sort(_eig_gjgt(G, [1, -1]))[::-1]
        got = np.array([r["S"][0] ** 2, -r["S"][1] ** 2])
        scale = np.max(np.abs(lam))
        kappa = np.linalg.cond(G / np.linalg.norm(G, axis=0))
        assert np.max(np.abs(got - lam)) <= 64 * EPS * kappa ** 2 * scale


@pytest.mark.parametrize("m,n,n_plus", [(12, 10, 6), (16, 16, 4), (20, 14, 13)])
def test_eigenvalues_of_gjgt(m, n, n_plus):
    g = np.random.default_rng(22 + n)
    G = g.standard_normal((m, n))
    r = oracle.gesvj(G, n_plus=n_plus)
    assert r["converged"]
    j = _jvec(n, n_plus)
    lam = _eig_gjgt(G, j)
    lam = lam[np.argsort(-np.abs(lam))][:n]  # the n non-zero eigenvalues
    got = j * r["S"] ** 2
    scale = np.max(np.abs(lam))
    assert np.max(np.abs(np.sort(got) - np.sort(lam))) <= 1e-12 * scale


@pytest.mark.parametrize("order", ["row", "rr"])
def test_hsvd_invariants(order):
    g = np.random.default_rng(23)
    m, n, n_plus = 60, 48, 30
    G = g.standard_normal((m, n))
    r = oracle.gesvj(G, n_plus=n_plus, order=order)
    U, S, V = r["U"], r["S"], r["V"]
    j = _jvec(n, n_plus)
    assert r["converged"]
    vmax = max(1.0, np.max(np.abs(V)) ** 2)
    assert np.max(np.abs(V.T @ (j[:, None] * V) - np.diag(j))) <= 1e-13 * n * vmax
    assert np.linalg.norm(G @ V - U * S) <= 1e-13 * n * np.linalg.norm(G) * np.linalg.norm(V, 2)
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
    # sum_j j_i ||g_i||^2 = sum_i j_i sigma_i^2 (trace of G J G^T)
    t0 = np.sum(j * np.sum(G ** 2, axis=0))
    assert abs(np.sum(j * S ** 2) - t0) <= 1e-13 * n * np.sum(G ** 2)
    # output order: positive part non-increasing, negative part non-decreasing
    assert np.all(np.diff(S[:n_plus]) <= 0) and np.all(np.diff(S[n_plus:]) >= 0)
    assert r["rotations"] > 0


def test_identity_signature_is_the_svd():
    g = np.random.default_rng(24)
    G = g.standard_normal((30, 20))
    a = oracle.gesvj(G)
    b = oracle.gesvj(G, n_plus=20)
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["V"], b["V"])


def test_negative_signature_uses_trig_rotations_only():
    g = np.random.default_rng(25)
    G = g.standard_normal((30, 20))
    a = oracle.gesvj(G)
    b = oracle.gesvj(G, n_plus=0)
    assert b["clamps"] == 0
    assert np.array_equal(np.sort(a["S"]), b["S"])  # same rotations, ascending order
