"""Pins for the SVD adjoint oracle: central finite differences through the
oracle's forward SVD (the same losses the GPU backward is checked with)."""
import numpy as np

import oracle
from oracle import adjoint
from paper_1401_2720_amd import inputs


def _loss(A, w, W, k):
    r = oracle.gesvj(A)
    return adjoint.loss_and_grads(r["U"], r["S"], r["V"], w, W, k)[0]


def test_sigma_gradient_is_outer_product():
    """d sigma_i / dA = u_i v_i^T, checked by finite differences of sigma_i."""
    g = np.random.default_rng(41)
    A = inputs.prescribed(12, 9, 1.0 + 0.1 * np.arange(9), g)
    r = oracle.gesvj(A)
    h = 1e-6
    for i in (0, 4, 8):
        grad = adjoint.svd_adjoint(r["U"], r["S"], r["V"], ds=np.eye(9)[i])
        E = g.standard_normal(A.shape)
        fd = (oracle.gesvj(A + h * E)["S"][i] - oracle.gesvj(A - h * E)["S"][i]) / (2 * h)
        assert abs(fd - np.sum(grad * E)) <= 1e-8 * max(1.0, abs(fd))
        assert np.allclose(grad, np.outer(r["U"][:, i], r["V"][:, i]), atol=1e-14)


def test_full_loss_finite_differences():
    g = np.random.default_rng(42)
    for (m, n) in [(10, 10), (14, 9)]:
        A = inputs.prescribed(m, n, 1.0 + 0.05 * np.arange(n), g)
        w = g.standard_normal(n)
        W = g.standard_normal((m, n))
        k = 4
        r = oracle.gesvj(A)
        _, dU, ds, dV = adjoint.loss_and_grads(r["U"], r["S"], r["V"], w, W, k)
        grad = adjoint.svd_adjoint(r["U"], r["S"], r["V"], dU, ds, dV)
        h = 1e-6
        for _ in range(4):
            E = g.standard_normal(A.shape)
            fd = (_loss(A + h * E, w, W, k) - _loss(A - h * E, w, W, k)) / (2 * h)
            an = np.sum(grad * E)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (m, n, fd, an)


def test_projector_term_matters_for_tall():
    """For m > n the (I - U U^T) dU term is not zero; dropping it breaks the
    finite-difference agreement (pins that term)."""
    g = np.random.default_rng(43)
    m, n, k = 16, 6, 3
    A = inputs.prescribed(m, n, 1.0 + 0.2 * np.arange(n), g)
    w = np.zeros(n)
    W = g.standard_normal((m, n))
    r = oracle.gesvj(A)
    _, dU, ds, dV = adjoint.loss_and_grads(r["U"], r["S"], r["V"], w, W, k)
    full = adjoint.svd_adjoint(r["U"], r["S"], r["V"], dU, ds, dV)
    proj = (np.eye(m) - r["U"] @ r["U"].T) @ dU / r["S"][None, :] @ r["V"].T
    assert np.linalg.norm(proj) > 1e-3 * np.linalg.norm(full)
    E = g.standard_normal(A.shape)
    h = 1e-6
    fd = (_loss(A + h * E, w, W, k) - _loss(A - h * E, w, W, k)) / (2 * h)
    assert abs(fd - np.sum(full * E)) <= 1e-7 * max(1.0, abs(fd))
    assert abs(fd - np.sum((full - proj) * E)) > 1e-5 * max(1.0, abs(fd))
