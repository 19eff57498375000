"""GPU checks of the differentiable SVD (JacobiSVD / jsvd_svd_backward).

Loss L = sum_i w_i sigma_i + ||U_k V_k^T o W||_F^2 (k = 8), seeded N(0,1)
weights, matrices Q1 diag(1 + 0.01 i) Q2^T.  Bars: the backward against the
oracle adjoint built from the oracle's SVD (relative 1e-9 in the Frobenius
norm), against central finite differences with h = 1e-6 along seeded random
directions (relative 1e-6), and the closed form dL/dA = U diag(w) V^T when
W = 0.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint
from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _loss(U, S, V, w, W, k):
    P = U[..., :, :k] @ V[..., :, :k].transpose(-1, -2)
    return (w * S).sum() + ((P * W) ** 2).sum()


def _grad(A, w, W, k, recompute=False):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    X = A.clone().requires_grad_(True)
    U, S, V = jsvd.svd(X, recompute=recompute)
    L = _loss(U, S, V, w, W, k)
    L.backward()
    return float(L), X.grad.detach().clone()


def _value(A, w, W, k):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    with torch.no_grad():
        U, S, V = jsvd.svd(A)
        return float(_loss(U, S, V, w, W, k))


def _fd_check(A, w, W, k, grad, seed, ndir=3, h=1e-6):
    torch = _torch()
    g = torch.Generator(device="cpu").manual_seed(seed)
    for _ in range(ndir):
        E = torch.randn(A.shape, generator=g, dtype=torch.float64).to(A.device)
        fd = (_value(A + h * E, w, W, k) - _value(A - h * E, w, W, k)) / (2 * h)
        an = float((grad * E).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1.0), (fd, an)


def _oracle_grad(A, w, W, k):
    r = oracle.gesvj(A)
    _, dU, ds, dV = adjoint.loss_and_grads(r["U"], r["S"], r["V"], w, W, k)
    return adjoint.svd_adjoint(r["U"], r["S"], r["V"], dU, ds, dV)


@pytest.mark.parametrize("b,m,n", [(8, 64, 64), (4, 96, 64), (3, 40, 17)])
def test_batched_backward_against_oracle_and_fd(b, m, n):
    torch = _torch()
    print(f"backward batch {b} x {m}x{n}", flush=True)
    g = inputs.rng(60 + m + n)
    sig = 1.0 + 0.01 * np.arange(n)
    A = np.stack([inputs.prescribed(m, n, sig, g) for _ in range(b)])
    w = g.standard_normal((b, n))
    W = g.standard_normal((b, m, n))
    k = min(8, n)
    At = torch.from_numpy(A).cuda()
    wt, Wt = torch.from_numpy(w).cuda(), torch.from_numpy(W).cuda()
    _, grad = _grad(At, wt, Wt, k)
    gh = grad.cpu().numpy()
    for i in range(b):
        ref = _oracle_grad(A[i], w[i], W[i], k)
        assert np.linalg.norm(gh[i] - ref) <= 1e-9 * np.linalg.norm(ref), i
    _fd_check(At, wt, Wt, k, grad, seed=b + m + n)
    _, grad_rc = _grad(At, wt, Wt, k, recompute=True)
    assert torch.equal(grad, grad_rc)


def test_sigma_only_closed_form():
    """W = 0: dL/dA = U diag(w) V^T exactly (d sigma_i = u_i v_i^T dA v... )."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    g = inputs.rng(71)
    A = torch.from_numpy(inputs.prescribed(128, 100, 1.0 + 0.01 * np.arange(100), g)).cuda()
    w = torch.from_numpy(g.standard_normal(100)).cuda()
    X = A.clone().requires_grad_(True)
    U, S, V = jsvd.svd(X)
    (w * S).sum().backward()
    ref = (U * w) @ V.t()
    assert float((X.grad - ref).abs().max()) <= 1e-13 * float(ref.abs().max()) * 100


def test_large_single_backward_fd():
    """One 1024 x 1024 matrix of the differentiable workload."""
    torch = _torch()
    d = inputs.differentiable_set(batch=1, n_small=8)
    print("backward 1024 x 1024", flush=True)
    A = torch.from_numpy(d["large"]).cuda()
    w = torch.from_numpy(d["w_large"]).cuda()
    W = torch.from_numpy(d["W_large"]).cuda()
    L, grad = _grad(A, w, W, d["k"])
    assert np.isfinite(L)
    _fd_check(A, w, W, d["k"], grad, seed=5, ndir=2)


def test_differentiable_workload_256x64x64():
    """The differentiable workload's batch itself: 256 matrices 64 x 64 with
    sigma_i = 1 + 0.01 i (seed 6), every gradient against the oracle adjoint,
    the batch loss against central differences."""
    torch = _torch()
    d = inputs.differentiable_set()
    print("backward 256 x 64x64", flush=True)
    A, w, W, k = d["small"], d["w_small"], d["W_small"], d["k"]
    At = torch.from_numpy(A).cuda()
    wt, Wt = torch.from_numpy(w).cuda(), torch.from_numpy(W).cuda()
    _, grad = _grad(At, wt, Wt, k)
    gh = grad.cpu().numpy()
    worst = 0.0
    for i in range(A.shape[0]):
        ref = _oracle_grad(A[i], w[i], W[i], k)
        rel = np.linalg.norm(gh[i] - ref) / np.linalg.norm(ref)
        worst = max(worst, rel)
        assert rel <= 1e-9, (i, rel)
    print(f"  worst relative gradient error {worst:.2e}", flush=True)
    _fd_check(At, wt, Wt, k, grad, seed=256, ndir=2)
