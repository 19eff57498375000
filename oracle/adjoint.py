"""Oracle for the SVD adjoint (reverse-mode derivative): test infrastructure.

The paper has no backward.  This is the published adjoint of the economy
SVD A = U diag(s) V^T (m >= n, distinct singular values), written out as
defined, with numpy matrix products:

  F_ij = 1 / (s_j^2 - s_i^2) for i != j, F_ii = 0,
  J = U^T dU,  K = V^T dV,
  dA = U [diag(ds) + (F o (J - J^T)) diag(s) + diag(s) (F o (K - K^T))] V^T
       + (I - U U^T) dU diag(s)^{-1} V^T.

Pinned by central finite differences of losses through the oracle's forward
SVD (tests/test_oracle_adjoint.py).
"""
import numpy as np


def svd_adjoint(U, s, V, dU=None, ds=None, dV=None):
    m, n = U.shape
    S2 = s * s
    with np.errstate(divide="ignore"):
        F = 1.0 / (S2[None, :] - S2[:, None])
    F[np.arange(n), np.arange(n)] = 0.0
    M = np.diag(ds) if ds is not None else np.zeros((n, n))
    extra = np.zeros((m, n))
    if dU is not None:
        J = U.T @ dU
        M = M + (F * (J - J.T)) * s[None, :]
        extra = (np.eye(m) - U @ U.T) @ dU / s[None, :]
    if dV is not None:
        K = V.T @ dV
        M = M + s[:, None] * (F * (K - K.T))
    return U @ M @ V.T + extra @ V.T


def loss_and_grads(U, s, V, w, W, k):
    """L = sum_i w_i s_i + ||U_k V_k^T o W||_F^2 and its adjoints (dU, ds, dV)."""
    P = U[:, :k] @ V[:, :k].T
    L = float(w @ s + np.sum((P * W) ** 2))
    GP = 2.0 * P * W * W
    dU = np.zeros_like(U)
    dV = np.zeros_like(V)
    dU[:, :k] = GP @ V[:, :k]
    dV[:, :k] = GP.T @ U[:, :k]
    return L, dU, w.copy(), dV
