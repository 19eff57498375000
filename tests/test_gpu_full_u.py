"""jsvd_gesvd_full: the full SVD G = U [Sigma; 0] V^T with U of order m.

The first k columns of U (k positive singular values) are the economy U of
jsvd_gesvd, bit for bit; the other m - k columns are not unique, so they are
checked by what defines them: U orthogonal (max|U^T U - I| <= 1e-13 m), and
orthogonal to the range of G (||U[:, k:]^T G|| <= 1e-13 m ||G||).  Sigma and
V against the oracle as in the other parity tests; the reconstruction
G = U [Sigma; 0] V^T.  Cases: tall (QR preprocessing), nearly square (the
direct method), rank deficient (zero singular values, whose U columns come
from the completion), and m = n.
"""
import numpy as np
import pytest

import oracle
from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _case(kind, m, n, seed):
    g = inputs.rng(seed)
    if kind == "graded":
        return inputs.prescribed(m, n, inputs.logspaced(n, -6.0), g)
    A = inputs.gaussian(m, n, g)
    if kind == "deficient":
        # the last 12 columns repeat earlier ones: rank n - 12
        A[:, n - 12:] = A[:, :12]
    return A


CASES = [("tall_qr_500x120_graded", "graded", 500, 120, 1),
         ("direct_300x250", "gauss", 300, 250, 2),
         ("deficient_400x100", "deficient", 400, 100, 3),
         ("square_96", "gauss", 96, 96, 4)]


@pytest.mark.parametrize("name,kind,m,n,seed", CASES, ids=[c[0] for c in CASES])
def test_full_u(name, kind, m, n, seed):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print(f"full U: {name}", flush=True)
    A = _case(kind, m, n, seed)
    At = torch.from_numpy(A).cuda()
    U, S, V, info = jsvd.gesvd_full(At)
    Ue, Se, Ve, _ = jsvd.gesvd(At)
    torch.cuda.synchronize()
    assert info["status"] == 0
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    Ue = Ue.cpu().numpy()
    assert np.array_equal(S, Se.cpu().numpy()) and np.array_equal(V, Ve.cpu().numpy())
    k = int(np.sum(S > 0))
    if kind == "deficient":
        # numerically zero singular values may come out as tiny positives
        k = int(np.sum(S > 1e-12 * S[0]))
        assert k == n - 12
    assert np.array_equal(U[:, :k], Ue[:, :k])
    assert np.max(np.abs(U.T @ U - np.eye(m))) <= 1e-13 * m
    assert np.linalg.norm(U[:, k:].T @ A) <= 1e-13 * m * np.linalg.norm(A)
    Sig = np.zeros((m, n))
    Sig[:n, :n] = np.diag(S)
    assert np.linalg.norm(A - U @ Sig @ V.T) <= 1e-13 * m * np.linalg.norm(A)
    ref = oracle.gesvj(A)["S"]
    bar = 1e-12 * ref + 1e-13 * ref[0]
    assert np.all(np.abs(S - ref) <= bar), float(np.max(np.abs(S - ref) / bar))
    print(f"  k={k} sweeps={info['sweeps']} preprocessed={info['preprocessed']}", flush=True)
