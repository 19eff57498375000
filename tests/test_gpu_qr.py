"""QR preprocessing of tall matrices (eq. (2.1)): G P = Q [R; 0] by blocked
Householder reflections on the GPU, the Jacobi method on R^T, U = Q [V_x; 0],
V = P U_x.  Checked against the oracle's SVD (one-sided Jacobi on G itself,
no QR) with the bars of test_gpu_parity.py, against the direct GPU path, for
ragged panel counts and sizes, for bitwise determinism, and for the
fallback to the direct path when R is singular."""
import numpy as np
import pytest

import oracle
from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _say(msg):
    print(msg, flush=True)


def _run(A, **kw):
    torch = _torch()
    from paper_1401_2720_amd import _binding as B
    U, S, V, info = B.gesvd(torch.from_numpy(np.asfortranarray(A)).cuda(), **kw)
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


def _check(A, U, S, V, ref, strict_rel=None):
    n = S.shape[0]
    tol = 1e-12 * ref + 1e-13 * ref[0]
    err = np.abs(S - ref)
    assert np.all(err <= tol), f"sigma: worst {np.max(err / np.maximum(tol, 1e-300)):.2f} x tol"
    if strict_rel is not None:
        big = ref >= 1e-3 * ref[0]
        assert np.max(err[big] / ref[big]) <= strict_rel
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)
    assert np.all(np.diff(S) <= 0)


QR_CASES = [
    # name, m, n, input kind
    ("tall300x70_graded", 300, 70, "graded"),      # 3 panels, the last of 6 columns
    ("tall1000x64_gauss", 1000, 64, "gauss"),      # 2 full panels, 2 panel workgroups
    ("tall2500x33_gauss", 2500, 33, "gauss"),      # a panel of 1 column, 5 workgroups
    ("square96_graded", 96, 96, "graded"),         # forced QR on a square matrix
    ("narrow700x5_gauss", 700, 5, "gauss"),
    # the largest m of the QR path: 64 panel workgroups, whose 64 partial sums
    # per column are gathered in one round trip
    ("tall32768x40_graded", 32768, 40, "graded"),
]


@pytest.mark.parametrize("name,m,n,kind", QR_CASES, ids=[c[0] for c in QR_CASES])
def test_qr_path_matches_oracle(name, m, n, kind):
    _say(f"qr case {name}: m={m} n={n}")
    g = inputs.rng(300 + m + n)
    A = (inputs.prescribed(m, n, inputs.logspaced(n, -6.0), g) if kind == "graded"
         else inputs.gaussian(m, n, g))
    U, S, V, info = _run(A, qr="on")
    assert info["status"] == 0 and info["preprocessed"] == 1, info
    ref = oracle.gesvj(A)
    _check(A, U, S, V, ref["S"], strict_rel=(1e-12 if kind == "gauss" else None))
    # the direct GPU path agrees
    U2, S2, V2, info2 = _run(A, qr="off")
    assert info2["preprocessed"] == 0
    assert np.max(np.abs(S - S2)) <= 1e-13 * S[0] * n
    _say(f"  sweeps qr={info['sweeps']} direct={info2['sweeps']}")


def test_qr_chosen_for_tall_and_deterministic():
    _say("qr auto choice and determinism")
    A = inputs.gaussian(800, 96, inputs.rng(41))
    r1 = _run(A)
    r2 = _run(A)
    assert r1[3]["preprocessed"] == 1
    for x, y in zip(r1[:3], r2[:3]):
        assert np.array_equal(x, y)
    r3 = _run(inputs.gaussian(150, 96, inputs.rng(42)))
    assert r3[3]["preprocessed"] == 0   # m < 2n: direct


def _rank_deficient(m, n, k, seed, zero_cols=0):
    """m x n of rank k: k Gaussian columns, the others random combinations
    of them (and zero_cols exactly zero columns among those)."""
    g = inputs.rng(seed)
    B = inputs.gaussian(m, k, g)
    A = np.concatenate([B, B @ g.standard_normal((k, n - k))], axis=1)
    if zero_cols:
        A[:, k:k + zero_cols] = 0.0
    return A[:, g.permutation(n)]


RD = [("rank100_of_120", 1000, 120, 100, 0),
      ("rank30_of_64_zero_columns", 500, 64, 30, 10),
      ("rank1_of_50", 400, 50, 1, 0),
      ("zero_column", 400, 40, 39, 1)]


@pytest.mark.parametrize("name,m,n,k,zc", RD, ids=[c[0] for c in RD])
def test_qr_rank_deficient_lq_path(name, m, n, k, zc):
    """Rank-deficient tall G keeps the QR path (eqs. (2.1)-(2.2)): pivoted QR
    of R, the LQ factorization of R_0, the Jacobi method on L_0; the k
    positive sigma against the oracle, the others zero, U's first k columns
    orthonormal and the others zero, V orthogonal, G = U Sigma V^T."""
    _say(f"qr rank deficient {name}: {m} x {n}, rank {k}")
    A = _rank_deficient(m, n, k, 43 + n, zc) if name != "zero_column" else None
    if A is None:
        A = inputs.gaussian(m, n, inputs.rng(43))
        A[:, 7] = 0.0
    U, S, V, info = _run(A, qr="on")
    assert info["status"] == 0
    assert info["preprocessed"] == 2 and info["rank"] == k, info
    assert np.all(S[k:] == 0.0) and np.all(S[:k] > 0) and np.all(np.diff(S) <= 0)
    assert np.all(U[:, k:] == 0.0)
    assert np.max(np.abs(U[:, :k].T @ U[:, :k] - np.eye(k))) <= 1e-13 * n
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)
    ref = oracle.gesvj(A)["S"]
    assert np.all(np.abs(S - ref) <= 1e-12 * ref + 1e-13 * ref[0]), \
        float(np.max(np.abs(S - ref) / (1e-12 * ref + 1e-13 * ref[0])))
    # A V_(k:) = 0: the last n - k columns of V span the null space
    assert np.linalg.norm(A @ V[:, k:]) <= 1e-13 * n * np.linalg.norm(A)
    _say(f"  sweeps={info['sweeps']}")


def test_qr_graded_full_rank_is_not_truncated():
    """Column groups 2^450 B1 and 2^-450 P2 (P2 orthogonal to B1): R's
    diagonal spans 2^900, but no column depends on the others, so the
    pivoted QR's scale-invariant rank test finds full rank and every sigma
    keeps its relative accuracy (the small group is not set to zero)."""
    _say("qr graded full rank")
    g = inputs.rng(45)
    B1, B2 = inputs.gaussian(300, 40, g), inputs.gaussian(300, 30, g)
    Q, _ = np.linalg.qr(B1)
    P2 = B2 - Q @ (Q.T @ B2)
    P2 = P2 - Q @ (Q.T @ P2)
    A = np.hstack([np.ldexp(B1, 450), np.ldexp(B2, -450)])
    s1 = np.ldexp(oracle.gesvj(B1)["S"], 450)
    s2 = np.ldexp(oracle.gesvj(P2)["S"], -450)
    U, S, V, info = _run(A, qr="on", scaled="off")
    assert info["status"] == 0 and info["rank"] == 70, info
    assert np.max(np.abs(S[:40] - s1) / s1) <= 1e-12
    assert np.max(np.abs(S[40:] - s2) / s2) <= 1e-12


def test_qr_zero_matrix_falls_back_to_direct():
    _say("qr zero matrix -> direct")
    A = np.zeros((300, 30))
    U, S, V, info = _run(A, qr="on")
    assert info["status"] == 0 and info["preprocessed"] == 0
    assert np.all(S == 0.0) and np.all(U == 0.0)
    assert np.max(np.abs(V.T @ V - np.eye(30))) <= 1e-13 * 30

def test_qr_path_reports_nan_input():
    """A NaN in a tall G on the QR path: R's diagonal is not finite, the call
    goes to the direct method, which reports JSVD_NONFINITE (3)."""
    _say("qr nan input")
    A = inputs.gaussian(400, 40, inputs.rng(44))
    A[11, 5] = np.nan
    _, _, _, info = _run(A, qr="on", allow=(1, 2, 3))
    assert info["status"] == 3
