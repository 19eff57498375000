"""Full-size workloads, checked by properties that hold at any size (the oracle
is too slow there) and by singular triplets sampled one by one:

  * 4096 x 4096 N(0,1), the benchmark configuration: sum sigma^2 = ||A||_F^2,
    U^T U = I, V^T V = I, A V = U Sigma, and for sampled i the residuals
    ||A v_i - s_i u_i||, ||A^T u_i - s_i v_i|| (each triplet is a singular
    triplet of A to the method's accuracy);
  * 8192 x 2048 with prescribed sigma log-spaced 1 .. 1e-10: sigma against the
    prescribed values within the representation error of A;
  * hyperbolic 2048 x 2048, J = diag(+1 x 1280, -1 x 768): j_i sigma_i^2
    against the eigenvalues of G J G^T (LAPACK, normwise), V^T J V = J and
    G V = U Sigma.
Bars as in test_gpu_parity.py.
"""
import numpy as np
import pytest

from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _orth(X):
    torch = _torch()
    n = X.shape[1]
    return float((X.t().contiguous() @ X - torch.eye(n, dtype=X.dtype, device=X.device)).abs().max())


def test_square_gaussian_4096():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print("4096 x 4096 N(0,1)", flush=True)
    A = torch.from_numpy(inputs.square_gaussian()).cuda()
    U, S, V, info = jsvd.gesvd(A)
    torch.cuda.synchronize()
    n = 4096
    assert info["status"] == 0 and info["converged"] == 1
    fro2 = float((A * A).sum())
    assert abs(float((S * S).sum()) - fro2) <= 1e-13 * n * fro2
    assert _orth(U) <= 1e-13 * n and _orth(V) <= 1e-13 * n
    res = float(torch.linalg.norm(A @ V - U * S) / torch.linalg.norm(A))
    assert res <= 1e-13 * n
    assert bool((S[1:] <= S[:-1]).all())
    s1 = float(S[0])
    for i in [0, 1, 100, 2047, 4000, 4095]:
        r1 = float(torch.linalg.norm(A @ V[:, i] - S[i] * U[:, i]))
        r2 = float(torch.linalg.norm(A.t() @ U[:, i] - S[i] * V[:, i]))
        assert r1 <= 1e-13 * n * s1 and r2 <= 1e-13 * n * s1, i


def test_tall_graded_8192x2048():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print("8192 x 2048, sigma 1 .. 1e-10", flush=True)
    A = torch.from_numpy(inputs.tall_graded()).cuda()
    U, S, V, info = jsvd.gesvd(A)
    torch.cuda.synchronize()
    assert info["status"] == 0
    sig = inputs.logspaced(2048, -10.0)
    s = S.cpu().numpy()
    eps = 2.0 ** -53
    # A = Q1 diag(sig) Q2^T in fp64 carries an error of order eps ||A|| sqrt(n)
    assert np.max(np.abs(s - sig)) <= 100 * eps * np.sqrt(2048)
    assert np.max(np.abs(s - sig)[sig >= 1e-3] / sig[sig >= 1e-3]) <= 1e-12
    assert _orth(V) <= 1e-13 * 2048
    res = float(torch.linalg.norm(A @ V - U * S) / torch.linalg.norm(A))
    assert res <= 1e-13 * 2048


def test_hyperbolic_2048():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print("hyperbolic 2048 x 2048, n+ = 1280", flush=True)
    G, J = inputs.hyperbolic_gaussian()
    Gt = torch.from_numpy(G).cuda()
    U, S, V, Jout, info = jsvd.hsvd(Gt, J)
    torch.cuda.synchronize()
    assert info["status"] == 0
    n = 2048
    j = torch.from_numpy(J.astype(np.float64)).cuda()
    vmax = max(1.0, float(V.abs().max()) ** 2)
    jo = torch.from_numpy(Jout.astype(np.float64)).cuda()
    vjv = V.t().contiguous() @ (j[:, None] * V)
    assert float((vjv - torch.diag(jo)).abs().max()) <= 1e-13 * n * vmax
    vn = float(torch.linalg.matrix_norm(V, ord=2))
    res = float(torch.linalg.norm(Gt @ V - U * S) / (torch.linalg.norm(Gt) * vn))
    assert res <= 1e-13 * n
    lam = np.linalg.eigvalsh((G * J) @ G.T)
    got = np.sort(Jout * S.cpu().numpy() ** 2)
    assert np.max(np.abs(got - np.sort(lam))) <= 1e-12 * np.max(np.abs(lam)) * vmax


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    return np.loadtxt(path, comments="#")


def _sigma_gate(s, ref, strict_from=1e-3):
    """The sigma bars: |s - s_orc| <= 1e-12 s_orc + 1e-13 s_orc[0] for every
    i, and relative 1e-12 outright for s_orc >= 1e-3 s_orc.max()."""
    err = np.abs(s - ref)
    assert np.all(err <= 1e-12 * ref + 1e-13 * ref.max()), float(np.max(err / ref))
    big = ref >= strict_from * ref.max()
    rel = float(np.max(err[big] / ref[big]))
    assert rel <= 1e-12, rel
    return rel


def test_square_gaussian_4096_sigma_against_oracle():
    """The benchmark workload's singular values against the oracle's
    (round-robin order run to convergence, tests/golden/make_sigma_golden.py),
    elementwise, in the launch configuration the benchmark times."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print("4096 x 4096 N(0,1): sigma against the oracle", flush=True)
    ref = _golden("sigma_gaussian4096_seed2.txt")
    A = torch.from_numpy(inputs.square_gaussian()).cuda()
    _, S, _, info = jsvd.gesvd(A)
    torch.cuda.synchronize()
    assert info["status"] == 0
    rel = _sigma_gate(S.cpu().numpy(), ref)
    print(f"  max rel sigma err {rel:.2e}", flush=True)


def test_square_gaussian_4096_one_buffer_gram_against_oracle():
    """The same with 16 Gram row splits (a tuning table with 1024 Gram
    workgroups per launch): 1024 workgroups are more than two per CU, so the
    Gram kernel takes its one-buffer loop instead of the two-buffer pipeline
    of the default 4 splits, and the inner kernel sums 16 partials."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    print("4096 x 4096 N(0,1), 16 Gram splits: sigma against the oracle", flush=True)
    ref = _golden("sigma_gaussian4096_seed2.txt")
    A = torch.from_numpy(inputs.square_gaussian()).cuda()
    table = {"n_upper": [8192], "block_w": [32], "gram_wg": [1024], "update_wg": [1024],
             "batch_g_groups": 0, "batch_block_min_n": 0}
    B.set_tuning(0, table)
    try:
        _, S, _, info = jsvd.gesvd(A)
        torch.cuda.synchronize()
    finally:
        B.set_tuning(0, B.load_tuning(0))
    assert info["status"] == 0 and info["block_w"] == 32
    rel = _sigma_gate(S.cpu().numpy(), ref)
    print(f"  max rel sigma err {rel:.2e}", flush=True)


def test_hyperbolic_2048_sigma_against_oracle():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print("hyperbolic 2048 x 2048: sigma against the oracle", flush=True)
    ref = _golden("sigma_hsvd2048_p1280_seed4.txt")
    G, J = inputs.hyperbolic_gaussian()
    _, S, _, Jout, info = jsvd.hsvd(torch.from_numpy(G).cuda(), J)
    torch.cuda.synchronize()
    assert info["status"] == 0
    assert np.array_equal(Jout, J)
    s = S.cpu().numpy()
    # each part in its own order (positive part non-increasing, negative
    # part non-decreasing): compare part by part
    rel_p = _sigma_gate(s[:1280], ref[:1280])
    rel_m = _sigma_gate(s[1280:], ref[1280:])
    print(f"  max rel sigma err +part {rel_p:.2e} -part {rel_m:.2e}", flush=True)
