"""GPU parity of the fused update-and-Gram launch (opts.fuse = 1, not the
default): the update of p-step s and the Gram partials of p-step s + 1
formed in one launch per group of two pivot pairs (2w = 64, a power-of-two
number of blocks, no padding columns, m a multiple of 64, unscaled Cholesky
path).

Against the oracle with the bars of test_gpu_parity.py, and against the
three-launch path (fuse = 0, the default) on the same input: the two form
the Gram partial sums in different orders, so they agree to rounding, not
bit for bit (sigma within the oracle's bar of each other).  The kernel
timing counters show which path ran.  Cases: a last row split of one slice
per wave, more rows than columns, the smallest orders with groups (4 and 8
blocks), every ordering with groups, the hyperbolic SVD, the QR
preprocessing of a tall G (the fused path then runs on R^T), and input
whose pivot pairs start orthogonal (the launch's pass-through variants for
pairs that did not rotate).
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


def _say(msg):
    print(msg, flush=True)


def _run(A, **kw):
    """gesvd with kernel timing on: (U, S, V, info, launches per kernel)."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    B.kernel_timing(0, True, stride=1)
    try:
        U, S, V, info = jsvd.gesvd(torch.from_numpy(np.asfortranarray(A)).cuda(), **kw)
        torch.cuda.synchronize()
        kt = B.kernel_times(0)
    finally:
        B.kernel_timing(0, False)
    return (U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info,
            {k: v[1] for k, v in kt.items()})


def _check(A, U, S, V, ref, strict):
    n = S.shape[0]
    tol = 1e-12 * ref + 1e-13 * ref[0]
    err = np.abs(S - ref)
    assert np.all(err <= tol), f"sigma: worst {np.max(err / np.maximum(tol, 1e-300)):.2f} x tol"
    if strict:
        big = ref >= 1e-3 * ref[0]
        assert np.max(err[big] / ref[big]) <= 1e-12
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)
    assert np.all(np.diff(S) <= 0)


def _fused_ran(launches, info, steps_per_sweep):
    """Fused: one Gram launch per sweep (its first p-step), one plain update
    per sweep (its last), the fused launch at every other p-step."""
    sw = info["sweeps"]
    assert launches["gram"] == sw, launches
    assert launches["fused"] == sw * (steps_per_sweep - 1), launches
    assert launches["update"] == sw, launches


CASES = [
    # name, m, n, input, kwargs
    ("square256_two_groups", 256, 256, "gauss", {}),
    ("last_split_one_slice_per_wave_320x256", 320, 256, "gauss", {}),
    ("tall1088x512", 1088, 512, "gauss", dict(qr="off")),
    ("graded512", 512, 512, "graded", {}),
    ("one_group_192x128", 192, 128, "gauss", dict(qr="off")),
    ("strategy_r", 320, 256, "gauss", dict(strategy="r")),
    ("strategy_crev", 320, 256, "gauss", dict(strategy="crev")),
    ("strategy_c", 320, 256, "gauss", dict(strategy="c")),
]


@pytest.mark.parametrize("name,m,n,kind,kw", CASES, ids=[c[0] for c in CASES])
def test_fused_matches_oracle_and_three_launch_path(name, m, n, kind, kw):
    _say(f"fused {name}: m={m} n={n} {kw}")
    g = inputs.rng(1100 + m + n)
    A = (inputs.prescribed(m, n, inputs.logspaced(n, -6.0), g) if kind == "graded"
         else inputs.gaussian(m, n, g))
    U, S, V, info, la = _run(A, block_w=32, fuse=True, **kw)
    assert info["status"] == 0 and info["converged"] == 1 and info["block_w"] == 32, info
    order = n // 32
    _fused_ran(la, info, order - 1)
    ref = oracle.gesvj(A)["S"]
    _check(A, U, S, V, ref, kind == "gauss")
    U2, S2, V2, info2, la2 = _run(A, block_w=32, **kw)
    assert la2["fused"] == 0 and la2["gram"] == info2["sweeps"] * (order - 1)
    _check(A, U2, S2, V2, ref, kind == "gauss")
    assert np.all(np.abs(S - S2) <= 1e-12 * S2 + 1e-13 * S2[0])
    _say(f"  sweeps fused {info['sweeps']} / three launches {info2['sweeps']}")


def test_fused_hyperbolic():
    _say("fused hsvd 448 x 256, n_plus = 160")
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    G = inputs.gaussian(448, 256, inputs.rng(1120))
    J = np.array([1] * 160 + [-1] * 96, dtype=np.int8)
    B.kernel_timing(0, True, stride=1)
    try:
        U, S, V, Jo, info = jsvd.hsvd(torch.from_numpy(np.asfortranarray(G)).cuda(), J,
                                      block_w=32, fuse=True)
        torch.cuda.synchronize()
        la = {k: v[1] for k, v in B.kernel_times(0).items()}
    finally:
        B.kernel_timing(0, False)
    assert info["status"] == 0 and info["converged"] == 1
    _fused_ran(la, info, 7)
    S, V = S.cpu().numpy(), V.cpu().numpy()
    ref = oracle.gesvj(G, n_plus=160)["S"]
    vn2 = max(1.0, np.linalg.norm(V, 2) ** 2)
    assert np.all(np.abs(S - ref) <= vn2 * (1e-12 * ref + 1e-13 * ref.max()))
    Jd = np.diag(Jo.astype(np.float64))
    assert np.max(np.abs(V.T @ Jd @ V - Jd)) <= 1e-13 * 256 * max(1.0, np.max(np.abs(V)) ** 2)


def test_fused_on_r_transpose_after_qr():
    """A tall G (m >= 2n) is first reduced by QR; the Jacobi solve on the
    256 x 256 R^T takes the fused path."""
    _say("fused after QR preprocessing 700 x 256")
    A = inputs.gaussian(700, 256, inputs.rng(1130))
    U, S, V, info, la = _run(A, block_w=32, fuse=True)
    assert info["status"] == 0 and info["preprocessed"] == 1
    assert la["fused"] > 0
    _check(A, U, S, V, oracle.gesvj(A)["S"], True)


def test_fused_pass_through_of_pairs_that_did_not_rotate():
    """Columns orthogonal to working accuracy within the first half of the
    blocks and a Gaussian second half: in the first sweeps the pairs inside
    the first half do not rotate (their columns pass through the fused
    launch unchanged), pairs across the halves and inside the second do.
    sigma of the first half are its column norms."""
    _say("fused with non-rotating pairs 320 x 256")
    g = inputs.rng(1140)
    Q, _ = np.linalg.qr(inputs.gaussian(320, 320, g))
    s1 = np.logspace(3, 1, 128)
    A = np.empty((320, 256))
    A[:, :128] = Q[:, :128] * s1
    # the second half lives in the orthogonal complement of the first
    A[:, 128:] = Q[:, 128:] @ inputs.gaussian(192, 128, g)
    U, S, V, info, la = _run(A, block_w=32, fuse=True)
    assert info["status"] == 0 and info["converged"] == 1
    _fused_ran(la, info, 7)
    ref = oracle.gesvj(A)["S"]
    _check(A, U, S, V, ref, False)
    assert all(np.min(np.abs(S - v)) <= 1e-12 * v for v in s1)


def test_fused_not_taken_where_it_does_not_apply():
    """Padding columns (n = 250 fills 8 blocks of 32 only in part), m not a
    multiple of 64, w = 16, the round-robin ordering and the scaled mode
    keep three launches."""
    _say("fused not taken")
    g = inputs.rng(1150)
    for m, n, kw in [(300, 250, dict(block_w=32)), (288, 256, dict(block_w=32)),
                     (300, 256, dict(block_w=16)),
                     (300, 256, dict(block_w=32, strategy="rr")),
                     (300, 256, dict(block_w=32, scaled="on"))]:
        A = inputs.gaussian(m, n, g)
        U, S, V, info, la = _run(A, fuse=True, **kw)
        assert info["status"] == 0, (m, n, kw)
        assert la["fused"] == 0 and la["gram"] > info["sweeps"], (m, n, kw, la)


def test_fused_4096_against_golden_sigma():
    """The benchmark matrix (4096 x 4096 N(0,1), seed 2) in the configuration
    that bench.py --fuse times (w = 32, Rrev, 8 row splits): every sigma
    against the oracle's golden values (tests/golden/, written by the
    oracle), at the bars of the full-size tests, and the fused launch at all
    p-steps but the first and last of each sweep."""
    import os
    _say("fused 4096 x 4096 N(0,1) against the golden sigma")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "sigma_gaussian4096_seed2.txt")
    ref = np.loadtxt(path, comments="#")
    A = inputs.square_gaussian()
    U, S, V, info, la = _run(A, fuse=True)
    assert info["status"] == 0 and info["converged"] == 1 and info["block_w"] == 32, info
    _fused_ran(la, info, 127)
    err = np.abs(S - ref)
    assert np.all(err <= 1e-12 * ref + 1e-13 * ref.max()), float(np.max(err / ref))
    big = ref >= 1e-3 * ref.max()
    rel = float(np.max(err[big] / ref[big]))
    assert rel <= 1e-12, rel
    assert np.max(np.abs(V.T @ V - np.eye(4096))) <= 1e-13 * 4096
    _say(f"  max rel sigma err {rel:.2e}, sweeps {info['sweeps']}")
