"""GPU parity: the HIP path through the C ABI against the oracle.

Bars (floating point; the method is iterative, so the two sides follow
different but valid pivot orders and agree to the accuracy the method
guarantees, not bit for bit):
  * sigma: |s - s_orc| <= 1e-12 s_orc + 1e-13 s_orc[0] elementwise, and
    1e-12 relative for s >= 1e-3 s[0] on unstructured inputs;
  * orthogonality: max|U^T U - I|, max|V^T V - I| <= 1e-13 n;
  * reconstruction: ||A - U S V^T||_F / ||A||_F <= 1e-13 n;
  * singular vectors, after aligning signs, for well separated sigma:
    ||v - v_orc|| <= 1e-12 s[0] / gap;
  * hyperbolic SVD: max|V^T J V - J| <= 1e-13 n max(1, max|V|^2) and
    ||G V - U S||_F <= 1e-13 n ||G||_F ||V||_2 (both scale with the size of
    the J-orthogonal V), sigma as above.
Integer outputs (strategy tables) are compared exactly in test_abi.py.
"""
import numpy as np
import pytest

import oracle
from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _jsvd():
    import paper_1401_2720_amd as jsvd
    jsvd.lib()
    return jsvd


def _say(msg):
    print(msg, flush=True)


def _run_gesvd(A, **kw):
    torch = _torch()
    jsvd = _jsvd()
    U, S, V, info = jsvd.gesvd(torch.from_numpy(np.asfortranarray(A)).cuda(), **kw)
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), (None if V is None else V.cpu().numpy()), info


def _check_sigma(s, ref, scale=1.0, strict_rel=None):
    tol = scale * (1e-12 * ref + 1e-13 * ref[0])
    err = np.abs(s - ref)
    assert np.all(err <= tol), f"sigma: worst {np.max(err / np.maximum(tol, 1e-300)):.2f} x tol"
    if strict_rel is not None:
        big = ref >= 1e-3 * ref[0]
        assert np.max(err[big] / ref[big]) <= strict_rel


def _check_svd(A, U, S, V, n):
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)
    assert np.all(np.diff(S) <= 0)


def _check_vectors(X, Xr, S):
    n = S.shape[0]
    for i in range(n):
        gap = np.min(np.abs(np.delete(S, i) - S[i])) if n > 1 else S[0]
        if gap < 1e-8 * S[0]:
            continue
        x, y = X[:, i], Xr[:, i]
        sgn = 1.0 if x @ y >= 0 else -1.0
        assert np.linalg.norm(x - sgn * y) <= 1e-12 * S[0] / gap + 1e-13 * n, i


def test_fp64_division_and_sqrt_correctly_rounded():
    """Section 4 assumes correctly rounded / and sqrt: device vs IEEE host."""
    torch = _torch()
    jsvd = _jsvd()
    g = np.random.default_rng(1)
    a = np.ldexp(g.uniform(1, 2, 200000), g.integers(-300, 300, 200000))
    b = np.ldexp(g.uniform(1, 2, 200000), g.integers(-300, 300, 200000))
    q, r = jsvd.diag_fp64(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    assert np.array_equal(q.cpu().numpy(), a / b)
    assert np.array_equal(r.cpu().numpy(), np.sqrt(a))


CASES = [
    # name, m, n, kwargs, input
    ("graded256_w16_rrev", 256, 256, dict(block_w=16, strategy="rrev"), "graded"),
    ("ragged300x200_w16_r", 300, 200, dict(block_w=16, strategy="r"), "gauss"),
    ("ragged257x129_w32_rrev", 257, 129, dict(block_w=32, strategy="rrev"), "gauss"),
    ("square64_w32_c", 64, 64, dict(block_w=32, strategy="c"), "gauss"),
    ("narrow100x10_w16_crev", 100, 10, dict(block_w=16, strategy="crev"), "gauss"),
    ("single_column", 40, 1, dict(block_w=16), "gauss"),
    ("odd_blocks_w16", 160, 144, dict(block_w=16), "gauss"),  # 9 block-columns
    ("block_oriented_ms1", 200, 192, dict(block_w=16, max_inner_sweeps=1), "gauss"),
    ("tall513x300_w32", 513, 300, dict(block_w=32), "graded"),
    # the full block variant of Section 4.3: up to M_s = 30 inner sweeps per
    # pivot block-pair (the inner stop on a sweep without rotation, the
    # published rotations' double buffer across inner sweep boundaries and
    # the counters summed over inner sweeps)
    ("full_block_graded256_w16_rrev", 256, 256,
     dict(block_w=16, strategy="rrev", max_inner_sweeps=30), "graded"),
    ("full_block_ragged300x231_w32", 300, 231, dict(block_w=32, max_inner_sweeps=30), "gauss"),
    ("full_block_ragged170x150_w16_c", 170, 150,
     dict(block_w=16, strategy="c", max_inner_sweeps=30), "gauss"),
    # the round-robin ordering (a comparison strategy of Section 6) at both
    # levels
    ("round_robin_ragged300x200_w16", 300, 200, dict(block_w=16, strategy="rr"), "gauss"),
    ("round_robin_full_block_graded256_w32", 256, 256,
     dict(block_w=32, strategy="rr", max_inner_sweeps=30), "graded"),
    # w = 64: the third blocking level (a block Jacobi with 16-column
    # sub-blocks on the Cholesky factor of each 128-column pivot pair)
    ("w64_ragged400x300", 400, 300, dict(block_w=64), "gauss"),
    ("w64_graded512", 512, 512, dict(block_w=64), "graded"),
    ("w64_full_block_ragged330x260_c", 330, 260,
     dict(block_w=64, strategy="c", max_inner_sweeps=30), "gauss"),
    ("w64_narrow200x90", 200, 90, dict(block_w=64), "gauss"),
]


@pytest.mark.parametrize("name,m,n,kw,kind", CASES, ids=[c[0] for c in CASES])
def test_gesvd_matches_oracle(name, m, n, kw, kind):
    _say(f"case {name}: m={m} n={n} {kw}")
    g = inputs.rng(100 + m + n)
    if kind == "graded":
        A = inputs.prescribed(m, n, inputs.logspaced(n, -6.0), g)
    else:
        A = inputs.gaussian(m, n, g)
    U, S, V, info = _run_gesvd(A, **kw)
    assert info["status"] == 0, info
    ref = oracle.gesvj(A)
    _check_sigma(S, ref["S"], strict_rel=(1e-12 if kind == "gauss" else None))
    _check_svd(A, U, S, V, n)
    _check_vectors(V, ref["V"], ref["S"])
    _check_vectors(U, ref["U"], ref["S"])
    _say(f"  sweeps={info['sweeps']} rotations={info['rotations']} w={info['block_w']}")


@pytest.mark.parametrize("inner", [0, 30], ids=["library_choice", "full_block_30"])
def test_small_graded_workload(inner):
    """256 x 256, sigma 1 .. 1e-6, Haar factors, w = 16, Rrev (the cyclic
    parallel order), the library's inner sweep choice and the full block
    variant with M_s = 30 (Section 4.3)."""
    A = inputs.small_graded()
    U, S, V, info = _run_gesvd(A, block_w=16, strategy="rrev", max_inner_sweeps=inner)
    assert info["status"] == 0 and info["converged"] == 1
    if inner == 30:
        # more than one inner sweep per pivot pair on average: the repeated
        # inner sweep did run
        assert info["inner_sweeps"] > info["pair_updates"]
    ref = oracle.gesvj(A)
    _check_sigma(S, ref["S"])
    _check_svd(A, U, S, V, 256)
    sig = inputs.logspaced(256, -6.0)
    assert np.max(np.abs(S - sig)) <= 20 * 256 * EPS


def test_deterministic_bitwise():
    """Section 6: the results are reproducible bit for bit."""
    A = inputs.gaussian(200, 160, inputs.rng(9))
    a = _run_gesvd(A, block_w=16)
    b = _run_gesvd(A, block_w=16)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_orthogonal_columns_no_rotation():
    import scipy.linalg
    H = scipy.linalg.hadamard(64).astype(np.float64)
    d = 2.0 ** np.arange(-20, 44, dtype=np.float64)[np.random.default_rng(9).permutation(64)]
    U, S, V, info = _run_gesvd(H * d, block_w=16)
    assert info["rotations"] == 0 and info["sweeps"] == 1
    assert np.array_equal(S, np.sort(d)[::-1] * 8.0)


def test_want_v_false_and_unsorted():
    A = inputs.gaussian(120, 96, inputs.rng(10))
    U, S, _, info = _run_gesvd(A, block_w=16, want_v=False, sort=False)
    ref = oracle.gesvj(A)
    _check_sigma(np.sort(S)[::-1], ref["S"])


def test_nonconvergence_reported():
    A = inputs.gaussian(128, 128, inputs.rng(11))
    _, S, _, info = _run_gesvd(A, block_w=16, max_sweeps=1)
    assert info["status"] == 1 and info["sweeps"] == 1 and info["converged"] == 0


@pytest.mark.parametrize("kind", ["duplicate", "zero"])
def test_rank_deficient_columns(kind):
    """Dependent columns make a pivot block Gram matrix only semidefinite
    (the paper assumes full rank after the preprocessing (2.1)-(2.2)); the
    zero pivot gives a zero row of R and the iteration goes on."""
    A = inputs.gaussian(64, 32, inputs.rng(12))
    if kind == "duplicate":
        A[:, 5] = A[:, 3]
    else:
        A[:, 20] = 0.0
    U, S, V, info = _run_gesvd(A, block_w=16)
    assert info["status"] == 0
    ref = oracle.gesvj(A)
    assert np.max(np.abs(S - ref["S"])) <= 1e-13 * 32 * ref["S"][0]
    assert S[-1] <= 1e-13 * S[0]
    assert np.max(np.abs(V.T @ V - np.eye(32))) <= 1e-13 * 32
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * 32 * np.linalg.norm(A)


def test_nan_input_reported():
    A = inputs.gaussian(64, 32, inputs.rng(13))
    A[7, 7] = np.nan
    _, _, _, info = _run_gesvd(A, block_w=16, allow=(1, 2, 3))
    assert info["status"] == 3


# --------------------------------------------------------------- hyperbolic

def _run_hsvd(G, J, **kw):
    torch = _torch()
    jsvd = _jsvd()
    U, S, V, Jout, info = jsvd.hsvd(torch.from_numpy(np.asfortranarray(G)).cuda(), J, **kw)
    torch.cuda.synchronize()
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), Jout, info


HCASES = [
    ("hsvd96x80_p48", 96, 80, 48, False, dict(block_w=16)),
    ("hsvd150x120_random_J_full_block", 150, 120, None, True,
     dict(block_w=16, max_inner_sweeps=30)),
    ("hsvd200x160_p100_w32_full_block", 200, 160, 100, False,
     dict(block_w=32, max_inner_sweeps=30)),
    ("hsvd130x100_random_J", 130, 100, None, True, dict(block_w=16)),
    ("hsvd128x128_p64_w32", 128, 128, 64, False, dict(block_w=32)),
    ("hsvd70x50_p17_ragged", 70, 50, 17, False, dict(block_w=16)),
    ("hsvd180x150_round_robin_w32", 180, 150, None, True, dict(block_w=32, strategy="rr")),
]


@pytest.mark.parametrize("name,m,n,n_plus,shuffle,kw", HCASES, ids=[c[0] for c in HCASES])
def test_hsvd_matches_oracle(name, m, n, n_plus, shuffle, kw):
    _say(f"case {name}: m={m} n={n} n_plus={n_plus} {kw}")
    g = inputs.rng(200 + m + n)
    G = inputs.gaussian(m, n, g)
    if shuffle:
        J = np.where(g.uniform(size=n) < 0.6, 1, -1).astype(np.int8)
    else:
        J = np.concatenate([np.ones(n_plus), -np.ones(n - n_plus)]).astype(np.int8)
    U, S, V, Jout, info = _run_hsvd(G, J, **kw)
    assert info["status"] == 0, info
    npl = int(np.sum(J == 1))
    assert np.array_equal(Jout, np.concatenate([np.ones(npl), -np.ones(n - npl)]).astype(np.int8))
    # oracle on the column-permuted (partitioned) problem
    perm = np.concatenate([np.nonzero(J == 1)[0], np.nonzero(J == -1)[0]])
    ref = oracle.gesvj(G[:, perm], n_plus=npl)
    # the same sigma bar as the ordinary SVD (no allowance for the growth of
    # the J-orthogonal V, whose kappa_2(V) = ||V||_2^2 is printed beside the
    # measured error)
    vn2 = np.linalg.norm(V, 2) ** 2
    bar = 1e-12 * ref["S"] + 1e-13 * ref["S"].max()
    ratio = float(np.max(np.abs(S - ref["S"]) / bar))
    rel = float(np.max(np.abs(S - ref["S"]) / ref["S"]))
    _say(f"  sigma: max rel err {rel:.2e}, err / bar {ratio:.3f}, ||V||_2^2 {vn2:.2f}")
    assert ratio <= 1.0
    jv = Jout.astype(np.float64)
    jin = J.astype(np.float64)
    vmax = max(1.0, np.max(np.abs(V)) ** 2)
    assert np.max(np.abs(V.T @ (jin[:, None] * V) - np.diag(jv))) <= 1e-13 * n * vmax
    assert np.linalg.norm(G @ V - U * S) <= 1e-13 * n * np.linalg.norm(G) * np.linalg.norm(V, 2)
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 1e-13 * n
    assert np.all(np.diff(S[:npl]) <= 0) and np.all(np.diff(S[npl:]) >= 0)
    _say(f"  sweeps={info['sweeps']} clamps={info['hyp_clamps']}")


def test_w64_falls_back_to_w32_for_hsvd_and_scaled_mode():
    """The third blocking level runs the ordinary unscaled SVD; asked for
    w = 64, the hyperbolic SVD and the scaled mode run with w = 32."""
    g = inputs.rng(16)
    G = inputs.gaussian(120, 100, g)
    J = np.concatenate([np.ones(60), -np.ones(40)]).astype(np.int8)
    U, S, V, Jout, info = _run_hsvd(G, J, block_w=64)
    assert info["status"] == 0 and info["block_w"] == 32
    ref = oracle.gesvj(G, n_plus=60)
    assert np.all(np.abs(S - ref["S"]) <= 1e-12 * ref["S"] + 1e-13 * ref["S"].max())
    A = inputs.gaussian(150, 130, g)
    U, S, V, info = _run_gesvd(A, block_w=64, scaled="on")
    assert info["status"] == 0 and info["block_w"] == 32 and info["scaled"] == 1
    U, S, V, info = _run_gesvd(A, block_w=64)
    assert info["status"] == 0 and info["block_w"] == 64 and info["scaled"] == 0
    ref = oracle.gesvj(A)
    _check_sigma(S, ref["S"], strict_rel=1e-12)
    _check_svd(A, U, S, V, 130)


def test_hsvd_identity_signature_equals_svd():
    A = inputs.gaussian(100, 64, inputs.rng(14))
    a = _run_gesvd(A, block_w=16)
    b = _run_hsvd(A, np.ones(64, np.int8), block_w=16)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("w", [16, 32])
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_stopped_early_keeps_g_and_v_consistent(sweeps, w):
    """When the sweep limit stops the iteration, G and V have seen the same
    transformations (eq. (2.4), G' = G V): the V update of each p-step runs
    in the next p-step's inner launch and the last one after the loop, so
    A V = U diag(S) and V^T V = I hold for the partial result as well."""
    _say(f"case stopped early: sweeps={sweeps} w={w}")
    n = 200
    A = inputs.gaussian(300, n, inputs.rng(15))
    U, S, V, info = _run_gesvd(A, block_w=w, max_sweeps=sweeps)
    assert info["sweeps"] == sweeps and info["converged"] == 0
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    assert np.linalg.norm(A @ V - U * S) <= 1e-13 * n * np.linalg.norm(A)


def test_hsvd_stopped_early_keeps_g_and_v_consistent():
    _say("case hsvd stopped early")
    m, n, npl = 160, 128, 80
    G = inputs.gaussian(m, n, inputs.rng(16))
    J = np.concatenate([np.ones(npl), -np.ones(n - npl)]).astype(np.int8)
    U, S, V, Jout, info = _run_hsvd(G, J, block_w=16, max_sweeps=2)
    assert info["sweeps"] == 2 and info["converged"] == 0
    Jm = np.diag(Jout.astype(np.float64))
    assert np.max(np.abs(V.T @ Jm @ V - Jm)) <= 1e-13 * n * max(1.0, np.max(np.abs(V)) ** 2)
    assert np.linalg.norm(G @ V - U * S) <= 1e-13 * n * np.linalg.norm(G) * np.linalg.norm(V, 2)
