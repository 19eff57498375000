"""GPU parity of the batched path (jsvd_gesvd_batched) against the oracle.

Each problem is compared with the oracle's SVD of the same matrix under the
bars of test_gpu_parity.py (sigma elementwise with the combined relative /
absolute tolerance, orthogonality and reconstruction <= 1e-13 n).  At the
full workload size (10,000 problems) a stratified sample is checked against
the oracle one by one and every problem against properties that hold at any
size; the launch is also captured in a HIP graph and replayed.
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


def _check(A, U, S, V, ref):
    m, n = A.shape
    tol = 1e-12 * ref["S"] + 1e-13 * ref["S"][0]
    assert np.all(np.abs(S - ref["S"]) <= tol), (m, n, np.max(np.abs(S - ref["S"]) / tol))
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * max(n, 8)
    nz = S > 0
    Un = U[:, nz]
    assert np.max(np.abs(Un.T @ Un - np.eye(Un.shape[1])), initial=0.0) <= 1e-13 * max(n, 8)
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * max(n, 8) * max(np.linalg.norm(A), 1e-300)
    assert np.all(np.diff(S) <= 0)


def _small_batch(seed=31, count=240):
    g = np.random.default_rng(seed)
    mats = []
    for i in range(count):
        n = int(g.integers(1, 81))
        m = n + int(g.integers(0, 41))
        if i % 5 == 0 and n > 1:
            mats.append(inputs.prescribed(m, n, inputs.logspaced(n, -8.0), g))
        else:
            mats.append(inputs.gaussian(m, n, g))
    mats += [inputs.gaussian(1, 1, g), inputs.gaussian(200, 160, g), inputs.gaussian(64, 64, g)]
    return mats


def test_batched_matches_oracle():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    mats = _small_batch()
    print(f"batched parity: {len(mats)} problems, n up to {max(a.shape[1] for a in mats)}",
          flush=True)
    b = jsvd.Batch(mats)
    jsvd.gesvd_batched(b)
    torch.cuda.synchronize()
    assert int(b.status.abs().sum()) == 0
    refs = oracle.gesvj_many(mats)
    for i, (A, ref) in enumerate(zip(mats, refs)):
        U, S, V = b.results(i)
        _check(A, U, S, V, ref)


def test_batched_deterministic_and_graph_replay():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    mats = _small_batch(seed=32, count=120)
    b = jsvd.Batch(mats)
    jsvd.gesvd_batched(b)
    torch.cuda.synchronize()
    A1, S1, V1 = b.A.clone(), b.S.clone(), b.V.clone()
    jsvd.gesvd_batched(b)
    torch.cuda.synchronize()
    assert torch.equal(A1, b.A) and torch.equal(S1, b.S) and torch.equal(V1, b.V)
    # capture the whole batched solve (input restore + launches) and replay it
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        jsvd.gesvd_batched(b)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        jsvd.gesvd_batched(b)
    for rep in range(3):
        b.A.zero_()
        b.S.zero_()
        b.V.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(A1, b.A) and torch.equal(S1, b.S) and torch.equal(V1, b.V), rep


def test_batched_full_workload_sampled():
    """10,000 problems, n ~ U{8..128}, m = n + U{0..64}, 20 % graded to 1e-8."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    data = inputs.ragged_batch()
    mats = data["mats"]
    print("batched full workload: 10000 problems", flush=True)
    b = jsvd.Batch(mats)
    jsvd.gesvd_batched(b)
    torch.cuda.synchronize()
    assert int(b.status.abs().sum()) == 0
    # every problem: sum of sigma^2 = ||A||_F^2 (segment sums)
    S = b.S.cpu().numpy()
    s2 = np.add.reduceat(S * S, b.s_off_host)
    a2 = np.add.reduceat(data["A"] * data["A"], b.a_off_host)
    assert np.max(np.abs(s2 - a2) / a2) <= 1e-13 * 128
    # stratified sample against the oracle, the largest problems included
    order = np.argsort(-(b.n_host.astype(np.int64) * b.m_host))
    pick = np.unique(np.concatenate([order[:8], order[::400], np.nonzero(data["special"])[0][:10]]))
    refs = oracle.gesvj_many([mats[i] for i in pick])
    for i, ref in zip(pick, refs):
        U, Si, V = b.results(int(i))
        _check(mats[i], U, Si, V, ref)


def _large_batch(seed=33):
    """Sizes around the blocking threshold and the block width (16): n not a
    multiple of 16, odd block counts (a padding block), n = 256 (the largest),
    m = n .. n + 64, graded spectra, and dependent columns (a zero column and
    a repeated one: semidefinite Gram matrices, zero Cholesky pivots)."""
    g = np.random.default_rng(seed)
    mats = []
    for n in (33, 47, 48, 64, 65, 80, 97, 113, 128, 144, 160, 193, 256):
        for extra in (0, 17, 64):
            mats.append(inputs.gaussian(n + extra, n, g))
        mats.append(inputs.prescribed(n + 5, n, inputs.logspaced(n, -8.0), g))
    A = inputs.gaussian(120, 100, g)
    A[:, 7] = 0.0
    A[:, 50] = A[:, 3]
    mats.append(A)
    return mats


def _with_block_threshold(dev, min_n):
    import paper_1401_2720_amd._binding as B
    base = B.load_tuning(dev)
    table = dict(base) if base else {"n_upper": [], "block_w": []}
    table["batch_block_min_n"] = min_n
    B.set_tuning(dev, table)
    return base


@pytest.mark.parametrize("min_n", [33, 0, 257], ids=["all_blocked", "default", "none_blocked"])
def test_batched_blocked_matches_oracle(min_n):
    """The blocked method (block-columns of 16, one inner sweep per pivot
    pair) against the oracle, with every problem of n >= 33 blocked, the
    built-in threshold, and blocking off."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    import paper_1401_2720_amd._binding as B
    mats = _large_batch()
    dev = torch.cuda.current_device()
    print(f"batched blocked parity: min_n={min_n}, {len(mats)} problems", flush=True)
    base = _with_block_threshold(dev, min_n)
    try:
        b = jsvd.Batch(mats)
        jsvd.gesvd_batched(b)
        torch.cuda.synchronize()
    finally:
        B.set_tuning(dev, base)
    assert int(b.status.abs().sum()) == 0
    refs = oracle.gesvj_many(mats)
    for i, (A, ref) in enumerate(zip(mats[:-1], refs[:-1])):
        U, S, V = b.results(i)
        _check(A, U, S, V, ref)
    # dependent columns: two zero singular values
    A, ref = mats[-1], refs[-1]
    U, S, V = b.results(len(mats) - 1)
    n = A.shape[1]
    assert np.all(np.abs(S - ref["S"]) <= 1e-12 * ref["S"] + 1e-13 * ref["S"][0])
    assert S[-1] <= 1e-13 * S[0] and S[-2] <= 1e-13 * S[0] and S[-3] > 1e-3 * S[0]
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13 * n
    big = S > 1e-8 * S[0]
    Ub = U[:, big]
    assert np.max(np.abs(Ub.T @ Ub - np.eye(Ub.shape[1]))) <= 1e-13 * n
    assert np.linalg.norm(A - (U * S) @ V.T) <= 1e-13 * n * np.linalg.norm(A)


def test_batched_blocked_nonfinite_input():
    """A NaN in a blocked problem ends that problem with JSVD_NONFINITE; the
    other problems of the batch are unaffected."""
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    g = np.random.default_rng(34)
    mats = [inputs.gaussian(100, 96, g), inputs.gaussian(90, 80, g), inputs.gaussian(40, 30, g)]
    mats[0][5, 40] = np.nan
    b = jsvd.Batch(mats)
    jsvd.gesvd_batched(b)
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert st[0] == 3 and st[1] == 0 and st[2] == 0, st
    refs = oracle.gesvj_many(mats[1:])
    for i, ref in zip((1, 2), refs):
        U, S, V = b.results(i)
        _check(mats[i], U, S, V, ref)
