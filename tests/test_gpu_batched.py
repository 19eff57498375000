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
