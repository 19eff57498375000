"""The C ABI's workspace calls and the batched call's workspace under HIP
graph capture, and the differentiable form's status handling.

  * jsvd_workspace_size / jsvd_workspace_size_batched report sizes that grow
    with the problem, and jsvd_reserve_batched lets the very first batched
    call be captured (it then allocates nothing);
  * a captured batched call keeps its workspace: a larger jsvd_gesvd, a
    larger backward and a larger batched call after the capture do not free
    it (the larger batched call runs in a new workspace), and every replay
    gives the same bits;
  * a batched call captured on a workspace too small for it is refused with
    JSVD_NO_MEMORY (no allocation during capture);
  * the differentiable SVD raises when its forward does not converge.
"""
import numpy as np
import pytest

from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _fresh_handles():
    """Each test here starts on a new library handle and leaves none behind
    whose batched workspace a graph has pinned."""
    from paper_1401_2720_amd import _binding as B
    B._HANDLES.clear()
    yield
    B._HANDLES.clear()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _mats(count, n_lo, n_hi, seed):
    g = inputs.rng(seed)
    out = []
    for _ in range(count):
        n = int(g.integers(n_lo, n_hi + 1))
        m = n + int(g.integers(0, 17))
        out.append(inputs.gaussian(m, n, g))
    return out


def test_workspace_sizes_grow_with_the_problem():
    _torch()
    import paper_1401_2720_amd as jsvd
    a = jsvd.workspace_size(256, 256)
    b = jsvd.workspace_size(1024, 1024)
    c = jsvd.workspace_size(8192, 1024)          # QR path: its factor on top
    d = jsvd.workspace_size(8192, 1024, qr="off")
    assert 0 < a < b and c > d > 0
    # the batched workspace is the work order and the queue counters: a few
    # bytes per problem, whatever the sizes of the problems
    small = jsvd.Batch(_mats(10, 8, 200, 1))
    large = jsvd.Batch(_mats(3000, 8, 12, 2))
    ws_small, ws_large = jsvd.workspace_size_batched(small), jsvd.workspace_size_batched(large)
    assert 0 < ws_small < ws_large <= 4 * 3000 + 4096


def _capture(torch, jsvd, batch):
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            jsvd.gesvd_batched(batch, restore=False)
    torch.cuda.current_stream().wait_stream(side)
    return graph


def _replay(torch, batch, graph):
    batch.A.copy_(batch.A0)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    return batch.A.clone(), batch.S.clone(), batch.V.clone()


def test_reserved_workspace_lets_the_first_call_be_captured():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    batch = jsvd.Batch(_mats(40, 8, 100, 3))
    jsvd.reserve_batched(batch)
    graph = _capture(torch, jsvd, batch)
    got = _replay(torch, batch, graph)
    jsvd.gesvd_batched(batch)          # eager, restores the inputs first
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(got, (batch.A, batch.S, batch.V)))


def test_capture_survives_larger_calls_on_the_same_handle():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    batch = jsvd.Batch(_mats(30, 8, 64, 4))
    jsvd.gesvd_batched(batch)          # eager first call sizes the workspace
    torch.cuda.synchronize()
    graph = _capture(torch, jsvd, batch)
    first = _replay(torch, batch, graph)
    # a much larger dense SVD and backward on the same handle
    A = torch.from_numpy(inputs.gaussian(1500, 1200, inputs.rng(5))).cuda()
    U, S, V, info = jsvd.gesvd(A)
    assert info["status"] == 0
    dA = jsvd.svd_backward(U, S, V, dS=torch.ones_like(S))
    torch.cuda.synchronize()
    assert bool(torch.isfinite(dA).all())
    # a larger batched call grows the workspace into a new allocation; the
    # captured one stays valid for its graph
    bigger = jsvd.Batch(_mats(400, 100, 200, 6))
    jsvd.gesvd_batched(bigger)
    torch.cuda.synchronize()
    assert int(bigger.status.abs().sum()) == 0
    second = _replay(torch, batch, graph)
    assert all(torch.equal(x, y) for x, y in zip(first, second))
    # and the larger batch gives the same bits as on a fresh handle
    got = (bigger.A.clone(), bigger.S.clone(), bigger.V.clone())
    from paper_1401_2720_amd import _binding as B
    B._HANDLES.clear()
    jsvd.gesvd_batched(bigger)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(got, (bigger.A, bigger.S, bigger.V)))


def test_capture_of_a_call_that_needs_more_workspace_is_refused():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    small = jsvd.Batch(_mats(10, 8, 30, 9))
    jsvd.gesvd_batched(small)
    torch.cuda.synchronize()
    bigger = jsvd.Batch(_mats(80, 100, 200, 10))
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    code = None
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            try:
                jsvd.gesvd_batched(bigger, restore=False)
            except jsvd.JsvdError as e:
                code = e.code
    torch.cuda.current_stream().wait_stream(side)
    assert code == 6


def test_differentiable_forward_raises_when_not_converged():
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    A = torch.from_numpy(inputs.gaussian(96, 80, inputs.rng(7))).cuda().requires_grad_(True)
    with pytest.raises(jsvd.JsvdError) as e:
        jsvd.svd(A, max_sweeps=1)
    assert e.value.code == 1
    Ab = torch.from_numpy(np.stack([inputs.gaussian(40, 30, inputs.rng(8 + i))
                                    for i in range(3)])).cuda()
    with pytest.raises(jsvd.JsvdError):
        jsvd.svd(Ab, max_sweeps=1)
