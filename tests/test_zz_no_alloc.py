"""jsvd_gesvd_batched_noalloc, the batched SVD for callers that cannot
allocate device memory, against jsvd_gesvd_batched through the C ABI: the
same kernels, so the same bits, on two calls in a row (the second with a
smaller batch, which must not see the first call's counters), with and
without V; a batch beyond the fixed scratch is refused before anything runs.
"""
import numpy as np
import pytest

from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def _mats(count, n_lo, n_hi, seed, graded_every=4):
    g = inputs.rng(seed)
    out = []
    for i in range(count):
        n = int(g.integers(n_lo, n_hi + 1))
        m = n + int(g.integers(0, 33))
        if i % graded_every == 0:
            out.append(inputs.prescribed(m, n, inputs.logspaced(n, -8.0), g))
        else:
            out.append(inputs.gaussian(m, n, g))
    return out


def _run(torch, jsvd, batch, noalloc):
    print(f"  {'noalloc' if noalloc else 'workspace'} call: {batch.count} problems, "
          f"max n {batch.max_n}", flush=True)
    jsvd.gesvd_batched(batch, noalloc=noalloc)
    torch.cuda.synchronize()
    out = [batch.A.clone(), batch.S.clone(), batch.status.clone(), batch.sweeps.clone()]
    if batch.want_v:
        out.append(batch.V.clone())
    return out


@pytest.mark.parametrize("want_v", [True, False])
def test_noalloc_equals_batched_on_two_calls(want_v):
    torch = _torch()
    import paper_1401_2720_amd as jsvd
    print(f"no-alloc batched, want_v={want_v}", flush=True)
    first = jsvd.Batch(_mats(700, 8, 150, 31), want_v=want_v)     # blocked and pointwise
    second = jsvd.Batch(_mats(90, 8, 60, 32), want_v=want_v)      # smaller batch after it
    a1 = _run(torch, jsvd, first, noalloc=True)
    a2 = _run(torch, jsvd, second, noalloc=True)
    b1 = _run(torch, jsvd, first, noalloc=False)
    b2 = _run(torch, jsvd, second, noalloc=False)
    for x, y in zip(a1, b1):
        assert torch.equal(x, y)
    for x, y in zip(a2, b2):
        assert torch.equal(x, y)
    assert int(a1[2].abs().sum()) == 0 and int(a2[2].abs().sum()) == 0
    # a few problems of the smaller batch against the definition: A V = U S
    for i in (0, 1, second.count - 1):
        U, S, V = second.results(i)
        A = second.A0[int(second.a_off_host[i]):][: U.size].cpu().numpy().reshape(U.shape, order="F")
        if want_v:
            assert np.linalg.norm(A @ V - U * S) <= 1e-13 * A.shape[1] * np.linalg.norm(A)
        assert np.all(np.diff(S) <= 0)


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    torch = _torch()
    import ctypes
    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    small = jsvd.Batch(_mats(4, 8, 16, 33))
    h = B._handle(0, torch.cuda.current_stream().cuda_stream)
    o = B.make_opts()
    limit = 1048576
    rc = jsvd.lib().jsvd_gesvd_batched_noalloc(
        h, limit + 1, small.max_m, small.max_n, B._vp(small.m.data_ptr()),
        B._vp(small.n.data_ptr()), B._vp(small.a_off.data_ptr()), B._vp(small.s_off.data_ptr()),
        B._vp(small.v_off.data_ptr()), B._vp(small.A.data_ptr()), B._vp(small.S.data_ptr()),
        B._vp(small.V.data_ptr()), ctypes.byref(o), B._vp(small.status.data_ptr()),
        B._vp(small.sweeps.data_ptr()))
    assert rc == -2
