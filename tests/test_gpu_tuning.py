"""Tuned choices through the C ABI (jsvd_set_tuning): the w table decides the
block width when opts leave it to the library, an invalid table is refused,
and the batched kernel's G/V split changes who does the work but not one bit
of the result."""
import numpy as np
import pytest

from paper_1401_2720_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture
def dev():
    torch = _torch()
    from paper_1401_2720_amd import _binding as B
    d = torch.cuda.current_device()
    B._handle(d, torch.cuda.current_stream(d).cuda_stream)
    yield d
    B.set_tuning(d, B.load_tuning(d))  # back to the installed table (or none)


def test_width_table_decides_block_w(dev):
    torch = _torch()
    from paper_1401_2720_amd import _binding as B
    print("tuning: w table", flush=True)
    A = torch.from_numpy(inputs.gaussian(300, 200, inputs.rng(21))).cuda()
    out = {}
    for w in (16, 32):
        B.set_tuning(dev, {"n_upper": [100, 10 ** 6], "block_w": [32 if w == 16 else 16, w]})
        _, S, _, info = B.gesvd(A)
        assert info["block_w"] == w and info["status"] == 0
        out[w] = S.cpu().numpy()
    assert np.max(np.abs(out[16] - out[32])) <= 1e-13 * out[16][0]


def test_tile_shapes_follow_the_table(dev):
    """The Gram and update tile shapes of a tuning entry change the launch
    geometry (the Gram partial sums' workspace follows the row splits) and
    the result only within the rounding of a different summation order."""
    torch = _torch()
    import oracle
    from paper_1401_2720_amd import _binding as B
    import paper_1401_2720_amd as jsvd
    print("tuning: tile shapes", flush=True)
    A_np = inputs.gaussian(700, 640, inputs.rng(22))
    A = torch.from_numpy(A_np).cuda()
    ref = oracle.gesvj(A_np)["S"]
    sizes = {}
    for g, u in ((64, 64), (512, 1024), (4096, 8192)):
        B.set_tuning(dev, {"n_upper": [10 ** 6], "block_w": [32], "gram_wg": [g],
                           "update_wg": [u]})
        sizes[g] = jsvd.workspace_size(700, 640)
        _, S, V, info = B.gesvd(A)
        assert info["status"] == 0 and info["block_w"] == 32
        s = S.cpu().numpy()
        assert np.max(np.abs(s - ref) / ref) <= 1e-12
        Vh = V.cpu().numpy()
        assert np.max(np.abs(Vh.T @ Vh - np.eye(640))) <= 1e-13 * 640
    assert sizes[64] < sizes[512] <= sizes[4096]


def test_invalid_table_refused(dev):
    from paper_1401_2720_amd import _binding as B
    for bad in ({"n_upper": [10], "block_w": [24]},
                {"n_upper": [10, 5], "block_w": [16, 32]},
                {"n_upper": [], "block_w": [], "batch_g_groups": 2},
                {"n_upper": [], "block_w": [], "batch_block_min_n": 20},
                {"n_upper": [], "block_w": [], "batch_block_min_n": 300},
                {"n_upper": [10], "block_w": [16], "gram_wg": [32], "update_wg": [0]},
                {"n_upper": [10], "block_w": [16], "gram_wg": [0], "update_wg": [9000]}):
        with pytest.raises(B.JsvdError):
            B.set_tuning(dev, bad)


def test_batched_split_bitwise_equal(dev):
    torch = _torch()
    from paper_1401_2720_amd import _binding as B
    print("tuning: batched split", flush=True)
    data = inputs.ragged_batch(seed=23, count=300)
    res = []
    for g in (8, 16, 24):
        B.set_tuning(dev, {"n_upper": [], "block_w": [], "batch_g_groups": g})
        b = B.Batch(data["mats"])
        B.gesvd_batched(b)
        torch.cuda.synchronize()
        res.append((b.A.cpu().numpy(), b.S.cpu().numpy(), b.V.cpu().numpy(),
                    b.sweeps.cpu().numpy()))
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert np.array_equal(x, y)
