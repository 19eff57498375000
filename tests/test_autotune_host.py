"""Host logic of the autotuner and of the tuning table (no GPU): the
compression of per-size winners into the (n_upper, block_w) table, and the
jsvd_tuning structure the binding builds from it."""
import pytest

from paper_1401_2720_amd import _binding as B
from paper_1401_2720_amd import autotune


def test_table_from_merges_runs_of_the_same_width():
    rows = [{"n": 256, "block_w": 16}, {"n": 1024, "block_w": 16}, {"n": 512, "block_w": 16},
            {"n": 2048, "block_w": 32}, {"n": 4096, "block_w": 32}]
    t = autotune.table_from(rows, {8: 0.3, 16: 0.2, 24: 0.25})
    assert t == {"n_upper": [1024, 4096], "block_w": [16, 32], "gram_wg": [0, 0],
                 "update_wg": [0, 0], "batch_g_groups": 16}


def test_table_from_takes_the_fastest_block_threshold():
    rows = [{"n": 256, "block_w": 16}]
    t = autotune.table_from(rows, {16: 0.2}, {33: 0.13, 65: 0.12, 257: 0.17})
    assert t == {"n_upper": [256], "block_w": [16], "gram_wg": [0], "update_wg": [0],
                 "batch_g_groups": 16, "batch_block_min_n": 65}


def test_table_from_alternating():
    rows = [{"n": 256, "block_w": 32}, {"n": 512, "block_w": 16}, {"n": 1024, "block_w": 32}]
    t = autotune.table_from(rows, {})
    assert t == {"n_upper": [256, 512, 1024], "block_w": [32, 16, 32], "gram_wg": [0, 0, 0],
                 "update_wg": [0, 0, 0]}


def test_table_from_keeps_entries_whose_tile_shapes_differ():
    rows = [{"n": 1024, "block_w": 16, "gram_wg": 512, "update_wg": 1024},
            {"n": 2048, "block_w": 16, "gram_wg": 512, "update_wg": 1024},
            {"n": 3072, "block_w": 32, "gram_wg": 512, "update_wg": 1024},
            {"n": 4096, "block_w": 32, "gram_wg": 1024, "update_wg": 1024}]
    t = autotune.table_from(rows, {})
    assert t == {"n_upper": [2048, 3072, 4096], "block_w": [16, 32, 32],
                 "gram_wg": [512, 512, 1024], "update_wg": [1024, 1024, 1024]}


def test_tuning_struct_fields_and_limits():
    t = B.tuning_struct({"n_upper": [2048, 8192], "block_w": [16, 32], "batch_g_groups": 20})
    assert t.count == 2 and list(t.n_upper)[:2] == [2048, 8192]
    assert list(t.block_w)[:2] == [16, 32] and t.batch_g_groups == 20
    assert t.batch_block_min_n == 0
    assert B.tuning_struct({"batch_block_min_n": 81}).batch_block_min_n == 81
    with pytest.raises(ValueError):
        B.tuning_struct({"n_upper": [1], "block_w": []})
    with pytest.raises(ValueError):
        B.tuning_struct({"n_upper": list(range(9)), "block_w": [16] * 9})
    t = B.tuning_struct({"n_upper": [4096], "block_w": [32], "gram_wg": [1024],
                         "update_wg": [2048]})
    assert t.gram_wg[0] == 1024 and t.update_wg[0] == 2048
    with pytest.raises(ValueError):
        B.tuning_struct({"n_upper": [4096], "block_w": [32], "gram_wg": [1, 2]})


def test_set_tuning_rejects_null_handle():
    # argument checks happen before any device work
    assert B.lib().jsvd_set_tuning(None, None) == -1
