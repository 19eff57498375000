"""Autotuner: measures the library's tunable choices on this device and
writes them to tuning.json beside this file, where the binding picks them up
for every new handle (jsvd_set_tuning).

    python -m paper_1401_2720_amd.autotune [--quick] [--out PATH]

Tuned:
  * the block width w of the dense SVD / HSVD, over w in {16, 32, 64}, on seeded
    N(0,1) square matrices of several orders n: the table maps each measured
    n to the fastest w (a problem takes the entry of the first measured n
    that is >= its n, or the last one);
  * for that w and n, the tile shapes of the p-step kernels: the number of
    workgroups of a Gram launch (its row splits) and of an update launch
    (its row chunks per pivot pair), over a small grid;
  * the split of the batched kernel's 32 half waves between rotating G and
    applying the rotations to V, on the 10000-problem ragged batch (n 8..128,
    m = n + 0..64, the synthetic stand-in of the batched workload), with
    blocking off so that every problem takes the pointwise kernel;
  * then, with that split, the smallest n of a batched problem that takes
    the blocked method (block-columns of 16), same batch.

Every candidate is timed twice after a warm-up run and the faster time is
kept; times are the library's own solve times (dense) and the wall time of
one batched call between stream synchronisations (batched).
"""
import argparse
import datetime
import json
import sys
import time

import numpy as np

from . import inputs

DENSE_ORDERS = (256, 512, 1024, 2048, 3072, 4096, 8192)
WIDTHS = (16, 32, 64)
GRAM_WG = (256, 512, 1024)
UPDATE_WG = (512, 1024, 2048)
G_GROUPS = (8, 12, 16, 20, 24)
BLOCK_MIN_N = (33, 49, 65, 81, 97, 257)  # 257: no problem blocked


def _time_dense(B, A, w, reps=2):
    import torch
    best = None
    for it in range(reps + 1):
        torch.cuda.synchronize()
        _, _, _, info = B.gesvd(A, block_w=w)
        torch.cuda.synchronize()
        if it:
            best = info["seconds"] if best is None else min(best, info["seconds"])
    return best


def tune_dense(orders=DENSE_ORDERS, widths=WIDTHS, gram_wg=GRAM_WG, update_wg=UPDATE_WG,
               seed=11):
    """Per order n: the fastest w with the built-in tile shapes, then for
    that w the fastest (Gram, update) workgroup counts."""
    import torch
    from . import _binding as B
    dev = torch.cuda.current_device()
    rows = []
    for n in orders:
        A = torch.from_numpy(inputs.gaussian(n, n, inputs.rng(seed + n))).cuda()
        B.set_tuning(dev, None)
        times = {w: _time_dense(B, A, w) for w in widths}
        best = min(times, key=times.get)
        shapes = {}
        for g in gram_wg:
            for u in update_wg:
                B.set_tuning(dev, {"n_upper": [n], "block_w": [best], "gram_wg": [g],
                                   "update_wg": [u]})
                shapes[(g, u)] = _time_dense(B, A, best)
        B.set_tuning(dev, None)
        g_best, u_best = min(shapes, key=shapes.get)
        rows.append({"n": n, "times_s": {str(w): t for w, t in times.items()}, "block_w": best,
                     "shape_times_s": {f"{g}/{u}": t for (g, u), t in shapes.items()},
                     "gram_wg": g_best, "update_wg": u_best})
        print(json.dumps(rows[-1]), flush=True)
    return rows


def _time_batched(B, batch, reps=2):
    import torch
    best = None
    for it in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.gesvd_batched(batch)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if it:
            best = dt if best is None else min(best, dt)
    return best


def tune_batched(groups=G_GROUPS, block_min=BLOCK_MIN_N, count=10000):
    """Returns ({g_groups: seconds}, {block_min_n: seconds})."""
    import torch
    from . import _binding as B
    data = inputs.ragged_batch(count=count)
    batch = B.Batch(data["mats"])
    dev = torch.cuda.current_device()
    times = {}
    for g in groups:
        B.set_tuning(dev, {"n_upper": [], "block_w": [], "batch_g_groups": g,
                           "batch_block_min_n": 257})
        times[g] = _time_batched(B, batch)
        print(json.dumps({"batch_g_groups": g, "seconds": times[g]}), flush=True)
    g_best = int(min(times, key=times.get))
    btimes = {}
    for mn in block_min:
        B.set_tuning(dev, {"n_upper": [], "block_w": [], "batch_g_groups": g_best,
                           "batch_block_min_n": mn})
        btimes[mn] = _time_batched(B, batch)
        print(json.dumps({"batch_block_min_n": mn, "seconds": btimes[mn]}), flush=True)
    B.set_tuning(dev, None)
    return times, btimes


def table_from(dense_rows, batched_times, block_times=None):
    dense_rows = sorted(dense_rows, key=lambda r: r["n"])
    n_upper, block_w, gram_wg, update_wg = [], [], [], []
    for r in dense_rows:
        key = (r["block_w"], r.get("gram_wg", 0), r.get("update_wg", 0))
        if block_w and (block_w[-1], gram_wg[-1], update_wg[-1]) == key:
            n_upper[-1] = r["n"]          # extend the run of the same choices
        else:
            n_upper.append(r["n"])
            block_w.append(key[0])
            gram_wg.append(key[1])
            update_wg.append(key[2])
    table = {"n_upper": n_upper, "block_w": block_w, "gram_wg": gram_wg,
             "update_wg": update_wg}
    if batched_times:
        table["batch_g_groups"] = int(min(batched_times, key=batched_times.get))
    if block_times:
        table["batch_block_min_n"] = int(min(block_times, key=block_times.get))
    return table


def main(argv=None):
    import torch
    from . import _binding as B
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="orders up to 1024, batch of 2000")
    ap.add_argument("--out", default=B.TUNING_PATH)
    a = ap.parse_args(argv)
    dev = torch.cuda.current_device()
    B._handle(dev, torch.cuda.current_stream(dev).cuda_stream)
    B.set_tuning(dev, None)  # measure from the built-in rule, not an older table
    orders = tuple(n for n in DENSE_ORDERS if n <= 1024) if a.quick else DENSE_ORDERS
    dense = tune_dense(orders)
    batched, blocked = tune_batched(count=2000 if a.quick else 10000)
    table = table_from(dense, batched, blocked)
    props = torch.cuda.get_device_properties(dev)
    rec = {"arch": props.gcnArchName.split(":")[0], "device": props.name,
           "date": datetime.date.today().isoformat(),
           "dense": dense, "batched_seconds": {str(k): v for k, v in batched.items()},
           "batched_block_min_n_seconds": {str(k): v for k, v in blocked.items()},
           "table": table}
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(table))
    return 0


if __name__ == "__main__":
    sys.exit(main())
