#!/usr/bin/env python3
"""Benchmark: FP64 one-sided block Jacobi SVD of a 4096 x 4096 N(0,1) matrix
on one MI355X, through the C ABI.

One step = one complete SVD (strategy tables from the handle's cache, V := I,
block sweeps of Gram / Cholesky + inner Jacobi / update until no proper
rotation, singular values, U and the output order).  The input is already
in HBM; each step first restores it from a device copy (U overwrites it).

Prints one JSON line with the time per SVD, the roofline of the dominant
kernel (per-kernel times from HIP events recorded by the library on the
stream it launches on) and the oracle timed on a bounded sample on the
host cores.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 matrix (= FP64 vector)
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--block-w", type=int, default=0)
    ap.add_argument("--strategy", default="rrev")
    ap.add_argument("--max-inner-sweeps", type=int, default=0, help="0 = library's choice")
    ap.add_argument("--fuse", action="store_true",
                    help="the update fused into the next p-step's Gram launch (opts.fuse)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle sample (0 = skip)")
    ap.add_argument("--no-forms", action="store_true",
                    help="leave the batched and differentiable forms out of the svd4096 line")
    ap.add_argument("--workload", default="svd4096",
                    choices=["svd4096", "tall", "batched", "backward", "svd4096_qrfactor"],
                    help="svd4096: the benchmark line; tall: the 8192 x 2048 graded SVD (QR "
                         "preprocessing); batched / backward: the other forms; "
                         "svd4096_qrfactor: the benchmark matrix with the QR shortening of "
                         "the pivot pairs (opts.factorize = 1)")
    ap.add_argument("--batched-scaled", default="auto", choices=["auto", "on"],
                    help="batched workload: 'on' runs every problem with DDRJAC pairs and "
                         "DRDSSQ norms (opts.scaled = 2)")
    return ap.parse_args()


TIMING_STRIDE = 8


def kernel_roofline(name, avg_ms, per_launch):
    """Roofline entry of one p-step kernel from its algorithmic work per
    launch: HBM- or MFMA-bound by its arithmetic intensity against the
    ridge point; the inner kernel, whose Cholesky and Jacobi work is a chain
    of dependent FP64 vector operations, against the FP64 vector peak."""
    sec = avg_ms * 1e-3
    if name == "inner":
        # achieved: the inner Jacobi's algorithmic cost per launch, 36 w n^2
        # s_in flops per block sweep over the nb - 1 launches of a sweep;
        # achieved_actual: the same work counted from the run's rotations,
        # inner sweeps and Cholesky factorizations
        achieved = per_launch["inner_flops_model"] / sec / 1e12
        actual = per_launch["inner_flops"] / sec / 1e12
        return {"kernel": "inner", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None, "achieved_actual": actual,
                "frac_actual": actual / PEAK_FP64_TFLOPS,
                "v_stream_gbs": per_launch["inner_v_bytes"] / sec / 1e9}
    flops = per_launch[name + "_flops"]
    bytes_ = per_launch[name + "_bytes"]
    if flops / max(bytes_, 1) >= RIDGE:
        achieved = flops / sec / 1e12
        return {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                "intensity_flop_per_byte": flops / bytes_}
    achieved = bytes_ / sec / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
            "intensity_flop_per_byte": flops / bytes_}


def measured_traffic(kernel_name, w):
    """HBM bytes per launch of a p-step kernel from the committed rocprofv3
    counter summary, or None when there is none for this kernel or its
    sources changed since the counters were taken."""
    from paper_1401_2720_amd import prof_summary
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    name = f"{kernel_name}_kernel<{2 * w}>"
    entry = rec.get("kernels", {}).get(name)
    if entry is None or entry.get("sources_sha256") != prof_summary.kernel_sources_sha256(kernel_name):
        return None
    return entry["hbm_bytes_per_launch"]


def oracle_sweeps(default):
    """Sweeps the oracle takes to converge on the benchmark matrix (recorded
    by tests/golden/make_sigma_golden.py in the header of its output)."""
    path = os.path.join(ROOT, "tests", "golden", "sigma_gaussian4096_seed2.txt")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("# oracle:") and " sweeps," in line:
                    return int(line.split(" sweeps,")[0].split()[-1]), "oracle's own"
    except OSError:
        pass
    return default, "the GPU run's"


def cpu_baseline(A, gpu_sweeps, target_s):
    """The oracle (round-robin OpenMP ordering) on the first rounds of the
    first sweep of the same matrix, scaled to seconds per SVD with the
    number of sweeps the oracle needs on it."""
    import numpy as np
    import oracle
    n = A.shape[1]
    rounds_per_sweep = n - 1 + (n & 1)
    probe = 32
    t0 = time.perf_counter()
    oracle.gesvj(A, order="rr", max_sweeps=1, max_rounds=probe, sort=False)
    t_probe = time.perf_counter() - t0
    rounds = int(max(probe, min(rounds_per_sweep, target_s / max(t_probe / probe, 1e-9))))
    t0 = time.perf_counter()
    oracle.gesvj(A, order="rr", max_sweeps=1, max_rounds=rounds, sort=False)
    t = time.perf_counter() - t0
    per_sweep = t / rounds * rounds_per_sweep
    del np
    sweeps, whose = oracle_sweeps(gpu_sweeps) if n == 4096 else (gpu_sweeps, "the GPU run's")
    return {"value": per_sweep * sweeps, "unit": "s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"round-robin oracle, first {rounds} of {rounds_per_sweep} rounds of "
                       f"sweep 1 on the same {A.shape[0]}x{n} input ({t:.1f} s); per-sweep "
                       f"time x {sweeps} sweeps ({whose} sweep count on this matrix)")}


def measure_batched(steps, warmup, cpu_seconds, plain_sample=200, scaled="auto"):
    """10,000 uneven problems (n ~ U{8..128}, m = n + U{0..64}, 20 % graded)
    in the two persistent launches, captured in a HIP graph and replayed;
    beside it the plain form (one jsvd_gesvd per problem, synchronising per
    sweep) on a fixed seeded sample of the same problems."""
    import numpy as np
    import torch

    import oracle
    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import inputs
    data = inputs.ragged_batch()
    b = jsvd.Batch(data["mats"])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, warmup)):
            jsvd.gesvd_batched(b, scaled=scaled)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        jsvd.gesvd_batched(b, scaled=scaled)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / steps * 1e3
    sw = b.sweeps.cpu().numpy().astype(np.float64)
    m = b.m_host.astype(np.float64)
    n = b.n_host.astype(np.float64)
    # algorithmic flops of the method each problem takes, per sweep:
    # pointwise: n(n-1)/2 pairs x (dots 6m + rotation of G and V 6(m+n));
    # blocked (block-columns of w = 16, nb = ceil(n/16), nb(nb-1)/2 pivot
    # pairs of 2w = 32 columns): per pair the Gram matrix 2w(2w+1)m, the
    # Cholesky (2w)^3/3, one inner sweep of 2w(2w-1)/2 pairs x (dots 6(2w)
    # + rotation of R and V' 6(4w)), and G and V times V' 2(m+n)(2w)^2
    blk = (n >= jsvd.batched_block_min_n()) & (scaled != "on")
    w2 = 32.0
    nb = np.ceil(n / 16.0)
    per_pair = (w2 * (w2 + 1) * m + w2 ** 3 / 3 + w2 * (w2 - 1) / 2 * (6 * w2 + 12 * w2)
                + 2 * (m + n) * w2 ** 2)
    f_blk = nb * (nb - 1) / 2 * per_pair
    f_pt = n * (n - 1) / 2 * (6 * m + 6 * (m + n))
    flops = float(np.sum(sw * np.where(blk, f_blk, f_pt)))
    achieved = flops / (ms * 1e-3) / 1e12
    status = int(b.status.abs().sum())
    del graph

    # the plain form on a seeded sample of the same problems, one call each
    mats = data["mats"]
    pick = np.sort(inputs.rng(55).choice(len(mats), size=min(plain_sample, len(mats)),
                                         replace=False))
    dev_mats = [torch.from_numpy(mats[i]).cuda() for i in pick]
    for A in dev_mats[:4]:
        jsvd.gesvd(A)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for A in dev_mats:
        jsvd.gesvd(A)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - p0) / len(dev_mats)
    plain = {"svds_per_s": 1.0 / plain_s, "sample": f"{len(dev_mats)} seeded problems of the "
             "10000, one jsvd_gesvd each (synchronises once per sweep)",
             "batched_over_plain": (10000 / (ms * 1e-3)) * plain_s}
    cpu = None
    if cpu_seconds > 0:
        # oracle on the problems in index order (one per OpenMP thread) until
        # the sample reaches the target time, scaled to problems per second
        done, t_cpu, k = 0, 0.0, 64
        many = oracle.gesvj_many
        if scaled == "on":
            from oracle import rdssq
            many = rdssq.gesvj_many
        while t_cpu < cpu_seconds and done < len(mats):
            chunk = mats[done:done + k]
            c0 = time.perf_counter()
            many(chunk)
            t_cpu += time.perf_counter() - c0
            done += len(chunk)
            k *= 2
        cpu = {"value": done / t_cpu, "unit": "SVDs/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"first {done} of the 10000 problems ({t_cpu:.1f} s)"}
    return {"svds_per_s": 10000 / (ms * 1e-3), "ms_per_batch": ms, "steps": steps,
            "sweeps_mean": float(sw.mean()), "sweeps_max": int(sw.max()),
            "not_converged": status,
            "roofline": {"kernel": "batched", "bound": "alu", "achieved": achieved,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                         "algorithmic_flops_per_launch": flops},
            "plain_form": plain, "cpu_baseline": cpu}


def bench_batched(args):
    r = measure_batched(args.steps, args.warmup, args.cpu_seconds, scaled=args.batched_scaled)
    out = {"metric": "batched small SVDs/s", "value": r["svds_per_s"], "unit": "SVDs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_batch"],
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "batched_10000_ragged_n8-128", "seed": 5, "graph": True,
                      "scaled": args.batched_scaled,
                      "sweeps_mean": r["sweeps_mean"], "sweeps_max": r["sweeps_max"],
                      "not_converged": r["not_converged"]},
           "roofline": r["roofline"], "plain_form": r["plain_form"],
           "cpu_baseline": r["cpu_baseline"]}
    print(json.dumps(out), flush=True)


def measure_backward(steps, warmup):
    """Forward + backward of the differentiable SVD: 256 x (64 x 64) and one
    1024 x 1024, loss sum w_i s_i + ||U_k V_k^T o W||_F^2, k = 8; beside it
    the plain forward (jsvd_gesvd_batched / jsvd_gesvd through the binding,
    no autograd) on the same matrices."""
    import torch

    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import inputs
    d = inputs.differentiable_set()
    res = {}
    for name, A, w, W in [("256x64x64", d["small"], d["w_small"], d["W_small"]),
                          ("1024x1024", d["large"], d["w_large"], d["W_large"])]:
        A = torch.from_numpy(A).cuda()
        w = torch.from_numpy(w).cuda()
        W = torch.from_numpy(W).cuda()
        fwd, bwd, plain = [], [], []
        for it in range(warmup + steps):
            X = A.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, S, V = jsvd.svd(X)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P = U[..., :, :8] @ V[..., :, :8].transpose(-1, -2)
            L = (w * S).sum() + ((P * W) ** 2).sum()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if A.dim() == 3:
                batch = jsvd.Batch.from_uniform(A)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                jsvd.gesvd_batched(batch, restore=False)
            else:
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                jsvd.gesvd(A)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            if it >= warmup:
                fwd.append(t1 - t0)
                bwd.append(t2 - t1)
                plain.append(t4 - t3)
        b = A.shape[0] if A.dim() == 3 else 1
        n = A.shape[-1]
        f, g, p = (1e3 * sum(x) / len(x) for x in (fwd, bwd, plain))
        res[name] = {"forward_ms": f, "loss_backward_ms": g, "plain_forward_ms": p,
                     "forward_backward_over_plain": (f + g) / p,
                     "backward_gemm_flops": b * 8.0 * n ** 3}
    total_ms = sum(v["forward_ms"] + v["loss_backward_ms"] for v in res.values())
    return {"forward_backward_s": total_ms / 1e3, "parts": res}


def bench_backward(args):
    r = measure_backward(args.steps, args.warmup)
    out = {"metric": "differentiable SVD forward+backward time", "value": r["forward_backward_s"],
           "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": r["forward_backward_s"] * 1e3, "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "svd_backward_256x64x64_and_1024x1024", "seed": 6, "k": 8,
                      "parts": r["parts"]},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def measure_tall(steps, warmup):
    """The tall workload: 8192 x 2048, Q1 diag(sigma) Q2^T with sigma
    log-spaced 1 .. 1e-10 (seed 3), through jsvd_gesvd (QR preprocessing of
    eq. (2.1), the Jacobi method on R^T); one step = one SVD, the input
    restored from a device copy first."""
    import numpy as np
    import torch

    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    from paper_1401_2720_amd import inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    A_host = inputs.tall_graded()
    m, n = A_host.shape
    A0 = torch.from_numpy(A_host).to(dev).t().contiguous()  # column-major copy (n x m)
    work = torch.empty_like(A0)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    L = jsvd.lib()
    h = B._handle(0, torch.cuda.current_stream(dev).cuda_stream)
    opts = B.make_opts()
    info = B.Info()

    def step():
        work.copy_(A0)
        rc = L.jsvd_gesvd(h, m, n, ctypes.c_void_p(work.data_ptr()), m,
                          ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), n,
                          ctypes.byref(opts), ctypes.byref(info))
        if rc != 0:
            raise B.JsvdError(rc, "jsvd_gesvd")

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(steps):
        step()
        sweeps.append(info.sweeps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    sig = inputs.logspaced(n, -10.0)
    s = S.cpu().numpy()
    return {"s": ms / 1e3, "ms": ms, "m": m, "n": n, "block_w": info.block_w,
            "preprocessed": info.preprocessed, "sweeps": sweeps,
            "accuracy": {"max_abs_sigma_err": float(np.max(np.abs(s - sig))),
                         "max_rel_sigma_err_above_1e-3": float(np.max(
                             np.abs(s - sig)[sig >= 1e-3] / sig[sig >= 1e-3]))}}


def measure_small_and_hsvd(steps, warmup):
    """Two more single-matrix workloads, seconds per solve through the
    binding (input restored from a device copy each step, included):
    small_256: 256 x 256, sigma log-spaced 1 .. 1e-6, Haar factors (seed 1),
    w = 16, Rrev; hsvd_2048: the hyperbolic SVD of a 2048 x 2048 N(0,1)
    matrix (seed 4) with J = diag(+1 x 1280, -1 x 768)."""
    import numpy as np
    import torch

    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import inputs
    out = {}
    A = torch.from_numpy(inputs.small_graded()).cuda()
    sig = inputs.logspaced(256, -6.0)

    def small():
        return jsvd.gesvd(A, block_w=16, strategy="rrev")

    G, J = inputs.hyperbolic_gaussian()
    Gd = torch.from_numpy(G).cuda()

    def hyp():
        return jsvd.hsvd(Gd, J)

    for name, fn in (("small_256", small), ("hsvd_2048", hyp)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        info = r[-1]
        rec = {"s": sec, "sweeps": info["sweeps"], "block_w": info["block_w"],
               "status": info["status"]}
        if name == "small_256":
            s = r[1].cpu().numpy()
            rec["max_abs_sigma_err"] = float(np.max(np.abs(s - sig)))
        out[name] = rec
    del np
    return out


def bench_tall(args):
    r = measure_tall(args.steps, args.warmup)
    out = {"metric": "FP64 SVD time (s) at 8192x2048", "value": r["s"], "unit": "s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms"],
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "svd_tall_graded_8192x2048", "m": r["m"], "n": r["n"],
                      "seed": 3, "block_w": r["block_w"], "preprocessed": r["preprocessed"],
                      "sweeps": r["sweeps"]},
           "accuracy": r["accuracy"], "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_qrfactor(args):
    """The benchmark matrix (4096 x 4096 N(0,1), seed 2) with the QR
    shortening of the pivot block-pairs (Section 4.2) in place of the
    Cholesky factor; one step = one SVD; sigma against the oracle's golden
    values; per-kernel event times (the first kernel of a p-step is the QR
    kernel here)."""
    import numpy as np
    import torch

    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    from paper_1401_2720_amd import inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n = args.n
    A0 = torch.from_numpy(inputs.square_gaussian(seed=2, n=n)).to(dev).t().contiguous()
    work = torch.empty_like(A0)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    L = jsvd.lib()
    h = B._handle(0, torch.cuda.current_stream(dev).cuda_stream)
    opts = B.make_opts(block_w=args.block_w, strategy=args.strategy,
                       max_inner_sweeps=args.max_inner_sweeps, factorize="qr")
    info = B.Info()

    def step():
        work.copy_(A0)
        rc = L.jsvd_gesvd(h, n, n, ctypes.c_void_p(work.data_ptr()), n,
                          ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), n,
                          ctypes.byref(opts), ctypes.byref(info))
        if rc != 0:
            raise B.JsvdError(rc, "jsvd_gesvd")

    for _ in range(args.warmup):
        step()
    B.kernel_timing(0, True, stride=TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(args.steps):
        step()
        sweeps.append(info.sweeps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    kt = B.kernel_times(0)
    B.kernel_timing(0, False)
    acc = None
    gold = os.path.join(ROOT, "tests", "golden", "sigma_gaussian4096_seed2.txt")
    if n == 4096 and os.path.exists(gold):
        ref = np.loadtxt(gold)
        s = S.cpu().numpy()
        big = ref >= 1e-3 * ref[0]
        acc = {"max_rel_sigma_err_above_1e-3": float(np.max(np.abs(s - ref)[big] / ref[big]))}
    out = {"metric": f"FP64 SVD time (s) at n={n}, QR shortening", "value": ms / 1e3,
           "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"svd_gaussian_{n}x{n}_qrfactor", "m": n, "n": n, "seed": 2,
                      "block_w": info.block_w, "factorize": "qr", "sweeps": sweeps},
           "kernels_avg_us": {("qrfac" if k == "gram" else k): kt[k][0] / kt[k][1] * 1e3
                              for k in kt if kt[k][1] > 0},
           "accuracy": acc, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU level is not part of "
              "it); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "tall":
        return bench_tall(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "backward":
        return bench_backward(args)
    if args.workload == "svd4096_qrfactor":
        return bench_qrfactor(args)
    import numpy as np
    import torch

    import paper_1401_2720_amd as jsvd
    from paper_1401_2720_amd import _binding as B
    from paper_1401_2720_amd import inputs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    m = n = args.n
    A_host = inputs.square_gaussian(seed=2, n=n)
    A0 = torch.from_numpy(A_host).to(dev).t().contiguous()  # column-major copy (n x m)
    work = torch.empty_like(A0)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    L = jsvd.lib()
    h = B._handle(0, stream.cuda_stream)
    opts = B.make_opts(block_w=args.block_w, strategy=args.strategy,
                       max_inner_sweeps=args.max_inner_sweeps, fuse=args.fuse)
    info = B.Info()

    def step():
        work.copy_(A0)
        rc = L.jsvd_gesvd(h, m, n, ctypes.c_void_p(work.data_ptr()), m,
                          ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), n,
                          ctypes.byref(opts), ctypes.byref(info))
        if rc != 0:
            raise B.JsvdError(rc, "jsvd_gesvd")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around the p-step kernels of every TIMING_STRIDE-th p-step:
    # live kernel durations over the timed region without the events' own
    # cost (about 4 us per launch) inflating the measured SVD time
    B.kernel_timing(0, True, stride=TIMING_STRIDE)
    sweeps, rotations, inner_sweeps, updates = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        sweeps.append(info.sweeps)
        rotations.append(info.rotations)
        inner_sweeps.append(info.inner_sweeps)
        updates.append(info.pair_updates)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = B.kernel_times(0)
    B.kernel_timing(0, False)
    ms_per_step = (t1 - t0) / args.steps * 1e3
    w = info.block_w
    bw = 2 * w
    nb = info.n_blocks
    npairs = nb // 2
    steps_per_sweep = nb - 1

    # algorithmic work per launch, averaged over all p-steps of the timed
    # solves (pairs whose block pair needed no rotation skip the updates):
    #   gram    the pivot Gram matrices, a symmetric product: bw (bw + 1) m
    #           flops per pair on the m x bw columns (read once);
    #   update  [G_p G_q] V'_pq for the pairs with a transformation: 2 m bw^2
    #           flops, the columns read and written;
    #   inner   Cholesky (bw^3 / 3), per inner step and pair the three dot
    #           products (6 bw) and per rotation the update of two columns of
    #           R and of V' (12 bw), FP64 vector work; the same launch also
    #           streams the previous p-step's V update (2 n bw^2 flops, n x bw
    #           columns read and written per transformed pair);
    #   fused   the update of a p-step and the next p-step's Gram matrices in
    #           one launch: both kernels' flops, G read once and the
    #           transformed pairs' columns written.
    launches = sum(sweeps) * steps_per_sweep
    upd_per_launch = sum(updates) / max(launches, 1)
    rot_per_launch = sum(rotations) / max(launches, 1)
    isw_per_launch = sum(inner_sweeps) / max(launches, 1)
    per_launch = {
        "gram_flops": npairs * float(bw) * (bw + 1) * m,
        "gram_bytes": npairs * m * bw * 8.0,
        "update_flops": upd_per_launch * 2.0 * m * bw * bw,
        "update_bytes": upd_per_launch * m * bw * 8.0 * 2,
        "inner_flops": (isw_per_launch * (bw - 1) * (bw // 2) * 6.0 * bw
                        + rot_per_launch * 12.0 * bw + npairs * bw ** 3 / 3.0),
        # the algorithmic model of the inner Jacobi: per block sweep about
        # n^2 / (2 w^2) pivot block-pairs, each inner sweep (2w - 1) w pivot
        # pairs at 6 (2w) flops for the dot products and 12 (2w) for rotating
        # R and V', i.e. 36 w n^2 s_in flops (s_in inner sweeps per pivot
        # block-pair), over the nb - 1 launches of a sweep
        "inner_flops_model": 36.0 * w * n * n * (isw_per_launch / npairs) / steps_per_sweep,
        "inner_v_flops": upd_per_launch * 2.0 * n * bw * bw,
        "inner_v_bytes": upd_per_launch * n * bw * 8.0 * 2,
    }
    per_launch["fused_flops"] = per_launch["update_flops"] + per_launch["gram_flops"]
    per_launch["fused_bytes"] = per_launch["gram_bytes"] + upd_per_launch * m * bw * 8.0
    # kernels that ran in the timed p-steps (with the update fused into the
    # next Gram launch, the plain Gram and update kernels run only at the
    # first and last p-step of a sweep, which the sampled steps may miss)
    kt = {k: v for k, v in kt.items() if v[1] > 0}
    avg = {k: (kt[k][0] / kt[k][1]) for k in kt}
    rooflines = {}
    for name in ("gram", "inner", "update", "fused"):
        if name not in kt:
            continue
        r = kernel_roofline(name, avg[name], per_launch)
        r["avg_launch_us"] = avg[name] * 1e3
        r["launches"] = kt[name][1]
        r["traffic"] = measured_traffic(name, w)
        # HBM rate from the counted bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        # calibrated) over this run's average launch time
        r["traffic_gbs"] = (r["traffic"] / (avg[name] * 1e-3) / 1e9
                            if r["traffic"] is not None else None)
        r["algorithmic_per_launch"] = {k: v for k, v in per_launch.items() if k.startswith(name)}
        rooflines[name] = r
    dominant = max(kt, key=lambda k: kt[k][0])
    roof = dict(rooflines[dominant])
    roof["timed_every_nth_pstep"] = TIMING_STRIDE
    # FP64 MFMA rate of the two contraction kernels over their HIP-event
    # times.  The Gram kernel forms the T(T+1)/2 tiles on and above the
    # diagonal of each pair's (2w)^2 Gram matrix (T = 2w/16).
    tiles = bw // 16
    gram_exec = npairs * 2.0 * m * bw * bw * (tiles * (tiles + 1) / 2) / (tiles * tiles)
    mfma = {"peak_tflops": PEAK_FP64_TFLOPS}
    for name, fl in (("gram", gram_exec), ("update", per_launch["update_flops"]),
                     ("fused", gram_exec + per_launch["update_flops"])):
        if name not in kt:
            continue
        tf = fl / (avg[name] * 1e-3) / 1e12
        mfma[name] = {"executed_flops_per_launch": fl, "tflops": tf,
                      "frac": tf / PEAK_FP64_TFLOPS, "avg_launch_us": avg[name] * 1e3}

    # accuracy of the last step against properties that hold at any size
    Ucm = work.t()
    s = S
    fro2 = float((A0 * A0).sum())
    sum_s2 = float((s * s).sum())
    Vm = V.t()  # V is stored column-major: its transpose view is the matrix
    orth_v = float((Vm.t().contiguous() @ Vm - torch.eye(n, dtype=torch.float64, device=dev))
                   .abs().max())
    orth_u = float((Ucm.t().contiguous() @ Ucm - torch.eye(n, dtype=torch.float64, device=dev))
                   .abs().max())

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(A_host, int(np.median(sweeps)), args.cpu_seconds)

    # the two other forms, measured in the same process after the timed
    # region: the batched solve (graph replay) against the plain form on a
    # sample of its problems, and the differentiable SVD against the plain
    # forward
    forms = None
    if not args.no_forms:
        torch.cuda.synchronize()
        bat = measure_batched(steps=5, warmup=1, cpu_seconds=0)
        bwd = measure_backward(steps=3, warmup=1)
        tall = measure_tall(steps=3, warmup=1)
        more = measure_small_and_hsvd(steps=5, warmup=2)
        forms = {"batched_svds_per_s": bat["svds_per_s"], "batched": bat,
                 "differentiable_forward_backward_s": bwd["forward_backward_s"],
                 "differentiable": bwd["parts"],
                 "tall_8192x2048_s": tall["s"], "tall_8192x2048": tall,
                 "small_256_s": more["small_256"]["s"], "small_256": more["small_256"],
                 "hsvd_2048_s": more["hsvd_2048"]["s"], "hsvd_2048": more["hsvd_2048"]}

    out = {
        "metric": "FP64 SVD time (s) at n=4096",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"svd_gaussian_{m}x{n}", "m": m, "n": n, "seed": 2,
                   "block_w": w, "strategy": args.strategy, "fused": "fused" in kt,
                   "max_inner_sweeps": args.max_inner_sweeps, "sweeps": sweeps,
                   "rotations": rotations[-1]},
        "roofline": roof,
        "rooflines": rooflines,
        "mfma": mfma,
        # the FP64 MFMA rate of a p-step's Gram and update work
        "gram_update_mfma_frac": (gram_exec + per_launch["update_flops"])
        / ((avg["fused"] if "fused" in avg else avg["gram"] + avg["update"]) * 1e-3) / 1e12
        / PEAK_FP64_TFLOPS,
        "forms": forms,
        "kernels_avg_us": {k: avg[k] * 1e3 for k in avg},
        "kernels_share": {k: kt[k][0] / max(sum(v[0] for v in kt.values()), 1e-9) for k in kt},
        "accuracy": {"fro2_rel": abs(sum_s2 - fro2) / fro2, "orth_u": orth_u, "orth_v": orth_v},
        "cpu_baseline": cpu,
        "context": {"paper_k20c_s_n4096": 46.357804, "paper_c2070_s_n4096": 84.4665,
                    "note": "paper: Cholesky factors with spectrum Lambda(2), other hardware"},
        "steps_per_sweep": steps_per_sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
