"""Write the oracle's singular values of the two full-size square workloads.

Calls only the oracle (round-robin ordering, run to convergence: a sweep
with no rotation at all) and the seeded input generators; nothing from the
GPU library.  Output, one value per line in the final order (%.17e, which
round-trips binary64 exactly):

  sigma_gaussian4096_seed2.txt   4096 x 4096 N(0,1), seed 2: the ordinary SVD
  sigma_hsvd2048_p1280_seed4.txt 2048 x 2048 N(0,1), seed 4, J = diag(+1 x
                                 1280, -1 x 768): the hyperbolic SVD (the
                                 positive part non-increasing, then the
                                 negative part non-decreasing)

Run: python tests/golden/make_sigma_golden.py  (several minutes on 8 cores)
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1401_2720_amd import inputs  # noqa: E402


def _write(name, S, r, what, secs):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write(f"# {what}\n")
        f.write(f"# oracle: round-robin one-sided Jacobi, {r['sweeps']} sweeps, "
                f"{r['rotations']} rotations, converged={r['converged']}, "
                f"{secs:.0f} s on {oracle.num_threads()} threads\n")
        for v in S:
            f.write(f"{v:.17e}\n")
    print(f"wrote {path}", flush=True)


def main():
    which = sys.argv[1:] or ["gaussian4096", "hsvd2048"]
    if "gaussian4096" in which:
        A = inputs.square_gaussian(seed=2, n=4096)
        t0 = time.time()
        r = oracle.gesvj(A, order="rr", want_v=False, max_sweeps=100)
        _write("sigma_gaussian4096_seed2.txt", r["S"], r,
               "singular values of the 4096 x 4096 N(0,1) matrix, seed 2", time.time() - t0)
    if "hsvd2048" in which:
        G, J = inputs.hyperbolic_gaussian(seed=4, n=2048, n_plus=1280)
        t0 = time.time()
        r = oracle.gesvj(G, n_plus=1280, order="rr", want_v=False, max_sweeps=100)
        _write("sigma_hsvd2048_p1280_seed4.txt", r["S"], r,
               "hyperbolic singular values of the 2048 x 2048 N(0,1) matrix, seed 4, "
               "J = diag(+1 x 1280, -1 x 768)", time.time() - t0)


if __name__ == "__main__":
    main()
