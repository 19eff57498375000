"""Strategy and variant study of the block Jacobi SVD on synthetic inputs.

    python -m paper_1401_2720_amd.study [--quick] [--json OUT]

For each input it runs every parallel strategy (R, Rrev, C, Crev; Section 3,
and the round-robin ordering RR that Section 6 compares against)
in the block-oriented (one inner sweep, M_s = 1) and the full-block (inner
sweeps to convergence, at most 30) variant, and for the 4096 matrix both
block widths, and prints sweeps, rotations, inner sweeps, the library's own
solve time, and how far the singular values are from those of the first run
(all variants compute the same SVD, so they agree to rounding) and from
reference values: the prescribed singular values of the graded inputs and,
with --golden, values computed independently for the square inputs.  This is the
shape of the paper's comparison of strategies and variants (Section 6), on
synthetic stand-ins for its test matrices.
"""
import argparse
import json
import sys

import numpy as np

from . import inputs

STRATEGIES = ("rrev", "r", "crev", "c", "rr")


def _cases(quick):
    cases = [("graded256", lambda: inputs.small_graded(), None, (16,))]
    if not quick:
        cases += [
            ("gaussian4096", lambda: inputs.square_gaussian(), None, (16, 32)),
            ("hsvd2048", lambda: inputs.hyperbolic_gaussian(), "hsvd", (32,)),
            ("tall8192x2048", lambda: inputs.tall_graded(), None, (32,)),
        ]
    return cases


def _reference(name, golden_dir):
    """Singular values each input is checked against: the prescribed ones
    for the graded inputs, else a file of values computed elsewhere (one per
    line, '#' comments) in golden_dir, if given and present."""
    if name == "graded256":
        return inputs.logspaced(256, -6.0)
    if name == "tall8192x2048":
        return inputs.logspaced(2048, -10.0)
    files = {"gaussian4096": "sigma_gaussian4096_seed2.txt",
             "hsvd2048": "sigma_hsvd2048_p1280_seed4.txt"}
    if golden_dir and name in files:
        import os
        path = os.path.join(golden_dir, files[name])
        if os.path.exists(path):
            return np.loadtxt(path, comments="#")
    return None


def run(quick=False, strategies=STRATEGIES, inner=(1, 30), golden_dir=None):
    import torch
    from . import _binding as B
    rows = []
    for name, make, kind, widths in _cases(quick):
        data = make()
        if kind == "hsvd":
            G, J = data
            A = torch.from_numpy(G).cuda()
        else:
            A = torch.from_numpy(data).cuda()
        ref = None
        exact = _reference(name, golden_dir)
        for w in widths:
            for ms in inner:
                for st in strategies:
                    torch.cuda.synchronize()
                    if kind == "hsvd":
                        _, S, _, _, info = B.hsvd(A, J, block_w=w, strategy=st, max_inner_sweeps=ms)
                    else:
                        _, S, _, info = B.gesvd(A, block_w=w, strategy=st, max_inner_sweeps=ms)
                    torch.cuda.synchronize()
                    s = S.cpu().numpy()
                    if ref is None:
                        ref = s
                    row = dict(input=name, w=w, inner="block-oriented" if ms == 1 else "full block",
                               strategy=st, sweeps=info["sweeps"], converged=info["converged"],
                               rotations=info["rotations"], inner_sweeps=info["inner_sweeps"],
                               seconds=info["seconds"],
                               sigma_dev=float(np.max(np.abs(s - ref)) / max(ref[0], 1e-300)),
                               sigma_err=(float(np.max(np.abs(s - exact)) / exact.max())
                                          if exact is not None else None))
                    rows.append(row)
                    print(json.dumps(row), flush=True)
    return rows


def table(rows):
    out = ["| input | w | variant | strategy | sweeps | rotations | inner sweeps | time (s) | max dev of sigma / sigma_1 | max err vs reference / sigma_1 |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        err = f"{r['sigma_err']:.1e}" if r.get("sigma_err") is not None else "-"
        out.append(f"| {r['input']} | {r['w']} | {r['inner']} | {r['strategy']} | {r['sweeps']} | "
                   f"{r['rotations']} | {r['inner_sweeps']} | {r['seconds']:.3f} | {r['sigma_dev']:.1e} | {err} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="only the 256 x 256 graded input")
    ap.add_argument("--json", help="also write the rows to this file")
    ap.add_argument("--golden", help="directory with reference singular values of the square "
                    "inputs (sigma_gaussian4096_seed2.txt, sigma_hsvd2048_p1280_seed4.txt)")
    a = ap.parse_args(argv)
    rows = run(quick=a.quick, golden_dir=a.golden)
    print(table(rows))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
