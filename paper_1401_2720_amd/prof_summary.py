"""Summaries of rocprofv3 output for the p-step kernels.

    python -m paper_1401_2720_amd.prof_summary traffic FETCH.csv WRITE.csv OUT.json
    python -m paper_1401_2720_amd.prof_summary stats KERNEL_STATS.csv
    python -m paper_1401_2720_amd.prof_summary mfma MFMA.csv KERNEL_STATS.csv

``traffic`` reads two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
counter collections of the same program, averages the counters (KiB per
dispatch) of the Gram, inner, update and fused update-and-Gram kernels, and converts them to HBM
bytes with the factors that the same counters give for a device copy of
known size inside the program (torch's copy of the input matrix,
``__amd_rocclr_copyBufferRectAligned``, ``--calib-bytes`` read and written).
Each kernel's entry carries the SHA-256 of the sources it is built from, so
that a reader can tell whether the figures still describe the code.

``stats`` prints a markdown table of a ``--kernel-trace --stats`` summary.

``mfma`` reads a ``rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64
SQ_VALU_MFMA_BUSY_CYCLES`` collection (FP64 MFMA operations / 512 and MFMA
busy cycles summed over SIMDs, per dispatch) and the kernel-trace summary of
the same workload, and prints per p-step kernel the MFMA FLOPs per launch,
the achieved FP64 MFMA rate over the traced average duration and the MFMA
pipe's busy fraction (busy cycles per SIMD / duration in cycles).
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COMMON = ["jsvd_device.h", "jsvd_internal.h"]
KERNEL_SOURCES = {"gram": ["jsvd_gram.hip"],
                  "inner": ["jsvd_inner.hip", "jsvd_rows.h", "jsvd_blocked.h", "jsvd_qrpair.h"],
                  "update": ["jsvd_update.hip", "jsvd_rows.h"],
                  "fused": ["jsvd_fused.hip"]}
PSTEP = re.compile(r"\b(gram|inner|update|fused)_kernel<(\d+)(?:, (?:true|false))*>")


def kernel_sources_sha256(kernel):
    """SHA-256 over the sources of one p-step kernel ('gram', 'inner', 'update',
    'fused')."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel] + COMMON:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _counter_means(path, calib_kernel):
    per = collections.defaultdict(list)
    calib = []
    for row in csv.DictReader(open(path)):
        name = row["Kernel_Name"]
        value = float(row["Counter_Value"])
        m = PSTEP.search(name)
        if m:
            per[f"{m.group(1)}_kernel<{m.group(2)}>"].append(value)
        elif calib_kernel in name:
            calib.append(value)
    return per, calib


def traffic(fetch_csv, write_csv, out, calib_kernel, calib_bytes, workload, command):
    fetch, fcal = _counter_means(fetch_csv, calib_kernel)
    write, wcal = _counter_means(write_csv, calib_kernel)
    if not fcal or not wcal:
        raise SystemExit(f"no dispatch of {calib_kernel} in the counter files")
    kib = calib_bytes / 1024.0
    # the calibration copy is the largest dispatch of that kernel
    f_factor = kib / max(fcal)
    w_factor = kib / max(wcal)
    kernels = {}
    for name in sorted(set(fetch) & set(write)):
        f, w = fetch[name], write[name]
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        kernels[name] = {
            "dispatches": len(f),
            "fetch_kib": round(fm, 1), "write_kib": round(wm, 1),
            "fetch_kib_max": round(max(f), 1), "write_kib_max": round(max(w), 1),
            "hbm_bytes_per_launch": round((fm * f_factor + wm * w_factor) * 1024),
            "hbm_bytes_per_launch_max": round((max(f) * f_factor + max(w) * w_factor) * 1024),
            "sources_sha256": kernel_sources_sha256(PSTEP.search(name).group(1)),
        }
    rec = {"workload": workload, "command": command,
           "calibration": {"kernel": calib_kernel, "bytes_read": calib_bytes,
                           "bytes_written": calib_bytes, "fetch_kib": round(max(fcal), 1),
                           "write_kib": round(max(wcal), 1), "fetch_factor": round(f_factor, 4),
                           "write_factor": round(w_factor, 4)},
           "kernels": kernels}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def stats(path, keep="jsvd"):
    print("| kernel | calls | total (ms) | average (us) | share | min (us) | max (us) |")
    print("|---|---|---|---|---|---|---|")
    for row in csv.DictReader(open(path)):
        name = row["Name"]
        if keep not in name:
            continue
        m = re.search(r"(\w+(?:<[^>]*>)?)\(", name)
        short = m.group(1) if m else name[:48]
        print(f"| {short} | {row['Calls']} | {float(row['TotalDurationNs']) / 1e6:.1f} | "
              f"{float(row['AverageNs']) / 1e3:.1f} | {float(row['Percentage']):.1f} % | "
              f"{float(row['MinNs']) / 1e3:.1f} | {float(row['MaxNs']) / 1e3:.1f} |")


def mfma(counter_csv, stats_csv, simds=1024, clock_ghz=2.4, peak_tflops=78.6):
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    for row in csv.DictReader(open(counter_csv)):
        m = PSTEP.search(row["Kernel_Name"])
        if m:
            per[f"{m.group(1)}_kernel<{m.group(2)}>"][row["Counter_Name"]].append(
                float(row["Counter_Value"]))
    avg_us = {}
    for row in csv.DictReader(open(stats_csv)):
        m = PSTEP.search(row["Name"])
        if m:
            avg_us[f"{m.group(1)}_kernel<{m.group(2)}>"] = float(row["AverageNs"]) / 1e3
    print("| kernel | FP64 MFMA FLOP per launch (mean / max) | MFMA busy cycles per SIMD (mean) | "
          "average duration (us) | achieved TFLOP/s | of 78.6 peak | MFMA pipe busy |")
    print("|---|---|---|---|---|---|---|")
    out = {}
    for name in sorted(per):
        mops = per[name].get("SQ_INSTS_VALU_MFMA_MOPS_F64", [0.0])
        busy = per[name].get("SQ_VALU_MFMA_BUSY_CYCLES", [0.0])
        flops, fmax = 512 * sum(mops) / len(mops), 512 * max(mops)
        if flops == 0 or name not in avg_us:
            continue
        b = sum(busy) / len(busy) / simds
        us = avg_us[name]
        tf = flops / (us * 1e-6) / 1e12
        frac_busy = b / (us * 1e-6 * clock_ghz * 1e9)
        out[name] = dict(flops=flops, flops_max=fmax, busy_per_simd=b, avg_us=us, tflops=tf,
                         peak_frac=tf / peak_tflops, busy_frac=frac_busy)
        print(f"| {name} | {flops / 1e9:.3f} G / {fmax / 1e9:.3f} G | {b:.0f} | {us:.1f} | {tf:.1f} | "
              f"{100 * tf / peak_tflops:.1f} % | {100 * frac_busy:.1f} % |")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--calib-kernel", default="__amd_rocclr_copyBufferRectAligned")
    t.add_argument("--calib-bytes", type=int, default=4096 * 4096 * 8)
    t.add_argument("--workload", default="")
    t.add_argument("--command", default="")
    mf = sub.add_parser("mfma")
    mf.add_argument("counter_csv")
    mf.add_argument("stats_csv")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--keep", default="jsvd")
    a = ap.parse_args(argv)
    if a.cmd == "traffic":
        rec = traffic(a.fetch_csv, a.write_csv, a.out, a.calib_kernel, a.calib_bytes,
                      a.workload, a.command)
        json.dump(rec, sys.stdout, indent=1)
        print()
    elif a.cmd == "mfma":
        mfma(a.counter_csv, a.stats_csv)
    else:
        stats(a.csv, a.keep)


if __name__ == "__main__":
    main()
