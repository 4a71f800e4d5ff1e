"""Summaries of rocprofv3 output for the kernels of libfcmdp.

    python -m paper_2210_01837_amd.profiling stats DIR
        kernel-time table (markdown) from a `--kernel-trace --stats` run

    python -m paper_2210_01837_amd.profiling traffic \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
        --copy-bytes B --workload NAME --out FILE
        HBM bytes per launch of every kernel from two `--pmc FETCH_SIZE` /
        `--pmc WRITE_SIZE` runs, each scaled by what the same counter reads
        for a plain device copy of B bytes (the `bench.py --copy-calibrate`
        run), written as JSON with a hash of the kernel sources so that a
        reader can tell when the counters no longer describe the code.

    python -m paper_2210_01837_amd.profiling compute --pmc DIR [--pmc DIR] \
        --workload NAME --out FILE
        executed arithmetic per launch of every kernel from `--pmc` runs of
        the FLOP and instruction counters (FP64 and FP32 vector FLOPs,
        FP32 matrix-core operations, VALU instructions and wavefronts), as
        JSON with the same source hash.

Only CSV files are read; nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")

# translation unit (plus the headers it includes) of each profiled kernel
KERNEL_SOURCES = {
    "k_columns_mfma": ["columns_seg.hip", "colmath.h", "fcmdp_internal.h"],
    "k_spread_wave": ["spread_interp.hip", "es.h", "fcmdp_internal.h"],
    "k_spread_mfma": ["spread_mfma.hip", "fcmdp_internal.h"],
    "k_interp_tiled": ["spread_interp.hip", "es.h", "fcmdp_internal.h"],
    "k_interp_part": ["interp_part.hip", "fcmdp_internal.h"],
    "k_interp_sum": ["interp_part.hip", "fcmdp_internal.h"],
    "k_fftw_x_r2c": ["fft.hip", "fcmdp_internal.h"],
    "k_fftw_y": ["fft.hip", "fcmdp_internal.h"],
    "k_fftw_y_pipe": ["fft.hip", "fcmdp_internal.h"],
    "k_fftw_x_c2r": ["fft.hip", "fcmdp_internal.h"],
    "k_records": ["prep.hip", "es.h", "fcmdp_internal.h"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """fcmdp::k_columns_mfma<0>(...) -> k_columns_mfma (also inside an
    anonymous namespace)"""
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    base = base.split("<")[0]
    return base.split("::")[-1].strip()


def _find(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(d: str):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e6,
             float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"]))
            for r in rows]


def counter_means(d: str):
    """{short kernel name: {counter: mean value per dispatch}}"""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(
            float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in agg.items()}


def stats_markdown(d: str) -> str:
    out = ["| kernel | calls | avg ms | total ms | % |", "|---|---|---|---|---|"]
    for name, calls, avg, tot, pct in kernel_stats(d):
        n = name if len(name) < 90 else name[:87] + "..."
        out.append(f"| `{n}` | {calls} | {avg:.3f} | {tot:.3f} | {pct:.2f} |")
    return "\n".join(out)


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes,
            workload):
    fetch = counter_means(fetch_dir)
    write = counter_means(write_dir)
    cf = counter_means(copy_fetch_dir)
    cw = counter_means(copy_write_dir)

    def copy_counter(table, counter):
        # the plain copy is the dispatch whose counter is largest
        return max(v.get(counter, 0.0) for v in table.values())

    f_factor = copy_bytes / (copy_counter(cf, "FETCH_SIZE") * 1024.0)
    w_factor = copy_bytes / (copy_counter(cw, "WRITE_SIZE") * 1024.0)
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith("k_"):
            continue
        fk = fetch.get(k, {}).get("FETCH_SIZE", 0.0)
        wk = write.get(k, {}).get("WRITE_SIZE", 0.0)
        kernels[k] = {"fetch_kib_raw": fk, "write_kib_raw": wk,
                      "bytes_per_launch": fk * 1024.0 * f_factor + wk * 1024.0 * w_factor,
                      "source_hash": source_hash(k) if k in KERNEL_SOURCES else None}
    return {"workload": workload, "fetch_factor": f_factor,
            "write_factor": w_factor, "copy_bytes": copy_bytes,
            "kernels": kernels}


def compute(pmc_dirs, workload):
    """Executed FLOPs per launch: SQ_INSTS_VALU_FLOPS_FP64 (+ _TRANS) and
    _FP32 (+ _TRANS) count the FLOPs of each wavefront instruction per lane
    (2 FMA + ADD + MUL + TRANS), so the executed vector FLOPs are 64 times
    them; SQ_INSTS_VALU_MFMA_MOPS_F32 counts matrix-core operations in units
    of 512 FLOPs."""
    merged = collections.defaultdict(dict)
    for d in pmc_dirs:
        for k, cs in counter_means(d).items():
            merged[k].update(cs)
    kernels = {}
    for k, cs in sorted(merged.items()):
        if not k.startswith("k_"):
            continue
        g = cs.get
        e = {"counters": cs,
             "fp64_vector_flops": 64.0 * (g("SQ_INSTS_VALU_FLOPS_FP64", 0.0) +
                                          g("SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0)),
             "fp32_vector_flops": 64.0 * (g("SQ_INSTS_VALU_FLOPS_FP32", 0.0) +
                                          g("SQ_INSTS_VALU_FLOPS_FP32_TRANS", 0.0)),
             "fp32_matrix_flops": 512.0 * g("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0),
             "source_hash": source_hash(k) if k in KERNEL_SOURCES else None}
        if g("SQ_WAVES"):
            e["valu_insts_per_wave"] = g("SQ_INSTS_VALU", 0.0) / g("SQ_WAVES")
        kernels[k] = e
    return {"workload": workload, "kernels": kernels}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-fetch", required=True)
    b.add_argument("--copy-write", required=True)
    b.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    b.add_argument("--workload", required=True)
    b.add_argument("--out", required=True)
    c = sub.add_parser("compute")
    c.add_argument("--pmc", action="append", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_markdown(args.dir))
    elif args.cmd == "compute":
        t = compute(args.pmc, args.workload)
        with open(args.out, "w") as fh:
            json.dump(t, fh, indent=1)
        print(json.dumps({k: {"fp64_gflop": round(v["fp64_vector_flops"] / 1e9, 3),
                              "fp32_gflop": round(v["fp32_vector_flops"] / 1e9, 3),
                              "mfma_f32_gflop": round(v["fp32_matrix_flops"] / 1e9, 3)}
                          for k, v in t["kernels"].items()}))
    else:
        t = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write,
                    args.copy_bytes, args.workload)
        with open(args.out, "w") as fh:
            json.dump(t, fh, indent=1)
        print(json.dumps({k: round(v["bytes_per_launch"] / 1e9, 3)
                          for k, v in t["kernels"].items()}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
