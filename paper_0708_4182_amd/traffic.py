"""HBM traffic per step-kernel launch from two rocprofv3 counter passes.

    python -m paper_0708_4182_amd.traffic FETCH_DIR WRITE_DIR --tile fused8:512x0

FETCH_DIR and WRITE_DIR hold the pmc_counter_collection.csv of a
``rocprofv3 --pmc FETCH_SIZE`` and a ``--pmc WRITE_SIZE`` run of the profiling
driver (csrc/step_driver.cpp) on the 8192 x 2048 channel (one run per tile and
counter).  A launch of a multi-step kernel (k_stepk) covers two or three time
steps and, like every step kernel, reads and writes each population once: its
algorithmic bytes per launch are the same 18 values per fluid node.  Each counter is scaled by what it reads for the copy of one FP32
population buffer in the same run (k_stream_copy, 9 * nx * ny * 4 bytes each
way; torch's __amd_rocclr_copyBuffer in runs of bench.py).  The result is
merged into profiles/traffic.json, keyed by storage and tile and stamped with
the hash of the kernel source, and printed as a markdown table.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_0708_4182_amd", "csrc", "lbm_kernels.hip")
OUT = os.path.join(ROOT, "profiles", "traffic.json")
STORAGE_NAMES = {0: "f32", 1: "f16", 2: "bf16"}
BYTES = {0: 4, 1: 2, 2: 2}
STEP_RE = re.compile(r"(k_step(?:k|2|8|_wide|_split)?)<(\d)[^>]*>")


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def per_kernel(csv_dir: str, counter: str):
    """{kernel name: [counter value per dispatch]} from a counter-collection CSV."""
    path = None
    for dirpath, _, files in os.walk(csv_dir):
        for f in files:
            if f.endswith("counter_collection.csv"):
                path = os.path.join(dirpath, f)
    if path is None:
        raise SystemExit(f"no counter_collection.csv under {csv_dir}")
    out = defaultdict(list)
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                out[row["Kernel_Name"]].append((int(row["Grid_Size"]), float(row["Counter_Value"])))
    return out


def mean(v):
    return sum(v) / len(v)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--tile", required=True, help="kernel:BXxROWS the runs used")
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()

    from paper_0708_4182_amd import inputs as I
    case = I.random_channel_case(nx=args.nx, ny=args.ny)
    fluid = int((case.solid == 0).sum())
    copy_bytes = 9 * args.nx * args.ny * 4

    kernel, t = args.tile.split(":")
    bx, rows = (int(v) for v in t.split("x"))
    tile = [bx, rows, kernel]

    fetch = per_kernel(args.fetch_dir, "FETCH_SIZE")
    write = per_kernel(args.write_dir, "WRITE_SIZE")

    def copy_kib(d):
        # the library's streaming copy (the profiling driver's calibration), else torch's device copy
        for key in ("k_stream_copy", "copyBuffer"):
            vals = [v for name, rows_ in d.items() if key in name for g, v in rows_]
            if vals:
                big = max(vals)
                return mean([v for v in vals if v > 0.9 * big])
        raise SystemExit("no calibration copy dispatch in the counter runs")

    ff = copy_bytes / 1024 / copy_kib(fetch)
    wf = copy_bytes / 1024 / copy_kib(write)
    table = json.load(open(args.out)) if os.path.exists(args.out) else {}
    table["_note"] = ("HBM bytes per step-kernel launch on the 8192x2048 random-step channel, from rocprofv3 "
                      "--pmc FETCH_SIZE and --pmc WRITE_SIZE passes (KiB per dispatch), each scaled by copy "
                      "bytes / counter for the FP32 population-buffer copy timed in the same run; written by "
                      "python -m paper_0708_4182_amd.traffic")
    sha = kernel_sha()
    lines = ["| kernel | storage | tile | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB | total MB | "
             "algorithmic MB | ratio |", "|---|---|---|---|---|---|---|---|---|---|"]
    for name in sorted(fetch):
        m = STEP_RE.search(name)
        if not m or name not in write:
            continue
        st = int(m.group(2))
        fk = mean([v for _, v in fetch[name]])
        wk = mean([v for _, v in write[name]])
        rb, wb = fk * 1024 * ff, wk * 1024 * wf
        alg = 18 * BYTES[st] * fluid
        rec = dict(kernel_sha=sha, tile=tile, fetch_kib=round(fk, 1), write_kib=round(wk, 1),
                   read_bytes=int(rb), write_bytes=int(wb), bytes_per_launch=int(rb + wb),
                   algorithmic_bytes=alg, ratio_to_algorithmic=round((rb + wb) / alg, 4),
                   calibration=dict(copy_bytes=copy_bytes, fetch_factor=round(ff, 4), write_factor=round(wf, 4)))
        key = STORAGE_NAMES[st]
        entries = [e for e in table.get(key, []) if isinstance(e, dict) and e.get("kernel_sha") == sha
                   and list(e.get("tile", [])) != tile] if isinstance(table.get(key), list) else []
        table[key] = entries + [rec]
        lines.append(f"| {m.group(0)} | {key} | {bx}x{rows} {kernel} | {fk:,.1f} | "
                     f"{wk:,.1f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | {(rb + wb) / 1e6:.1f} | {alg / 1e6:.1f} | "
                     f"{(rb + wb) / alg:.3f} |")
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(f"calibration: copy {copy_bytes} B, FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {wf:.4f}; fluid nodes {fluid}")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
