"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_1907_01995_amd.profsum stats  <prefix>_kernel_stats.csv
    python -m paper_1907_01995_amd.profsum pmc    <prefix>_counter_collection.csv COUNTER
    python -m paper_1907_01995_amd.profsum traffic --fetch F.csv --write W.csv --kernel k_sweep2 \
        --copy-bytes BYTES --out profiles/traffic_<kernel>_<workload>.json

`stats` prints calls, total and average duration per kernel (from a
`--kernel-trace --stats --output-format csv` run).  `pmc` prints the average
value of one counter per dispatch, per kernel.  `traffic` turns the FETCH_SIZE
and WRITE_SIZE of a kernel (KiB per dispatch) into bytes per launch, each scaled
by what the same counter reads for the plain device copy of known size that
`bench.py --calibrate-copy` adds to the run (the copy dispatches within 10% of
the largest), and records a hash of the kernel's sources so that a reader can tell
whether the counters still describe the current kernel.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {"k_sweep2": ["csrc/sweep.hip", "csrc/rac_internal.h"],
                  "k_tsweep": ["csrc/tsweep.hip", "csrc/batch.cpp", "csrc/rac_internal.h"]}


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^(]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    m = re.search(r"(__amd_rocclr_\w+)", name)
    return m.group(1) if m else name.split("(")[0][:60]


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of %s in %s" % (names, list(row)))


def stats(path):
    out = []
    for r in _rows(path):
        name = short_name(_col(r, "Name", "KernelName", "Kernel_Name"))
        calls = int(_col(r, "Calls"))
        total = float(_col(r, "TotalDurationNs", "Total_Duration_Ns"))
        out.append((name, calls, total / 1e3, total / max(calls, 1) / 1e3))
    out.sort(key=lambda t: -t[2])
    return out


def pmc_values(path, counter):
    acc = defaultdict(list)
    for r in _rows(path):
        if _col(r, "Counter_Name", "CounterName") != counter:
            continue
        name = short_name(_col(r, "Kernel_Name", "KernelName", "Name"))
        acc[name].append(float(_col(r, "Counter_Value", "CounterValue")))
    return acc


def pmc(path, counter):
    return {k: (len(v), sum(v) / len(v)) for k, v in pmc_values(path, counter).items()}


def copy_calibration(path, counter):
    """Average counter value of the calibration copies: the copy-kernel dispatches
    within 10% of the largest one (the calibration copies are the run's largest, all of
    one size; smaller copies, such as a workload's uploads, are left out)."""
    vals = [v for k, vs in pmc_values(path, counter).items() if "copy" in k.lower() for v in vs]
    if not vals:
        raise SystemExit("no copy kernel in the counter file (run bench.py with --calibrate-copy)")
    top = max(vals)
    big = [v for v in vals if v >= 0.9 * top]
    return len(big), sum(big) / len(big)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("pmc")
    b.add_argument("csv")
    b.add_argument("counter")
    c = sub.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--copy-bytes", type=float, required=True, help="bytes read (= bytes written) per copy")
    c.add_argument("--launch-bytes", type=float, default=None, help="algorithmic bytes per launch")
    c.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print("%-48s %7s %12s %10s" % ("kernel", "calls", "total_us", "avg_us"))
        for name, calls, tot, avg in stats(args.csv):
            print("%-48s %7d %12.1f %10.2f" % (name, calls, tot, avg))
        return
    if args.cmd == "pmc":
        for k, (n, v) in sorted(pmc(args.csv, args.counter).items(), key=lambda kv: -kv[1][1]):
            print("%-48s %6d dispatches  %s avg %.1f" % (k, n, args.counter, v))
        return
    fetch, write = pmc(args.fetch, "FETCH_SIZE"), pmc(args.write, "WRITE_SIZE")
    fk = [k for k in fetch if k.startswith(args.kernel)]
    wk = [k for k in write if k.startswith(args.kernel)]
    if not fk or not wk:
        raise SystemExit("kernel %s not in the counter files" % args.kernel)
    ncf, cf = copy_calibration(args.fetch, "FETCH_SIZE")
    ncw, cw = copy_calibration(args.write, "WRITE_SIZE")
    sf = args.copy_bytes / (cf * 1024.0)      # bytes per counted KiB, reads
    sw = args.copy_bytes / (cw * 1024.0)      # bytes per counted KiB, writes
    f_kib = fetch[fk[0]][1]
    w_kib = write[wk[0]][1]
    rec = {"kernel": fk[0], "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
           "copy_dispatches": [ncf, ncw], "copy_bytes": args.copy_bytes,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": sf, "write_scale": sw,
           "traffic_bytes_per_launch": f_kib * 1024.0 * sf + w_kib * 1024.0 * sw,
           "source_sha256": source_hash(args.kernel)}
    if args.launch_bytes:
        rec["algorithmic_bytes_per_launch"] = args.launch_bytes
        rec["traffic_over_algorithmic"] = rec["traffic_bytes_per_launch"] / args.launch_bytes
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    sys.exit(main())
