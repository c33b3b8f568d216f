"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1711_02003_amd.profiling trace <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1711_02003_amd.profiling traffic <fetch counter_collection.csv>
        <write counter_collection.csv> <kernel substring> <nodes> <out.txt> "<commands>"

The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by
what the same counters read for a plain device copy of known size (the
benchmark's 2 GiB copy probe): on this hardware FETCH_SIZE counts half of
the bytes such a copy reads.  The result is HBM bytes per launch of the named
kernel, tagged with a hash of the kernel sources so a stale figure is never
reported for changed code.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1711_02003_amd/csrc/lbcg_fused.hip", "paper_1711_02003_amd/csrc/lbcg_device.h"]
COPY_BYTES = 2 << 30  # the copy probe moves 2 GiB in and 2 GiB out per dispatch


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def trace_summary(stats_csv: str, out_md: str, command: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel trace: {os.path.basename(out_md)[:-3]}", "",
             f"Command: `{command}`", "",
             "| kernel | calls | avg us | min us | max us | share % |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f} |")
    txt = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(txt)
    return txt


def _per_kernel(counter_csv: str, counter: str):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic_summary(fetch_csv, write_csv, kernel_sub, nodes, out_txt, commands):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")

    def copy_kib(agg):
        vals = [v for k, vs in agg.items() if "copyBuffer" in k or "copy" in k.lower() for v in vs]
        return max(vals) if vals else None

    fc, wc = copy_kib(fetch), copy_kib(write)
    f_fac = COPY_BYTES / (fc * 1024) if fc else None
    w_fac = COPY_BYTES / (wc * 1024) if wc else None
    kf = [v for k, vs in fetch.items() if kernel_sub in k for v in vs]
    kw = [v for k, vs in write.items() if kernel_sub in k for v in vs]
    fkib = sum(kf) / len(kf)
    wkib = sum(kw) / len(kw)
    fb = fkib * 1024 * f_fac
    wb = wkib * 1024 * w_fac
    alg = 2 * 38 * 4 * nodes / 2  # read (or write) bytes of the algorithm
    lines = [
        f"kernel: {kernel_sub}",
        f"kernel_hash: {kernel_hash()}",
        f"commands: {commands}",
        f"dispatches: {len(kf)} fetch, {len(kw)} write",
        f"fetch_kib_per_dispatch: {fkib:.1f}",
        f"write_kib_per_dispatch: {wkib:.1f}",
        f"copy_probe_fetch_kib: {fc}",
        f"copy_probe_write_kib: {wc}",
        f"fetch_scale: {f_fac:.4f}",
        f"write_scale: {w_fac:.4f}",
        f"hbm_read_bytes_per_launch: {fb:.0f}",
        f"hbm_write_bytes_per_launch: {wb:.0f}",
        f"hbm_bytes_per_launch: {fb + wb:.0f}",
        f"algorithmic_bytes_per_launch: {2 * alg:.0f}",
        f"read_over_algorithmic: {fb / alg:.4f}",
        f"write_over_algorithmic: {wb / alg:.4f}",
    ]
    txt = "\n".join(lines) + "\n"
    with open(out_txt, "w") as f:
        f.write(txt)
    return txt


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        print(trace_summary(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif mode == "traffic":
        print(traffic_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6],
                              sys.argv[7]))
    else:
        raise SystemExit(__doc__)
