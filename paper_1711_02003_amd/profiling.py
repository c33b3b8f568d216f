"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1711_02003_amd.profiling trace <kernel_trace.csv> <out.md> <kernel>
        <timed dispatches> "<command>" [first]
    python -m paper_1711_02003_amd.profiling traffic <fetch counter_collection.csv>
        <write counter_collection.csv> <kernel> <timed dispatches> <nodes> <out.txt>
        "<commands>"
    python -m paper_1711_02003_amd.profiling forms <kernel_trace.csv> <out.md> <timed dispatches>
        "<command>"

<kernel> is a key of KERNELS: k_step_compact (the FP32 compact-state sweep
of the headline), k_step_fused (the FP32 pair-state sweep, periodic) or
geo_split (the FP32 split step of a lattice with geometry: three kernels per
step, reported per kernel and per step).  The benchmark first times
candidate launch shapes of a kernel (same kernel names), then runs the
timed region; the summaries therefore report the last <timed dispatches>
dispatches of each named kernel (the timed region; with `first`, the
timed region of the first run long enough to be one, for a full benchmark
run whose later forms run the same kernel on other lattices) besides the
per-kernel totals.

The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by
what the same counters read for a plain device copy of known size (the
benchmark's 2 GiB copy probe): on this hardware FETCH_SIZE counts half of
the bytes such a copy reads.  The result is bytes per launch of the named
kernel (per step, summed over its kernels, for geo_split) that leave the L2
towards memory, tagged with a hash of the kernel
sources so that a stale figure is never reported for changed code.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 << 30  # the copy probe moves 2 GiB in and 2 GiB out per dispatch
# Per measured kernel: the sources its code comes from, its algorithmic bytes
# per (fluid) node and step (FP32), and the patterns of its dispatch names
# (one per kernel of a step).  Pair state: every population pair read once
# and written once, 2 x 38 x 4.  Compact state: 19 totals and 5 colour
# scalars read once and written once, 2 x (19 x 4 + 20).  Geometry: the
# pairs and the node's link word, 2 x 38 x 4 + 4 (the split step also writes
# and reads back psi and 12 moments; that is overhead, not algorithm).
KERNELS = {
    "k_step_compact": (["paper_1711_02003_amd/csrc/lbcg_compact.hip", "paper_1711_02003_amd/csrc/lbcg_compact_sweep.h",
                        "paper_1711_02003_amd/csrc/lbcg_device.h"],
                       2 * (19 * 4 + 20), [r"k_step_compact<false, \d+, float>"]),
    "k_step_fused": (["paper_1711_02003_amd/csrc/lbcg_fused.hip", "paper_1711_02003_amd/csrc/lbcg_device.h"],
                     2 * 38 * 4, [r"k_step_fused<float, float, \d, false, false>"]),
    "geo_split": (["paper_1711_02003_amd/csrc/lbcg_geo.hip", "paper_1711_02003_amd/csrc/lbcg_device.h"],
                  2 * 38 * 4 + 4, [r"k_geo_moments<float>", r"k_geo_collide<float>", r"k_geo_boundary<float>"]),
    "geo_split_compact": (["paper_1711_02003_amd/csrc/lbcg_geo.hip", "paper_1711_02003_amd/csrc/lbcg_device.h",
                           "paper_1711_02003_amd/csrc/lbcg_compact_sweep.h"],
                          2 * (19 * 4 + 20) + 4,
                          [r"k_cgeo_moments<float>", r"k_cgeo_collide<float>", r"k_cgeo_boundary<float>"]),
}


def _matches(rows, pattern):
    return [r for r in rows if re.search(pattern, r["Kernel_Name"])]


def kernel_hash(kernel: str) -> str:
    """Hash of the kernel's sources and of the options its object is built with."""
    from paper_1711_02003_amd import build

    h = hashlib.sha256()
    for p in KERNELS[kernel][0]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
        if p.endswith(".hip"):
            h.update(" ".join(build.compile_flags(p)).encode())
    return h.hexdigest()[:16]


def _short(name: str, n: int = 90) -> str:
    return name if len(name) <= n else name[:n - 3] + "..."


def _first_run(ks, timed):
    """The last `timed` dispatches of the first run of at least `timed`
    consecutive dispatches with one launch shape: the headline's warm-up and
    timed steps, after the tuner's trials (runs of 6 per shape) and before
    the forms that later run the same kernel on other lattices."""
    runs, cur = [], []
    for r in ks:
        key = (r["Grid_Size_X"], r["Workgroup_Size_X"])
        if cur and (cur[-1]["Grid_Size_X"], cur[-1]["Workgroup_Size_X"]) != key:
            runs.append(cur)
            cur = []
        cur.append(r)
    if cur:
        runs.append(cur)
    for run in runs:
        if len(run) >= timed:
            return run[-timed:]
    return ks[-timed:]


def trace_summary(trace_csv, out_md, kernel_sub, timed, command, region="last"):
    rows = list(csv.DictReader(open(trace_csv)))
    per = collections.defaultdict(list)
    for r in rows:
        per[r["Kernel_Name"]].append(r)
    total = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows) or 1
    lines = [f"# rocprofv3 kernel trace: {os.path.basename(out_md).rsplit('.', 1)[0]}", "",
             f"Command: `{command}`", "", "All dispatches per kernel:", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for name, rs in sorted(per.items(), key=lambda kv: -sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                                                            for r in kv[1])):
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rs]
        lines.append(f"| `{_short(name)}` | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} | "
                     f"{100 * sum(d) * 1e3 / total:.1f} |")
    per_step = 0.0
    for pat in KERNELS[kernel_sub][2]:
        ks = _matches(rows, pat)
        ks.sort(key=lambda r: int(r["Start_Timestamp"]))
        tail = _first_run(ks, timed) if region == "first" else ks[-timed:]
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tail]
        span = (int(tail[-1]["End_Timestamp"]) - int(tail[0]["Start_Timestamp"])) / 1e3
        grid = {(r["Grid_Size_X"], r["Workgroup_Size_X"]) for r in tail}
        names = sorted({_short(r["Kernel_Name"], 70) for r in tail})
        per_step += sum(d) / len(d)
        which = (f"the last {len(tail)} dispatches of the first run of at least {timed} consecutive same-shape "
                 "dispatches" if region == "first" else f"the last {len(tail)} dispatches")
        lines += ["", f"Timed region: {which} matching `{pat}` ({', '.join(names)}; "
                      f"grid, workgroup = {sorted(grid)}):", "",
                  f"- average duration: {sum(d) / len(d):.1f} us (min {min(d):.1f}, max {max(d):.1f})",
                  f"- first start to last end: {span:.1f} us = {span / len(d):.1f} us per dispatch"]
    if len(KERNELS[kernel_sub][2]) > 1:
        lines += ["", f"Per step (sum of the kernels' average durations): {per_step:.1f} us"]
    txt = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(txt)
    return txt


def _kernel_values(counter_csv, counter, kernel_sub, timed):
    """Per step: the counter summed over the kernels of a step, averaged over
    the last `timed` dispatches of each; and the copy calibration."""
    rows = [r for r in csv.DictReader(open(counter_csv)) if r["Counter_Name"] == counter]
    copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    total, n = 0.0, None
    for pat in KERNELS[kernel_sub][2]:
        ks = _matches(rows, pat)
        ks.sort(key=lambda r: int(r["Dispatch_Id"]))
        vals = [float(r["Counter_Value"]) for r in ks[-timed:]]
        total += sum(vals) / len(vals)
        n = len(vals) if n is None else min(n, len(vals))
    return total, n, (max(copy) if copy else None)


def traffic_summary(fetch_csv, write_csv, kernel_sub, timed, nodes, out_txt, commands):
    fkib, nf, fc = _kernel_values(fetch_csv, "FETCH_SIZE", kernel_sub, timed)
    wkib, nw, wc = _kernel_values(write_csv, "WRITE_SIZE", kernel_sub, timed)
    f_fac = COPY_BYTES / (fc * 1024)
    w_fac = COPY_BYTES / (wc * 1024)
    fb, wb = fkib * 1024 * f_fac, wkib * 1024 * w_fac
    alg = KERNELS[kernel_sub][1] * nodes / 2  # read (or write) bytes of the algorithm
    lines = [
        f"kernel: {kernel_sub}",
        f"kernel_hash: {kernel_hash(kernel_sub)}",
        f"commands: {commands}",
        f"kernels_per_step: {len(KERNELS[kernel_sub][2])}",
        f"timed_dispatches: {nf} fetch, {nw} write (per kernel)",
        f"fetch_kib_per_launch: {fkib:.1f}",
        f"write_kib_per_launch: {wkib:.1f}",
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


# Per benchmark form: its kernels, as patterns of their dispatch names
# (FP16 instantiations appear mangled).
FORM_KERNELS = [("D3Q19 256³ droplets, FP32 pairs", r"k_step_fused<float, float, \d, false, false>"),
                ("D3Q19 256³ droplets, FP16 compact", r"k_step_compactILb0ELi\d+EDF16_"),
                ("D3Q19 256³ droplets, FP16 pairs", r"k_step_fusedIDF16_fLi\dELb0ELb0E"),
                ("D2Q9 4096² droplets, FP32 compact", r"k_step_compact2d<false>"),
                ("D2Q9 4096² droplets, FP32", r"k_step_fused2d<float, false>"),
                ("D2Q9 junction 8192×2048, FP32", r"k_step_fused2d<float, true>"),
                ("D3Q19 junction 512×128×64, FP32 split: moments", r"k_geo_moments<float>"),
                ("D3Q19 junction 512×128×64, FP32 split: collision", r"k_geo_collide<float>"),
                ("D3Q19 junction 512×128×64, FP32 split: inlets, outlets", r"k_geo_boundary<float>"),
                ("D3Q19 junction 512×128×64, FP32 compact split: moments", r"k_cgeo_moments<float>"),
                ("D3Q19 junction 512×128×64, FP32 compact split: collision", r"k_cgeo_collide<float>"),
                ("D3Q19 junction 512×128×64, FP32 compact split: inlets, outlets", r"k_cgeo_boundary<float>"),
                ("D3Q19 junction 512×128×64, FP16 compact split: moments", r"k_cgeo_momentsIDF16_"),
                ("D3Q19 junction 512×128×64, FP16 compact split: collision", r"k_cgeo_collideIDF16_"),
                ("D3Q19 junction 512×128×64, FP16 compact split: inlets, outlets", r"k_cgeo_boundaryIDF16_"),
                ("D3Q19 junction 512×128×64, FP16 split: moments", r"k_geo_momentsIDF16_"),
                ("D3Q19 junction 512×128×64, FP16 split: collision", r"k_geo_collideIDF16_"),
                ("D3Q19 junction 512×128×64, FP16 split: inlets, outlets", r"k_geo_boundaryIDF16_"),
                ("D3Q19 64 boxes batched, FP32 pairs", r"k_step_fused_batch<float, float, \d, false>"),
                ("D3Q19 64 boxes batched, FP32 compact", r"k_step_compact_batch")]


def forms_summary(trace_csv, out_md, timed, command):
    """Per benchmark form, the last `timed` dispatches of its fused kernel
    (each form's timed region comes after its warm-up and tuning)."""
    rows = list(csv.DictReader(open(trace_csv)))
    lines = ["# rocprofv3 kernel trace: benchmark forms (fused sweeps)", "",
             f"Command: `{command}`", "",
             f"Each form times {timed} steps after its warm-up (and, for the fused sweeps, after the tuner's "
             f"trial launches); the rows below take, per kernel, the last {timed} dispatches of its first run "
             f"of at least {timed} consecutive same-shape dispatches, i.e. that form's timed region (later "
             "forms run some of these kernels again on other lattices).", "",
             "| form | kernel | dispatches in run | avg us (timed) | min us | max us | "
             "first start to last end, per dispatch us |",
             "|---|---|---|---|---|---|---|"]
    for form, pat in FORM_KERNELS:
        ks = sorted(_matches(rows, pat), key=lambda r: int(r["Start_Timestamp"]))
        if not ks:
            continue
        tail = _first_run(ks, timed)
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tail]
        span = (int(tail[-1]["End_Timestamp"]) - int(tail[0]["Start_Timestamp"])) / 1e3
        lines.append(f"| {form} | `{pat}` | {len(ks)} | {sum(d) / len(d):.1f} | "
                     f"{min(d):.1f} | {max(d):.1f} | {span / len(d):.1f} |")
    txt = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(txt)
    return txt


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        print(trace_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6],
                            sys.argv[7] if len(sys.argv) > 7 else "last"))
    elif mode == "traffic":
        print(traffic_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]),
                              sys.argv[7], sys.argv[8]))
    elif mode == "forms":
        print(forms_summary(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5]))
    else:
        raise SystemExit(__doc__)
