"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1711_02003_amd.profiling trace <kernel_trace.csv> <out.md> <kernel substring>
        <timed dispatches> "<command>"
    python -m paper_1711_02003_amd.profiling traffic <fetch counter_collection.csv>
        <write counter_collection.csv> <kernel substring> <timed dispatches> <nodes> <out.txt>
        "<commands>"   (kernel substring k_step_compact or k_step_fused)
    python -m paper_1711_02003_amd.profiling forms <kernel_trace.csv> <out.md> <timed dispatches>
        "<command>"

The benchmark first times candidate launch shapes of the kernel (same kernel
name), then runs the timed region; both summaries therefore report the last
<timed dispatches> dispatches of the named kernel (the timed region) besides
the per-kernel totals.

The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by
what the same counters read for a plain device copy of known size (the
benchmark's 2 GiB copy probe): on this hardware FETCH_SIZE counts half of
the bytes such a copy reads.  The result is bytes per launch of the named
kernel that leave the L2 towards memory, tagged with a hash of the kernel
sources so that a stale figure is never reported for changed code.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 2 << 30  # the copy probe moves 2 GiB in and 2 GiB out per dispatch
# Per headline kernel: the sources its code comes from and its algorithmic
# bytes per node and step (FP32).  Pair state: every population pair read
# once and written once, 2 x 38 x 4.  Compact state: 19 totals and 5
# colour scalars read once and written once, 2 x (19 x 4 + 20).
KERNELS = {
    "k_step_compact": (["paper_1711_02003_amd/csrc/lbcg_compact.hip", "paper_1711_02003_amd/csrc/lbcg_compact_sweep.h",
                        "paper_1711_02003_amd/csrc/lbcg_device.h"],
                       2 * (19 * 4 + 20)),
    "k_step_fused": (["paper_1711_02003_amd/csrc/lbcg_fused.hip", "paper_1711_02003_amd/csrc/lbcg_device.h"],
                     2 * 38 * 4),
}


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


def trace_summary(trace_csv, out_md, kernel_sub, timed, command):
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
    ks = [r for r in rows if kernel_sub in r["Kernel_Name"]]
    ks.sort(key=lambda r: int(r["Start_Timestamp"]))
    tail = ks[-timed:]
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tail]
    span = (int(tail[-1]["End_Timestamp"]) - int(tail[0]["Start_Timestamp"])) / 1e3
    grid = {(r["Grid_Size_X"], r["Workgroup_Size_X"]) for r in tail}
    lines += ["", f"Timed region: the last {len(tail)} dispatches of `{kernel_sub}` "
                  f"(grid, workgroup = {sorted(grid)}):", "",
              f"- average duration: {sum(d) / len(d):.1f} us (min {min(d):.1f}, max {max(d):.1f})",
              f"- first start to last end: {span:.1f} us = {span / len(d):.1f} us per dispatch"]
    txt = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(txt)
    return txt


def _kernel_values(counter_csv, counter, kernel_sub, timed):
    rows = [r for r in csv.DictReader(open(counter_csv)) if r["Counter_Name"] == counter]
    copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    ks = [r for r in rows if kernel_sub in r["Kernel_Name"]]
    ks.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in ks[-timed:]], (max(copy) if copy else None)


def traffic_summary(fetch_csv, write_csv, kernel_sub, timed, nodes, out_txt, commands):
    kf, fc = _kernel_values(fetch_csv, "FETCH_SIZE", kernel_sub, timed)
    kw, wc = _kernel_values(write_csv, "WRITE_SIZE", kernel_sub, timed)
    f_fac = COPY_BYTES / (fc * 1024)
    w_fac = COPY_BYTES / (wc * 1024)
    fkib, wkib = sum(kf) / len(kf), sum(kw) / len(kw)
    fb, wb = fkib * 1024 * f_fac, wkib * 1024 * w_fac
    alg = KERNELS[kernel_sub][1] * nodes / 2  # read (or write) bytes of the algorithm
    lines = [
        f"kernel: {kernel_sub}",
        f"kernel_hash: {kernel_hash(kernel_sub)}",
        f"commands: {commands}",
        f"timed_dispatches: {len(kf)} fetch, {len(kw)} write",
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


FORM_KERNELS = [("D2Q9 4096² droplets, FP32 compact", "void lbcg::(anonymous namespace)::k_step_compact2d<false>"),
                ("D2Q9 4096² droplets, FP32", "void lbcg::k_step_fused2d<float, false>"),
                ("D2Q9 junction 8192×2048, FP32", "void lbcg::k_step_fused2d<float, true>"),
                ("D3Q19 junction 512×128×64, FP32", "void lbcg::k_step_fused<float, float, 8, true>"),
                ("D3Q19 junction 512×128×64, FP16", "_ZN4lbcg12k_step_fusedIDF16_fLi8ELb1EE"),
                ("D3Q19 64 boxes batched, FP32 compact", "lbcg::(anonymous namespace)::k_step_compact_batch")]


def forms_summary(trace_csv, out_md, timed, command):
    """Per benchmark form, the last `timed` dispatches of its fused kernel
    (each form's timed region comes after its warm-up and tuning)."""
    rows = list(csv.DictReader(open(trace_csv)))
    lines = ["# rocprofv3 kernel trace: benchmark forms (fused sweeps)", "",
             f"Command: `{command}`", "",
             f"Each form times {timed} steps after its warm-up (and, for the fused sweeps, after the tuner's "
             f"trial launches); the rows below take the last {timed} dispatches of each kernel, i.e. that "
             "form's timed region.", "",
             "| form | kernel | dispatches in run | avg us (timed) | min us | max us | "
             "first start to last end, per dispatch us |",
             "|---|---|---|---|---|---|---|"]
    for form, prefix in FORM_KERNELS:
        ks = sorted([r for r in rows if r["Kernel_Name"].startswith(prefix)], key=lambda r: int(r["Start_Timestamp"]))
        if not ks:
            continue
        tail = ks[-timed:]
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tail]
        span = (int(tail[-1]["End_Timestamp"]) - int(tail[0]["Start_Timestamp"])) / 1e3
        lines.append(f"| {form} | `{prefix.replace('void lbcg::', '')}` | {len(ks)} | {sum(d) / len(d):.1f} | "
                     f"{min(d):.1f} | {max(d):.1f} | {span / len(d):.1f} |")
    txt = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(txt)
    return txt


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        print(trace_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6]))
    elif mode == "traffic":
        print(traffic_summary(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), int(sys.argv[6]),
                              sys.argv[7], sys.argv[8]))
    elif mode == "forms":
        print(forms_summary(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5]))
    else:
        raise SystemExit(__doc__)
