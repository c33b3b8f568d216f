"""Benchmark of the regularized colour-gradient D3Q19 step on one MI355X.

Workload: the 27-droplet periodic D3Q19 box, 256^3, FP32 storage and
arithmetic (tau_R = 1, tau_B = 0.6, A = 0.005, beta = 0.7), fused
single-pass kernel on the compact state (receiver-side recolouring; the
pair-state sweep is reported among the forms).  A step is one full time step
of every node (both colours).  Prints one JSON line:

  value      whole-job two-component MLUPS (fluid nodes x steps / time), inputs
             resident in HBM, timed with HIP events on the simulation's stream;
  roofline   HBM roofline of the step's kernel: algorithmic bytes per node
             (read + write the state once: compact 2 x (19 x 4 + 20) = 192 B,
             pair state 2 x 38 x 4 = 304 B; with --precision f16, compact
             2 x (19 x 2 + 12) = 100 B, pair state 152 B) x nodes / average
             kernel time,
             against 8 TB/s; traffic = HBM bytes per launch from the rocprofv3
             FETCH_SIZE / WRITE_SIZE counters scaled by a copy-kernel
             calibration (null when the kernel source changed since the
             counters were taken);
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample;
  copy_probe achievable bandwidth of plain streams on this device (context):
             hand-written copy, read-only and write-only kernels and torch's
             device copy;
  forms      the other forms of the step, each measured on its own workload:
             pair_f32 (the same lattice on the pair-state sweep: per
             population its total and minority share), f16 (the same lattice
             with FP16 storage, compact and pair state), d2q9 (a 4096^2 D2Q9 box: compact and
             pair-state strip sweeps and the two-pass generic kernel),
             focusing2d (the 8192 x 2048 D2Q9 junction), focusing (the
             512 x 128 x 64 D3Q19 flow-focusing junction, FP32 and FP16),
             batched, batched_compact and batched_compact_f16 (64 uneven
             periodic boxes in one launch per time level, pair and compact
             state, the latter also with FP16 storage, vs the same boxes
             stepped one after another) and served (a Poisson stream of
             step-emulsifier requests through the continuous-batching server
             vs one request at a time; p50 / p99 time to result).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FORMS = ("pair_f32", "f16", "d2q9", "focusing2d", "focusing", "batched", "batched_compact", "batched_compact_f16",
         "served")
TRAFFIC_FILES = {"k_step_compact": os.path.join(ROOT, "profiles", "compact_d3q19_f32_256_traffic.txt"),
                 "k_step_fused": os.path.join(ROOT, "profiles", "fused_d3q19_f32_256_traffic.txt"),
                 "geo_split": os.path.join(ROOT, "profiles", "geo_split_d3q19_f32_junction_traffic.txt"),
                 "geo_split_compact": os.path.join(ROOT, "profiles", "geo_split_compact_d3q19_f32_junction_traffic.txt")}


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    current."""
    path = TRAFFIC_FILES[kernel]
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    from paper_1711_02003_amd.profiling import kernel_hash
    if vals.get("kernel_hash") != kernel_hash(kernel):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(torch, nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth on this device: the hand-written probes of
    libhbmprobe.so (a copy, a read-only and a write-only stream; 8- or 16-byte
    loads per lane, non-temporal stores; several grid sizes, best kept) and
    torch's device copy, each on a 2 GiB buffer, timed with HIP events on the
    stream they run on."""
    import ctypes as C

    from paper_1711_02003_amd import build as hipbuild
    lib = C.CDLL(hipbuild.PROBE_LIB)
    for fn in (lib.hbm_probe_copy, lib.hbm_probe_read, lib.hbm_probe_write):
        fn.restype = C.c_int
    lib.hbm_probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p]
    lib.hbm_probe_read.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    lib.hbm_probe_write.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    stream = torch.cuda.Stream()
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(2, dtype=torch.int64, device="cuda")
    src.fill_(1.0)
    torch.cuda.synchronize()
    h = stream.cuda_stream

    def timed(launch):
        for _ in range(2):
            assert launch() == 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            assert launch() == 0
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"bytes": nbytes}
    for kind, moved in (("copy", 2 * nbytes), ("read", nbytes), ("write", nbytes)):
        best, shape = 0.0, None
        for lane in ((8, 16) if kind != "write" else (8,)):
            for per_cu in (4, 16, 64):
                if kind == "copy":
                    ms = timed(lambda: lib.hbm_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, lane, per_cu, h))
                elif kind == "read":
                    ms = timed(lambda: lib.hbm_probe_read(src.data_ptr(), nbytes, sink.data_ptr(), lane, per_cu, h))
                else:
                    ms = timed(lambda: lib.hbm_probe_write(dst.data_ptr(), nbytes, per_cu, h))
                gbps = moved / ms / 1e6
                if gbps > best:
                    best, shape = gbps, {"lane_bytes": lane, "blocks_per_cu": per_cu}
        out[kind] = {"gbps": round(best, 1), **shape}
    with torch.cuda.stream(stream):
        ms = timed(lambda: (dst.copy_(src), 0)[1])
    out["torch_copy_gbps"] = round(2 * nbytes / ms / 1e6, 1)
    out["gbps"] = out["copy"]["gbps"]
    del src, dst, sink
    return out


def host_info():
    """The host the CPU baseline runs on: logical CPUs, CPU model, and the
    CPUs this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, steps=16, threads=16, steps_1t=2):
    """The FP64 oracle on this host: `steps` steps of the full lattice on
    `threads` threads (the value), and `steps_1t` steps on one thread."""
    import oracle
    from tests.helpers import oracle_for
    oracle.build(force=False)
    o = oracle_for(oracle, w, threads=threads)
    t = time.time()
    o.step(steps)
    dt = time.time() - t
    del o
    o1 = oracle_for(oracle, w, threads=1)
    t = time.time()
    o1.step(steps_1t)
    dt1 = time.time() - t
    del o1
    return {"value": round(w.fluid_nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} of the workload's {w.steps} steps on the full {w.dims[0]}^3 lattice on "
                      f"{threads} threads, and {steps_1t} steps on 1 thread; FP64, OpenMP over nodes",
            "single_thread_mlups": round(w.fluid_nodes * steps_1t / dt1 / 1e6, 3),
            "host": host_info()}


def time_sim(torch, sim, stream, steps, warmup):
    sim.step(warmup)
    sim.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def pair_f32_form(torch, lbcg, W, size, steps=200, warmup=10):
    w = W.droplets_27(L=size, seed=2)
    stream = torch.cuda.Stream()
    sim = lbcg.Sim.from_workload(w, precision="f32", kernel=lbcg.KERNEL_FUSED, stream=stream.cuda_stream)
    sim.step(1)
    shape = sim.tune()
    ms = time_sim(torch, sim, stream, steps, warmup)
    sim.close()
    mlups = w.fluid_nodes * steps / (ms / 1e3) / 1e6
    gbs = 304 * w.fluid_nodes * steps / (ms / 1e3) / 1e9
    return {"workload": w.name, "storage": "f32 pairs", "mlups": round(mlups, 1),
            "ms_per_step": round(ms / steps, 4), "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node": 304, "rows": shape["rows"],
            "zchunks": shape["zchunks"], "steps": steps}


def f16_form(torch, lbcg, W, size, steps=200, warmup=10):
    """FP16 storage (FP32 arithmetic) on the headline lattice: the compact
    state (100 B per node moved: 19 FP16 totals, M in FP32, V_axis and R_d
    in FP16, read and written once) and the pair state (152 B), each tuned."""
    w = W.droplets_27(L=size, seed=2)
    out = {"workload": w.name, "storage": "f16"}
    for name, kernel, bpn in (("compact", lbcg.KERNEL_COMPACT, 100), ("pairs", lbcg.KERNEL_FUSED, 152)):
        stream = torch.cuda.Stream()
        sim = lbcg.Sim.from_workload(w, precision="f16", kernel=kernel, stream=stream.cuda_stream)
        sim.step(1)
        shape = sim.tune()
        ms = time_sim(torch, sim, stream, steps, warmup)
        sim.close()
        mlups = w.fluid_nodes * steps / (ms / 1e3) / 1e6
        gbs = bpn * w.fluid_nodes * steps / (ms / 1e3) / 1e9
        out[name] = {"mlups": round(mlups, 1), "ms_per_step": round(ms / steps, 4),
                     "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node": bpn,
                     "shape": shape, "steps": steps}
    return out


def d2q9_form(torch, lbcg, W, steps=200, warmup=10):
    """D2Q9 4096^2 with 256 droplets, FP32 storage: the fused strip sweep on
    the compact state (tuned; 104 B per node: every total and the senders'
    4 colour scalars read and written once), on the pair state (tuned; 144 B
    per node: one read and one write of every population pair) and, for
    comparison, the two-pass generic kernel (a psi pass, then the step)
    against the same 144 B."""
    w = W.droplets_2d(n=4096, seed=6)
    out = {"workload": w.name, "storage": "f32", "bytes_per_node": 144, "steps": steps}
    for name, kernel, bpn in (("compact", lbcg.KERNEL_COMPACT, 104), ("fused", lbcg.KERNEL_FUSED, 144),
                              ("generic", lbcg.KERNEL_GENERIC, 144)):
        stream = torch.cuda.Stream()
        sim = lbcg.Sim.from_workload(w, precision="f32", kernel=kernel, stream=stream.cuda_stream)
        sim.step(2)
        if kernel != lbcg.KERNEL_GENERIC:
            sim.tune()
        ms = time_sim(torch, sim, stream, steps, warmup)
        info = sim.launch_info()
        sim.close()
        gbs = bpn * w.fluid_nodes * steps / (ms / 1e3) / 1e9
        out[name] = {"mlups": round(w.fluid_nodes * steps / (ms / 1e3) / 1e6, 1),
                     "ms_per_step": round(ms / steps, 4), "achieved_gbs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_node": bpn}
        if kernel != lbcg.KERNEL_GENERIC:
            out[name]["ychunks"] = info["zchunks"]
    return out


def focusing2d_form(torch, lbcg, W, steps=200, warmup=10):
    """D2Q9 flow-focusing junction 8192 x 2048 (the paper's 2-D device
    geometry: walls, three inlets, an outlet), FP32: the fused strip sweep
    (tuned) and the two-pass generic kernel, fluid-node MLUPS."""
    w = W.flow_focusing_2d(8192, 2048)
    out = {"workload": w.name, "fluid_nodes": w.fluid_nodes, "nodes": w.nodes, "steps": steps}
    for name, kernel in (("fused", lbcg.KERNEL_FUSED), ("generic", lbcg.KERNEL_GENERIC)):
        stream = torch.cuda.Stream()
        sim = lbcg.Sim.from_workload(w, precision="f32", kernel=kernel, stream=stream.cuda_stream)
        sim.step(1)
        if kernel == lbcg.KERNEL_FUSED:
            sim.tune()
        ms = time_sim(torch, sim, stream, steps, warmup)
        info = sim.launch_info()
        sim.close()
        out[name] = {"mlups": round(w.fluid_nodes * steps / (ms / 1e3) / 1e6, 1),
                     "ms_per_step": round(ms / steps, 4),
                     "frac": round((144 + 4) * w.fluid_nodes * steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        if kernel == lbcg.KERNEL_FUSED:
            out[name]["ychunks"] = info["zchunks"]
    return out


def focusing_form(torch, lbcg, W, steps=200, warmup=10, tune=True):
    """Flow-focusing cross junction 512 x 128 x 64 (walls, inlets, outlet):
    FP32 and FP16 storage, fluid-node MLUPS and all-node MLUPS, the tuned
    shape (rows 0: the split step) and its fraction of HBM peak on
    2 x 38 x E + 4 bytes per fluid node; for FP32 on the split step, the
    HBM bytes per step from the committed counter summary (when current);
    and the compact state (FP32 and FP16) on the split step."""
    w = W.flow_focusing(lam=3.0)
    out = {"workload": w.name, "fluid_nodes": w.fluid_nodes, "nodes": w.nodes, "steps": steps}
    for prec in ("f32", "f16"):
        stream = torch.cuda.Stream()
        sim = lbcg.Sim.from_workload(w, precision=prec, stream=stream.cuda_stream)
        sim.step(1)
        shape = sim.tune() if tune else sim.launch_info()
        ms = time_sim(torch, sim, stream, steps, warmup)
        sim.close()
        elem = 4 if prec == "f32" else 2
        out[prec] = {"mlups": round(w.fluid_nodes * steps / (ms / 1e3) / 1e6, 1),
                     "lattice_mlups": round(w.nodes * steps / (ms / 1e3) / 1e6, 1),
                     "ms_per_step": round(ms / steps, 4),
                     "frac": round((2 * 38 * elem + 4) * w.fluid_nodes * steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "rows": shape["rows"], "zchunks": shape["zchunks"]}
        if prec == "f32" and shape["rows"] == 0:
            out[prec]["traffic"] = read_traffic("geo_split")
    # the compact state on the split step: 2 x 96 (FP32) or 2 x 50 (FP16)
    # bytes per fluid node, plus the link word
    for prec, nbytes in (("f32", 2 * 96 + 4), ("f16", 2 * 50 + 4)):
        stream = torch.cuda.Stream()
        sim = lbcg.Sim.from_workload(w, precision=prec, kernel=lbcg.KERNEL_COMPACT, stream=stream.cuda_stream)
        sim.step(1)
        ms = time_sim(torch, sim, stream, steps, warmup)
        sim.close()
        out[prec + "_compact"] = {"mlups": round(w.fluid_nodes * steps / (ms / 1e3) / 1e6, 1),
                                  "lattice_mlups": round(w.nodes * steps / (ms / 1e3) / 1e6, 1),
                                  "ms_per_step": round(ms / steps, 4),
                                  "frac": round(nbytes * w.fluid_nodes * steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "bytes_per_fluid_node": nbytes}
        if prec == "f32":
            out[prec + "_compact"]["traffic"] = read_traffic("geo_split_compact")
    return out


def batched_form(torch, lbcg, W, steps=200, warmup=10, compact=False, precision="f32"):
    ws = W.batch_boxes(n_boxes=64, seed=4)
    nodes = sum(w.fluid_nodes for w in ws)
    stream = torch.cuda.Stream()
    kernel = lbcg.KERNEL_COMPACT if compact else lbcg.KERNEL_FUSED
    sims = [lbcg.Sim.from_workload(w, precision=precision, kernel=kernel, stream=stream.cuda_stream) for w in ws]
    for s in sims:
        s.step(2)
    b = lbcg.Batch(sims)
    info = b.launch_info()
    b.step(warmup)
    stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    e1.synchronize()
    ms_b = e0.elapsed_time(e1)
    b.close()
    # the same boxes stepped one after another, each in its own tuned shape
    for s in sims:
        s.tune()
        s.step(warmup)
    stream.synchronize()
    e0.record(stream)
    for s in sims:
        s.step(steps)
    e1.record(stream)
    e1.synchronize()
    ms_p = e0.elapsed_time(e1)
    for s in sims:
        s.close()
    mb = nodes * steps / (ms_b / 1e3) / 1e6
    mp = nodes * steps / (ms_p / 1e3) / 1e6
    if compact:
        bpn = 2 * (19 * 4 + 20) if precision == "f32" else 2 * (19 * 2 + 12)
    else:
        bpn = 2 * 19 * 2 * (4 if precision == "f32" else 2)
    return {"workload": "64 periodic D3Q19 boxes, edges U{32..96}, seed 4", "nodes": nodes,
            "state": "compact" if compact else "pairs", "storage": precision, "bytes_per_node": bpn,
            "steps": steps, "batched_mlups": round(mb, 1), "plain_mlups": round(mp, 1),
            "speedup": round(mb / mp, 3), "frac": round(mb * bpn / 1e3 / HBM_PEAK_GBS, 4),
            "rows": info["rows"], "zplanes": info["zplanes"], "blocks": info["blocks"]}


def served_form(torch, lbcg, W, n=64, steps_scale=0.1, loads=(0.8, 1.5), capacity=0.0):
    """A Poisson stream of n step-emulsifier requests (channel and reservoir
    sizes, inlet speeds and seed of the full 256-request stream) with step
    counts U{5000..20000} scaled by steps_scale, through the continuous-batching server and
    through the same server one request at a time.  The one-at-a-time capacity
    (requests per second with every request queued at t = 0) sets the arrival
    rate of each offered load; p50 / p99 time to result and fluid-node MLUPS
    per load and mode.  capacity > 0: use that one-at-a-time capacity (from an
    earlier run) instead of measuring it."""
    from paper_1711_02003_amd import serve
    lo, hi = int(5000 * steps_scale), int(20000 * steps_scale)
    last = [time.perf_counter()]

    def progress(done, total):
        # a line a minute at most, and the last one
        if done == total or time.perf_counter() - last[0] > 60:
            last[0] = time.perf_counter()
            log(f"served: {done} of {total} requests done")

    def reqs(rate, at_zero=False):
        specs = W.served_requests(n=n, seed=5, rate=rate, steps_lo=lo, steps_hi=hi)
        if at_zero:
            specs = [dict(r, arrival=0.0) for r in specs]
        return serve.requests_from_stream(specs, W.step_emulsifier)

    fps = []
    for r in reqs(1.0):
        w = r.make()
        p, _k = lbcg.make_params(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.A, w.beta, "f32",
                                 mask=w.mask, inlets=w.inlets, outlets=w.outlets)
        fps.append(lbcg.footprint(p))
    cap = int(sum(sorted(fps)[-8:]) * 1.05)  # room for about eight requests at once
    one = serve.LbcgBackend(cap, precision="f32", fields=False, tune_min=1)
    measured = capacity <= 0
    if measured:
        st0 = serve.Server(one, cap, slice_steps=256, max_running=1, keep_results=False,
                           progress=progress).run(reqs(1.0, True))
        capacity = st0.completed / st0.makespan_s
        log(f"served: one-at-a-time capacity {capacity:.2f} requests/s ({st0.as_dict()})")
    out = {"workload": f"{n} step-emulsifier requests (Poisson), steps U{{{lo}..{hi}}}, seed 5",
           "stand_in": "the full stream (256 requests, steps U{5000..20000})" if (n, lo, hi) == (256, 5000, 20000)
                       else f"the 256-request stream at reduced scale: {n} of its requests, step counts x "
                            f"{steps_scale} (U{{{lo}..{hi}}} instead of U{{5000..20000}}); same channel and "
                            "reservoir sizes, inlet speeds and arrival process",
           "plain_capacity_per_s": round(capacity, 3), "capacity_measured": measured, "arena_bytes": cap,
           "loads": {}}
    served_be = serve.LbcgBackend(cap, precision="f32", fields=False)
    for load in loads:
        rate = load * capacity
        plain = serve.Server(one, cap, slice_steps=256, max_running=1, keep_results=False,
                             progress=progress).run(reqs(rate))
        served = serve.Server(served_be, cap, slice_steps=256, keep_results=False, progress=progress).run(reqs(rate))
        row = {"arrival_rate_per_s": round(rate, 3), "served": served.as_dict(), "plain": plain.as_dict(),
               "mlups_ratio": round(served.mlups / plain.mlups, 3) if plain.mlups else None}
        out["loads"][str(load)] = row
        log(f"served load {load}: {row}")
    out["tile"] = list(served_be.tile) if served_be.tile else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--precision", default="f32", choices=["f32", "f16"])
    ap.add_argument("--kernel", default="compact", choices=["compact", "fused"],
                    help="compact state or the pair-state sweep")
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--zchunks", type=int, default=0)
    ap.add_argument("--tile-width", type=int, default=0, help="compact sweep: 64 or 32 (0: tuned)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the f16 / batched / served forms")
    ap.add_argument("--forms", default=",".join(FORMS),
                    help="comma-separated forms to run (default: all of " + ", ".join(FORMS) + ")")
    ap.add_argument("--no-form-tune", action="store_true",
                    help="focusing form: keep the automatic launch shape (for counter runs, where the "
                         "counted kernels run slower than the others the tuner compares them with)")
    ap.add_argument("--served-requests", type=int, default=64)
    ap.add_argument("--served-steps-scale", type=float, default=0.1)
    ap.add_argument("--served-loads", default="0.8,1.5",
                    help="offered loads, as fractions of the one-at-a-time capacity (comma-separated; empty: none)")
    ap.add_argument("--served-capacity", type=float, default=0.0,
                    help="one-at-a-time capacity in requests/s from an earlier run (0: measure it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU slab decomposition is design only)"}))
        sys.exit(2)

    import torch

    from paper_1711_02003_amd import lbcg
    from paper_1711_02003_amd import workloads as W

    w = W.droplets_27(L=args.size, seed=2)
    compact = args.kernel == "compact"
    kname = "k_step_compact" if compact else "k_step_fused"
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = lbcg.Sim.from_workload(w, precision=args.precision,
                                     kernel=lbcg.KERNEL_COMPACT if compact else lbcg.KERNEL_FUSED,
                                     tile=(args.rows, args.zchunks, args.tile_width))
    if not (args.rows or args.zchunks or args.tile_width):
        sim.step(1)
        sim.tune()  # launch shape chosen by timing candidates on this lattice
    info = sim.launch_info()
    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    diag = sim.diagnostics()
    sim.close()
    if diag["status"] != 0:
        print(json.dumps({"error": "non-finite state after the timed steps"}))
        sys.exit(1)

    N = w.fluid_nodes
    elem = 4 if args.precision == "f32" else 2
    bytes_node = (2 * (19 * 4 + 20) if elem == 4 else 2 * (19 * 2 + 12)) if compact else 2 * 2 * 19 * elem
    mlups = N * args.steps / (ms / 1e3) / 1e6
    achieved = bytes_node * N / (ms_step / 1e3) / 1e9
    traffic = read_traffic(kname) if args.precision == "f32" and args.size == 256 else None
    out = {
        "metric": "two-component MLUPS, D3Q19 regularized colour-gradient step",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": "D3Q19", "dims": list(w.dims),
                   "droplets": 27, "tau_R": w.tau_R, "tau_B": w.tau_B, "A": w.A, "beta": w.beta,
                   "storage": args.precision, "kernel": "fused compact" if compact else "fused",
                   "rows": info["rows"], "zchunks": info["zchunks"], "tile_width": info["tile_width"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_node": bytes_node},
        "wall_s": round(wall, 3),
    }
    log(f"headline {out['value']} MLUPS, {out['ms_per_step']} ms/step, shape {info}")
    if not args.no_copy_probe:
        out["copy_probe"] = copy_probe(torch)
    if not args.no_forms:
        run = {
            "pair_f32": lambda: pair_f32_form(torch, lbcg, W, args.size),
            "f16": lambda: f16_form(torch, lbcg, W, args.size),
            "d2q9": lambda: d2q9_form(torch, lbcg, W),
            "focusing2d": lambda: focusing2d_form(torch, lbcg, W),
            "focusing": lambda: focusing_form(torch, lbcg, W, tune=not args.no_form_tune),
            "batched": lambda: batched_form(torch, lbcg, W),
            "batched_compact": lambda: batched_form(torch, lbcg, W, compact=True),
            "batched_compact_f16": lambda: batched_form(torch, lbcg, W, compact=True, precision="f16"),
            "served": lambda: served_form(torch, lbcg, W, n=args.served_requests,
                                          steps_scale=args.served_steps_scale,
                                          loads=tuple(float(v) for v in args.served_loads.split(",") if v),
                                          capacity=args.served_capacity),
        }
        forms = {}
        for name in FORMS:
            if name in args.forms.split(","):
                forms[name] = run[name]()
                log(f"{name} {forms[name]}")
        out["forms"] = forms
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
