"""Served form: a stream of independent lattice requests on one GPU.

Requests arrive over time (each: a lattice, its initial fields, a step
count).  The server keeps one device arena; a request is admitted when its
``lbcg_footprint`` fits in a free slot of the arena (first fit, in arrival
order: a request that does not fit holds back the ones behind it, so large
requests are not starved).  All admitted requests advance together through
the batched fused step in slices of at most ``slice_steps`` time levels
(continuous batching: membership changes only at slice boundaries, finished
requests leave and queued ones join there).  A finished request's result
(diagnostics and fields of its final state) is copied to the host before its
slot is freed.

The loop keeps one slice queued ahead of the one it waits for: it queues
slice k + 1, then waits for slice k, reads back the requests that slice k
finished and admits new ones (their set-up and initialisation, and the
readbacks, go to a second stream), all while slice k + 1 runs.  A request
that finishes in slice k is no longer a member of slice k + 1, and its arena
slot is freed only after slice k has completed.

Metrics: time to result (completion minus arrival) per request, its p50 and
p99, and the aggregate rate in fluid-node updates per second.

The scheduling logic is independent of the device: ``Server`` drives a
backend object (``LbcgBackend`` for the HIP library; tests substitute a
host-only fake with the same methods).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

ALIGN = 256


class Arena:
    """First-fit allocator of byte ranges [0, capacity), 256-byte aligned."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free_list = [(0, self.capacity)]  # sorted (offset, size)
        self.used = {}

    def alloc(self, nbytes: int) -> Optional[int]:
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, size) in enumerate(self.free_list):
            if size >= need:
                if size == need:
                    self.free_list.pop(k)
                else:
                    self.free_list[k] = (off + need, size - need)
                self.used[off] = need
                return off
        return None

    def free(self, off: int):
        size = self.used.pop(off)
        fl = self.free_list
        fl.append((off, size))
        fl.sort()
        merged = []
        for o, s in fl:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free_list = merged

    @property
    def bytes_used(self) -> int:
        return sum(self.used.values())


@dataclass
class Request:
    id: int
    arrival: float               # seconds after the server starts
    steps: int
    make: Callable[[], object]   # builds the workload (workloads.Workload)
    nodes: int = 0               # fluid nodes (set at admission)
    footprint: int = 0
    offset: Optional[int] = None
    handle: object = None
    done_steps: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[dict] = None

    @property
    def left(self) -> int:
        return self.steps - self.done_steps


@dataclass
class Stats:
    completed: int
    makespan_s: float
    node_updates: float
    ttr: List[float] = field(default_factory=list)

    @property
    def mlups(self) -> float:
        return self.node_updates / self.makespan_s / 1e6 if self.makespan_s > 0 else 0.0

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.asarray(self.ttr), q)) if self.ttr else 0.0

    def as_dict(self) -> dict:
        return {"completed": self.completed, "makespan_s": round(self.makespan_s, 3),
                "mlups": round(self.mlups, 1), "p50_s": round(self.percentile(50), 3),
                "p99_s": round(self.percentile(99), 3)}


class Server:
    """Continuous-batching scheduler over a backend (see module docstring)."""

    def __init__(self, backend, capacity_bytes: int, slice_steps: int = 256,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, keep_results: bool = True,
                 max_running: int = 0, progress: Optional[Callable[[int, int], None]] = None):
        self.backend = backend
        self.max_running = int(max_running)  # 0 = no limit besides the arena
        self.arena = Arena(capacity_bytes)
        self.slice_steps = int(slice_steps)
        self.clock = clock
        self.sleep = sleep
        self.keep_results = keep_results
        self.progress = progress  # called as progress(completed, total) after each completion
        self.log: List[tuple] = []  # (time, event, request id)
        # per admitted request: the steps done so far by each request already
        # running when it joined (shows requests joining part-way through others)
        self.joined_with: dict = {}

    def _admit(self, r: Request, now: float, running=()) -> bool:
        w = r.make()
        fp = self.backend.footprint(w)
        if fp > self.arena.capacity:
            raise ValueError(f"request {r.id} needs {fp} bytes, more than the arena holds")
        off = self.arena.alloc(fp)
        if off is None:
            return False
        r.footprint, r.offset = fp, off
        r.handle = self.backend.create(w, off, fp)
        r.nodes = int(w.fluid_nodes)
        r.t_admit = now
        self.joined_with[r.id] = {o.id: (o.done_steps, o.steps) for o in running}
        self.log.append((now, "admit", r.id))
        return True

    def _finish(self, r: Request, t0: float, finished: List[Request]):
        res = self.backend.result(r.handle)
        r.result = res if self.keep_results else None
        self.backend.release(r.handle)
        self.arena.free(r.offset)
        r.handle = None
        r.t_done = self.clock() - t0
        self.log.append((r.t_done, "done", r.id))
        finished.append(r)
        if self.progress is not None:
            self.progress(len(finished), self.total)

    def run(self, requests: List[Request]) -> Stats:
        self.total = len(requests)
        queue = sorted(requests, key=lambda r: (r.arrival, r.id))
        running: List[Request] = []      # on the device with steps not yet queued
        finished: List[Request] = []
        inflight = None                  # (event of the queued slice, requests it finishes)
        t0 = self.clock()
        members = None
        updates = 0.0
        while queue or running or inflight:
            now = self.clock() - t0
            # admission in arrival order; stop at the first request that does not fit
            while queue and queue[0].arrival <= now:
                if self.max_running and len(running) >= self.max_running:
                    break
                if not self._admit(queue[0], now, running):
                    break
                running.append(queue.pop(0))
            queued = None
            if running:
                ids = tuple(r.id for r in running)
                if ids != members:
                    self.backend.regroup([r.handle for r in running])
                    members = ids
                n = [min(self.slice_steps, r.left) for r in running]
                self.backend.step([r.handle for r in running], n)
                ending = []
                for r, k in zip(running, n):
                    r.done_steps += k
                    updates += float(r.nodes) * k
                    if r.left == 0:
                        ending.append(r)
                running = [r for r in running if r.left > 0]
                queued = (self.backend.record(), ending)
            if inflight is not None:
                # the previous slice: wait for it (the one just queued runs
                # meanwhile) and read back the requests it finished
                self.backend.wait(inflight[0])
                for r in inflight[1]:
                    self._finish(r, t0, finished)
            inflight = queued
            if inflight is None and not running and queue:
                # idle device: sleep until the next arrival (an arrived
                # request fits the arena, now empty, at the next pass)
                now = self.clock() - t0
                if queue[0].arrival > now:
                    self.sleep(queue[0].arrival - now)
        self.backend.regroup([])
        makespan = self.clock() - t0
        ttr = [r.t_done - r.arrival for r in finished]
        return Stats(len(finished), makespan, updates, ttr)


class LbcgBackend:
    """The HIP library: one device arena (a torch uint8 tensor), handles
    created in arena slots, all running requests stepped together by the
    batched step that needs no batch object (lbcg_batch_step_noalloc), so
    that membership changes cost nothing.  Two streams: `stream` carries the
    slices; `side` carries each request's set-up, initialisation and result
    readback, which therefore never wait for a running slice (lbcg_set_stream
    moves a handle between them once the work before has completed)."""

    def __init__(self, capacity_bytes: int, precision: str = "f32", tile=None, fields: bool = True,
                 tune_min: int = 4, default_tile=(8, 32)):
        import torch

        from . import lbcg
        self.torch = torch
        self.lbcg = lbcg
        self.precision = precision
        self.stream = torch.cuda.Stream()
        self.side = torch.cuda.Stream()
        self.arena = torch.empty(int(capacity_bytes), dtype=torch.uint8, device="cuda")
        self.base = self.arena.data_ptr()
        # None: chosen by timing on the first group of at least tune_min
        # requests, then reused (default_tile until then)
        self.tile = tile
        self.tune_min = int(tune_min)
        self.default_tile = tuple(default_tile)
        self.fields = fields

    def footprint(self, w) -> int:
        p, _keep = self.lbcg.make_params(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.A, w.beta,
                                         self.precision, mask=w.mask, inlets=w.inlets,
                                         outlets=w.outlets)
        return self.lbcg.footprint(p)

    def create(self, w, offset: int, nbytes: int):
        # set up and initialised on the side stream (which init_fields
        # synchronizes), then handed to the slice stream
        s = self.lbcg.Sim.from_workload(w, precision=self.precision, stream=self.side.cuda_stream,
                                        dev_buf=(self.base + offset, nbytes))
        s.set_stream(self.stream.cuda_stream)
        return s

    def regroup(self, handles):
        if handles and self.tile is None and len(handles) >= self.tune_min:
            # one timing pass over candidate shapes on these states (they do
            # not change), once; the batch it needs is released again
            b = self.lbcg.Batch(handles)
            info = b.launch_info()
            b.close()
            self.tile = (info["rows"], info["zplanes"])

    def step(self, handles, nsteps):
        self.lbcg.batch_step_noalloc(handles, nsteps, self.tile or self.default_tile)

    def record(self):
        e = self.torch.cuda.Event()
        e.record(self.stream)
        return e

    def wait(self, event):
        event.synchronize()

    def result(self, s) -> dict:
        # the slice that finished the request has completed (waited for)
        s.set_stream(self.side.cuda_stream)
        d = s.diagnostics()
        out = {"diag": d}
        if self.fields:
            out["fields"] = s.fields()
        return out

    def release(self, s):
        s.close()


def requests_from_stream(specs, make_workload) -> List[Request]:
    """Requests from ``workloads.served_requests`` specs."""
    return [Request(id=r["id"], arrival=r["arrival"], steps=int(r["args"]["steps"]),
                    make=(lambda a=r["args"]: make_workload(**a))) for r in specs]
