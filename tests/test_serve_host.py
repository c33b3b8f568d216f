"""Host logic of the served form: arena allocator, admission by footprint,
continuous batching, the one-slice-ahead pipeline and the latency statistics
(no device; a fake backend with a simulated clock and a simulated device
timeline)."""
import numpy as np
import pytest

from paper_1711_02003_amd.serve import ALIGN, Arena, Request, Server, Stats


class FakeWorkload:
    def __init__(self, nodes):
        self.fluid_nodes = nodes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Device work costs 1 s per 1e6 node updates and runs on a simulated
    device timeline: a queued slice starts when the device is free and the
    host goes on at once; waiting for a slice's event moves the host clock to
    its end.  Set-up and readback cost `host_cost` seconds of host time each.
    Records every call."""

    def __init__(self, clock, capacity, bytes_per_node=10, host_cost=0.0):
        self.clock, self.capacity, self.bpn = clock, capacity, bytes_per_node
        self.host_cost = host_cost
        self.live = {}
        self.calls = []
        self.groups = []
        self.peak = 0
        self.server = None
        self.device_free = 0.0
        self.busy = 0.0  # total device time

    def footprint(self, w):
        return w.fluid_nodes * self.bpn

    def create(self, w, off, nbytes):
        self.clock.t += self.host_cost
        h = {"w": w, "off": off, "bytes": nbytes, "steps": 0}
        for o in self.live.values():  # slots never overlap
            assert off + nbytes <= o["off"] or o["off"] + o["bytes"] <= off
        assert off + nbytes <= self.capacity
        self.live[id(h)] = h
        self.peak = max(self.peak, sum(o["bytes"] for o in self.live.values()))
        return h

    def regroup(self, handles):
        self.groups.append(len(handles))

    def step(self, handles, n):
        self.calls.append(list(n))
        for h, k in zip(handles, n):
            h["steps"] += k
            assert id(h) in self.live  # never a released request
        cost = sum(h["w"].fluid_nodes * k for h, k in zip(handles, n)) / 1e6
        start = max(self.device_free, self.clock.t)
        self.device_free = start + cost
        self.busy += cost

    def record(self):
        return self.device_free

    def wait(self, event):
        self.clock.t = max(self.clock.t, event)

    def result(self, h):
        self.clock.t += self.host_cost
        return {"steps": h["steps"]}

    def release(self, h):
        del self.live[id(h)]


def _server(capacity=10_000_000, slice_steps=100):
    clk = FakeClock()
    be = FakeBackend(clk, capacity)
    return Server(be, capacity, slice_steps=slice_steps, clock=clk, sleep=clk.sleep), be, clk


def _req(i, t, steps, nodes):
    return Request(id=i, arrival=t, steps=steps, make=lambda n=nodes: FakeWorkload(n))


def test_arena_first_fit_and_merge():
    a = Arena(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(3 * ALIGN)
    z = a.alloc(ALIGN + 1)
    assert (x, y, z) == (0, ALIGN, 4 * ALIGN)
    assert a.alloc(5 * ALIGN) is None
    a.free(y)
    assert a.alloc(2 * ALIGN) == ALIGN  # first fit reuses the hole
    a.free(x)
    a.free(ALIGN)
    a.free(z)
    assert a.free_list == [(0, 10 * ALIGN)] and a.bytes_used == 0


def test_arena_random_no_overlap():
    rng = np.random.default_rng(0)
    a = Arena(1 << 20)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            a.free(off)
            del live[off]
        else:
            n = int(rng.integers(1, 50_000))
            off = a.alloc(n)
            if off is not None:
                assert off % ALIGN == 0 and off + n <= a.capacity
                for o, m in live.items():
                    assert off + n <= o or o + m <= off
                live[off] = n
        assert a.bytes_used + sum(s for _, s in a.free_list) == a.capacity


def test_every_request_completes_with_its_steps():
    srv, be, clk = _server()
    reqs = [_req(i, 0.5 * i, steps=150 + 37 * i, nodes=100_000 + 50_000 * (i % 3)) for i in range(12)]
    st = srv.run(reqs)
    assert st.completed == 12
    for r in reqs:
        assert r.result["steps"] == r.steps and r.done_steps == r.steps
        assert r.t_done >= r.arrival and r.t_admit >= r.arrival
    assert be.peak <= 10_000_000
    assert all(k <= 100 for call in be.calls for k in call)
    assert not be.live


def test_admission_by_footprint_holds_fifo_order():
    # capacity fits two small or one big request; the big one arrives second
    # and must be admitted before the small ones that arrive after it
    srv, be, clk = _server(capacity=2_000_000 + 4 * ALIGN, slice_steps=50)
    reqs = [_req(0, 0.0, 400, 100_000), _req(1, 0.01, 100, 200_000), _req(2, 0.02, 100, 50_000),
            _req(3, 0.03, 100, 50_000)]
    srv.run(reqs)
    admit = {rid: t for t, ev, rid in srv.log if ev == "admit"}
    assert admit[1] <= admit[2] <= admit[3]
    assert admit[1] >= reqs[0].t_done  # big one waited for room, not overtaken
    assert be.peak <= srv.arena.capacity


def test_continuous_batching_joins_midflight():
    srv, be, clk = _server(slice_steps=64)
    reqs = [_req(0, 0.0, 1000, 200_000), _req(1, 1.0, 200, 200_000), _req(2, 2.0, 200, 200_000)]
    srv.run(reqs)
    ev = [(e, rid) for _, e, rid in srv.log]
    # 1 and 2 join while 0 is still running and finish before it
    assert ev.index(("admit", 1)) < ev.index(("done", 0))
    assert ev.index(("done", 1)) < ev.index(("done", 0))
    assert max(be.groups) == 3 or max(be.groups) == 2


def test_stats_percentiles():
    st = Stats(completed=5, makespan_s=2.0, node_updates=4e6, ttr=[1.0, 2.0, 3.0, 4.0, 100.0])
    assert st.mlups == pytest.approx(2.0)
    assert st.percentile(50) == pytest.approx(3.0)
    assert st.percentile(99) == pytest.approx(np.percentile([1, 2, 3, 4, 100], 99))
    d = st.as_dict()
    assert d["completed"] == 5 and d["p50_s"] == 3.0


def test_request_larger_than_arena_is_an_error():
    srv, be, clk = _server(capacity=1000)
    with pytest.raises(ValueError):
        srv.run([_req(0, 0.0, 10, 1000)])


def test_max_running_serialises():
    clk = FakeClock()
    be = FakeBackend(clk, 10_000_000)
    srv = Server(be, 10_000_000, slice_steps=100, clock=clk, sleep=clk.sleep, max_running=1)
    reqs = [_req(i, 0.0, 200, 100_000) for i in range(4)]
    srv.run(reqs)
    assert max(be.groups) == 1
    done = sorted(r.t_done for r in reqs)
    assert done == [pytest.approx(20.0 * (i + 1)) for i in range(4)]


def test_pipeline_hides_setup_and_readback():
    # Arrivals every 10 s, each request 300 steps of 100k nodes (30 s of
    # device time alone; offered load 3), 2 s of host time per set-up and per
    # readback, slices of 50 steps (5 s of device time per request).  The
    # loop queues a slice before it waits for the previous one, so the host
    # work of one iteration (at most one set-up and one readback, 4 s) runs
    # while the device computes: the device never idles between the first
    # set-up and the last readback.
    clk = FakeClock()
    be = FakeBackend(clk, 100_000_000, host_cost=2.0)
    srv = Server(be, 100_000_000, slice_steps=50, clock=clk, sleep=clk.sleep)
    reqs = [_req(i, 10.0 * i, 300, 100_000) for i in range(8)]
    st = srv.run(reqs)
    assert st.completed == 8 and all(r.result["steps"] == 300 for r in reqs)
    assert be.busy == pytest.approx(240.0)
    assert st.makespan_s <= be.busy + 2.0 + 2.0 + 1e-9
    # a one-slice-at-a-time loop would add every set-up and readback
    assert st.makespan_s < be.busy + 8 * 4.0 - 20.0


def test_progress_reports_each_completion():
    clk = FakeClock()
    be = FakeBackend(clk, 10_000_000)
    seen = []
    srv = Server(be, 10_000_000, slice_steps=100, clock=clk, sleep=clk.sleep,
                 progress=lambda done, total: seen.append((done, total)))
    reqs = [_req(i, 0.3 * i, 150 + 50 * i, 100_000) for i in range(5)]
    st = srv.run(reqs)
    assert st.completed == 5
    assert seen == [(k, 5) for k in range(1, 6)]
