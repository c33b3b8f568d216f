"""Served form on the GPU: requests are served concurrently (several in the
device's mix at once, some admitted while others are part-way), and a
request's result in the mix is bitwise its result computed alone, which in
turn agrees with the FP64 oracle."""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_02003_amd import lbcg
    lbcg.load_library()
    return lbcg


def _overlap(srv):
    """Most requests on the device at once (replaying the server's admit/done
    log), and whether some request was admitted while another one had done
    part of its steps and was not finished."""
    running, most = set(), 0
    for _t, ev, rid in srv.log:
        if ev == "admit":
            running.add(rid)
            most = max(most, len(running))
        elif ev == "done":
            running.discard(rid)
    joined_mid = any(0 < done < total for others in srv.joined_with.values() for done, total in others.values())
    return most, joined_mid


def test_served_alone_vs_mix(L, orc):
    from paper_1711_02003_amd import serve
    specs = W.served_requests(n=6, seed=21, rate=40.0, steps_lo=150, steps_hi=400, scale=0.25)
    reqs = serve.requests_from_stream(specs, W.step_emulsifier)
    fps = []
    for r in reqs:
        w = r.make()
        p, _k = L.make_params(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.A, w.beta, "f32", mask=w.mask,
                              inlets=w.inlets, outlets=w.outlets)
        fps.append(L.footprint(p))
    cap = sum(sorted(fps)[-3:]) + 4 * serve.ALIGN  # about three requests at a time
    be = serve.LbcgBackend(cap, precision="f32", tile=(8, 16))
    srv = serve.Server(be, cap, slice_steps=64)
    st = srv.run(reqs)
    print(f"served {st.as_dict()}", flush=True)
    assert st.completed == len(reqs)
    most, joined_mid = _overlap(srv)
    print(f"  at most {most} requests at once; admitted part-way through another: {joined_mid}", flush=True)
    assert most >= 2 and joined_mid
    for r in reqs:
        w = r.make()
        alone = L.Sim.from_workload(w, precision="f32")
        alone.step(r.steps)
        f = alone.fields()
        g = r.result["fields"]
        for k in ("rhoR", "rhoB", "u", "psi"):
            assert np.array_equal(g[k], f[k]), (r.id, k)
        assert r.result["diag"]["step"] == r.steps
        alone.close()
    # the first and the largest request against the FP64 oracle
    for r in {reqs[0].id: reqs[0], max(reqs, key=lambda q: q.nodes).id: max(reqs, key=lambda q: q.nodes)}.values():
        w = r.make()
        o = oracle_for(orc, w, threads=8).step(r.steps).fields()
        g = r.result["fields"]
        fl = w.mask == 0
        ep = rel_l2(g["psi"][fl], o["psi"][fl])
        eu = rel_l2(g["u"][:, fl], o["u"][:, fl], floor=1e-4 * np.sqrt(fl.sum()))
        print(f"  request {r.id} {w.dims} x{r.steps} vs oracle: relL2 psi {ep:.2e} u {eu:.2e}", flush=True)
        assert ep < 1e-5 and eu < 1e-5
