"""Served form on the GPU: a request's result in a mix of concurrently served
requests is bitwise its result computed alone."""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_02003_amd import lbcg
    lbcg.load_library()
    return lbcg


def test_served_alone_vs_mix(L):
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
    joins = [e for _, e, _ in srv.log]
    assert joins.index("done") < len(joins) - 1  # some request finished while others ran
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
