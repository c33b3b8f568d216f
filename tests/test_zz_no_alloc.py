"""lbcg_batch_step_noalloc (the batched step for callers that cannot
allocate) against lbcg_batch_step, through the C ABI: bitwise the same
populations for every lattice, on two calls in a row (the second with fewer
and smaller lattices), on the pair-state sweep (periodic and geometry
lattices, FP32 and FP16) and on the compact sweep (FP32 and FP16); calls
beyond the fixed area's limits are refused before anything is queued."""
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


def _say(msg):
    print(msg, flush=True)


def _focusing():
    return W.flow_focusing(nx=128, ny=48, nz=14, lam=3.0, u_disp=0.02, u_side=0.03, A=0.01)


def _pair(L, ws, prec, kernel, stream):
    a = [L.Sim.from_workload(w, precision=prec, kernel=kernel, stream=stream.cuda_stream) for w in ws]
    b = [L.Sim.from_workload(w, precision=prec, kernel=kernel, stream=stream.cuda_stream) for w in ws]
    return a, b


def _same(L, a, b, ws):
    for sa, sb, w in zip(a, b, ws):
        fl = np.ones(w.shape, bool) if w.mask is None else w.mask == 0
        assert np.array_equal(sa.populations()[..., fl], sb.populations()[..., fl]), w.name
        assert sa.diagnostics()["step"] == sb.diagnostics()["step"]


@pytest.mark.parametrize("prec,kernel", [("f32", "fused"), ("f16", "fused"), ("f32", "compact"), ("f16", "compact")])
def test_noalloc_matches_batch_two_calls(L, prec, kernel):
    import torch
    stream = torch.cuda.Stream()
    kind = L.KERNEL_COMPACT if kernel == "compact" else L.KERNEL_FUSED
    tile = (8, 16)
    big = W.batch_boxes(n_boxes=5, seed=41, edge_lo=20, edge_hi=60)
    if kernel == "fused":
        big.append(_focusing())
    small = W.batch_boxes(n_boxes=3, seed=42, edge_lo=12, edge_hi=30)
    # first call: fresh handles (their first steps run alone), uneven steps
    a, b = _pair(L, big, prec, kind, stream)
    n1 = [70, 3, 0, 41, 1, 66][: len(big)]
    bat = L.Batch(a, tile=tile)
    bat.step(n1)
    bat.close()
    L.batch_step_noalloc(b, n1, tile)
    _say(f"{prec} {kernel}: first call, {len(big)} lattices, steps {n1}")
    _same(L, a, b, big)
    # second call, smaller: three small boxes, on the same area
    c, d = _pair(L, small, prec, kind, stream)
    for s in c + d:
        s.step(2)
    n2 = [5, 33, 17]
    bat = L.Batch(c, tile=tile)
    bat.step(n2)
    bat.close()
    L.batch_step_noalloc(d, n2, tile)
    _say(f"{prec} {kernel}: second call, {len(small)} lattices, steps {n2}")
    _same(L, c, d, small)
    # and the first set again, continuing where it stopped
    n3 = [9, 9, 30, 0, 2, 1][: len(big)]
    bat = L.Batch(a, tile=tile)
    bat.step(n3)
    bat.close()
    L.batch_step_noalloc(b, n3, tile)
    _same(L, a, b, big)


def test_noalloc_refuses_beyond_its_area(L):
    import torch
    stream = torch.cuda.Stream()
    tiny = W.batch_boxes(n_boxes=1, seed=43, edge_lo=8, edge_hi=8)[0]
    # more lattices than the area holds
    sims = [L.Sim.from_workload(tiny, precision="f32", kernel=L.KERNEL_FUSED, stream=stream.cuda_stream)
            for _ in range(L.NOALLOC_MAX_LATTICES + 1)]
    p0 = sims[0].populations()
    with pytest.raises(L.LbcgError) as e:
        L.batch_step_noalloc(sims, 1, (8, 4))
    assert e.value.status == L.E_INVAL
    assert np.array_equal(sims[0].populations(), p0) and sims[0].diagnostics()["step"] == 0
    for s in sims:
        s.close()
    # more blocks per level than the area holds: 128^3 with 4-row tiles and
    # one plane per chunk is 2 x 32 x 128 = 8192 blocks per lattice
    w = W.static_droplet_3d(n=128, R=20.0)
    sims = [L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED, stream=stream.cuda_stream)
            for _ in range(9)]
    with pytest.raises(L.LbcgError) as e:
        L.batch_step_noalloc(sims, 1, (4, 1))
    assert e.value.status == L.E_INVAL
    assert sims[0].diagnostics()["step"] == 0
    L.batch_step_noalloc(sims[:8], 1, (4, 1))  # exactly the limit
    assert all(s.diagnostics()["step"] == 1 for s in sims[:8])
    # invalid shapes and mixed kernels
    with pytest.raises(L.LbcgError):
        L.batch_step_noalloc(sims[:2], 1, (6, 4))
    comp = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, stream=stream.cuda_stream)
    with pytest.raises(L.LbcgError):
        L.batch_step_noalloc([comp], 1, (4, 8))
    with pytest.raises(L.LbcgError):
        L.batch_step_noalloc([sims[0], comp], 1, (8, 8))
    # plain BGK and the compact state with geometry stay off the batched
    # sweeps: refused, nothing stepped
    bgk = L.Sim.from_workload(tiny, precision="f32", collision=L.BGK, stream=stream.cuda_stream)
    assert bgk.launch_info()["kernel"] == L.KERNEL_FUSED
    geo = _focusing()
    cgeo = L.Sim.from_workload(geo, precision="f32", kernel=L.KERNEL_COMPACT, stream=stream.cuda_stream)
    for group in ([bgk], [sims[0], bgk], [cgeo]):
        with pytest.raises(L.LbcgError) as e:
            L.batch_step_noalloc(group, 1, (8, 8))
        assert e.value.status == L.E_INVAL
    assert bgk.diagnostics()["step"] == 0 and cgeo.diagnostics()["step"] == 0
    assert sims[0].diagnostics()["step"] == 1
    for s in sims + [comp, bgk, cgeo]:
        s.close()
