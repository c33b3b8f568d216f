"""GPU checks of the D3Q19 compact-state sweep with FP16 storage.

The FP16 compact state stores each node's 19 total deviations over w_i in
FP16, its minority share M in FP32 (with the majority flag) and V_axis and
R_d in FP16; every FP16 value is rounded stochastically with the node's
generator (seeded by the time step and the node index); arithmetic is FP32.
The bars are those of the FP16 pair state: the equivalent radius and the
Laplace pressure jump of a relaxed droplet within 1 % of the FP64 oracle's,
the colour-mass drift a random walk far below a repeated rounding error's,
bitwise invariance under the launch shape and under reads of the state, and
one-step agreement with the oracle within FP16's rounding unit at the full
256^3 size.
"""
import json
import os

import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, rel_l2
from tests.test_gpu_compact import _droplets
from tests.test_gpu_parity import _maxrel, _sampled_one_step

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")
# FP16's unit of a stored value: 2^-10 of a total's deviation over w_i (10
# mantissa bits), 2^-9 of a share (9 bits, the lowest holds the flag); a
# stochastic rounding moves a value by less than one unit.
U16_SHARE = 2.0 ** -9


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_02003_amd import lbcg
    lbcg.load_library()
    return lbcg


@pytest.fixture(scope="module")
def stream():
    import torch
    return torch.cuda.Stream()


def _say(msg):
    print(msg, flush=True)


def _compact16(L, w, **kw):
    s = L.Sim.from_workload(w, precision="f16", kernel=L.KERNEL_COMPACT, **kw)
    assert s.launch_info()["kernel"] == L.KERNEL_COMPACT
    return s


def test_compact_f16_droplet_within_one_percent(L):
    # Static D3Q19 droplet 96^3, R = 20, 3000 steps: R_eff and the Laplace
    # jump within 1 % of the FP64 oracle's (stored by
    # tests/golden/make_oracle_values.py) and of the FP32 compact state's.
    gold = json.load(open(GOLDEN))["d3q19_droplet_96_R20"]
    w = W.static_droplet_3d(n=96, R=20.0, tau=(1.0, 1.0), A=0.005, steps=3000)
    assert gold["steps"] == w.steps
    out = {}
    for prec in ("f32", "f16"):
        _say(f"droplet 96^3 compact {prec} x{w.steps}")
        s = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_COMPACT)
        s.step(w.steps)
        d = s.diagnostics(check=True)
        out[prec] = (d["R_eff"], d["p_in"] - d["p_out"])
        s.close()
    (r32, dp32), (r16, dp16) = out["f32"], out["f16"]
    _say(f"  R_eff f32 {r32:.4f} f16 {r16:.4f} oracle {gold['R_eff']:.4f}; "
         f"dp f32 {dp32:.4e} f16 {dp16:.4e} oracle {gold['dp']:.4e}")
    assert dp16 > 0
    assert abs(r16 / gold["R_eff"] - 1) < 0.01 and abs(dp16 / gold["dp"] - 1) < 0.01
    assert abs(r16 / r32 - 1) < 0.01 and abs(dp16 / dp32 - 1) < 0.01


def test_compact_f16_droplets_27_vs_oracle_and_drift(L, orc):
    # The 27-droplet recipe at 48^3 after 1000 steps: phase field within 1 %
    # (rel-L2) of the FP64 oracle's, per-colour mass drift below 1e-4.
    w = W.droplets_27(L=48, seed=2)
    _say("compact f16 48^3 x1000")
    s = _compact16(L, w)
    d0 = s.diagnostics()
    s.step(1000)
    d1 = s.diagnostics(check=True)
    g = s.fields()
    s.close()
    dr = abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"]
    db = abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"]
    o = oracle_for(orc, w, threads=16).step(1000)
    f = o.fields()
    ep = rel_l2(g["psi"], f["psi"])
    eu = rel_l2(g["u"], f["u"], floor=1e-4 * np.sqrt(w.nodes))
    _say(f"  relL2 psi {ep:.3e} u (floored) {eu:.3e}; colour drift R {dr:.2e} B {db:.2e}")
    assert ep < 1e-2 and eu < 1e-1
    assert dr < 1e-4 and db < 1e-4


@pytest.mark.parametrize("dims", [(96, 40, 24), (33, 17, 12), (5, 3, 2)])
def test_compact_f16_tile_shape_invariance(L, dims):
    # Every launch shape gives bitwise the same state: the random bits of a
    # stored value depend on the time step and the node only.
    w = _droplets(dims, seed=5)
    ref = None
    for tile in ((8, 1, 0), (8, 3, 0), (8, 0, 0), (8, 1, 32), (8, 0, 32)):
        s = _compact16(L, w, tile=tile)
        s.step(17)
        p = s.populations()
        s.close()
        if ref is None:
            ref = p
        else:
            assert np.array_equal(p, ref), tile


def test_compact_f16_reads_and_resume(L):
    # Reads leave the trajectory bitwise unchanged; a checkpoint (a pair
    # state) resumes on the FP16 compact or pair-state kernel within a few
    # FP16 units of the uninterrupted run.
    w = W.droplets_27(L=40, seed=9)
    a = _compact16(L, w)
    b = _compact16(L, w)
    for _ in range(4):
        a.step(10)
        a.populations()
        a.diagnostics()
    b.step(40)
    pa = a.populations()
    assert np.array_equal(pa, b.populations())
    c = _compact16(L, w)
    c.step(15)
    blob = c.get_state()
    c.close()
    for kernel in (L.KERNEL_COMPACT, L.KERNEL_FUSED):
        d = L.Sim.from_workload(w, precision="f16", kernel=kernel)
        d.set_state(blob)
        d.step(25)
        e = _maxrel(d.populations(), pa)
        _say(f"resume on kernel {kernel}: max rel {e:.2e}")
        assert e < 8 * U16_SHARE
        assert d.diagnostics()["step"] == 40
        d.close()


def test_compact_f16_agrees_with_f16_pairs(L):
    # The FP16 compact and FP16 pair states round differently (the pair state
    # rounds each population's share, the compact one M and V): after 200
    # steps their phase fields agree within FP16's share unit.
    w = _droplets((70, 37, 20), seed=3)
    a = _compact16(L, w)
    b = L.Sim.from_workload(w, precision="f16", kernel=L.KERNEL_FUSED)
    a.step(200)
    b.step(200)
    fa, fb = a.fields(), b.fields()
    e = float(np.abs(fa["psi"] - fb["psi"]).max())
    _say(f"compact f16 vs pair f16 70x37x20 x200: max |dpsi| {e:.2e}")
    assert e < 4 * U16_SHARE


def test_compact_f16_full_size_sampled(L, orc):
    # Full 256^3 lattice in the tuned launch shape: sampled nodes' next state
    # against the oracle's step from the same (read-out) state.  The read-out
    # and the stored output are each within one FP16 unit, so the bound is
    # twice a share's unit.
    w = W.droplets_27(L=256, seed=2)
    _say("full size 256^3 compact f16")
    s = _compact16(L, w)
    s.step(1)
    _say(f"  tuned {s.tune()}")
    d0 = s.diagnostics(check=True)
    s.step(20)
    worst = _sampled_one_step(L, orc, w, s)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2 * U16_SHARE
    d1 = s.diagnostics(check=True)
    for k in ("mass_R", "mass_B"):
        assert abs(d1[k] - d0[k]) / d0[k] < 1e-4, k
    s.close()


@pytest.mark.parametrize("kernel", ["fused", "compact"])
def test_f16_largest_lattice_and_beyond(L, orc, kernel):
    # FP16 storage halves the bytes per population, so the sweeps take
    # larger lattices within their 32-bit byte offsets: 383^3 (4.27 GB per
    # FP16 pair buffer) is the largest cube, one step at 32 sampled nodes
    # against the oracle within two units of a stored share; 384^3 (4.30 GB)
    # is refused.
    k = {"fused": L.KERNEL_FUSED, "compact": L.KERNEL_COMPACT}[kernel]
    w = W.droplets_27(L=383, seed=2)
    _say(f"383^3 f16 {kernel}")
    s = L.Sim.from_workload(w, precision="f16", kernel=k)
    assert s.launch_info()["kernel"] == k
    s.step(3)
    worst = _sampled_one_step(L, orc, w, s, n_samples=32, seed=383)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2 * U16_SHARE
    s.close()
    del w
    with pytest.raises(L.LbcgError):
        L.Sim("D3Q19", (384, 384, 384), 1.0, 0.6, 0.005, 0.7, "f16", kernel=k)


def test_compact_f16_batched_matches_plain_bitwise(L, stream):
    # FP16 compact lattices batched (and through the allocation-free step):
    # each lattice bitwise as stepped alone (the stochastic rounding draws
    # from the node's own generator, so the launch does not matter); fresh
    # handles take their pair-state step alone first; mixing precisions or
    # geometry is refused
    ws = W.batch_boxes(n_boxes=3, seed=15, edge_lo=20, edge_hi=52)
    nsteps = [40, 7, 33]  # a run of >= 32 levels replays graphs
    sims = [_compact16(L, w, stream=stream.cuda_stream) for w in ws]
    b = L.Batch(sims)
    info = b.launch_info()
    _say(f"FP16 compact batch shape {info}")
    assert info["rows"] == 8
    b.step(nsteps)
    b.close()
    L.batch_step_noalloc(sims, [3, 0, 5], (8, 16))
    for w, s, n in zip(ws, sims, [43, 7, 38]):
        ref = _compact16(L, w)
        ref.step(n)
        assert np.array_equal(s.populations(), ref.populations()), w.name
        assert s.diagnostics()["step"] == n
        ref.close()
    f32 = L.Sim.from_workload(ws[0], precision="f32", kernel=L.KERNEL_COMPACT, stream=stream.cuda_stream)
    with pytest.raises(L.LbcgError):
        L.Batch([sims[0], f32])
    with pytest.raises(L.LbcgError):
        L.batch_step_noalloc([sims[0], f32], [1, 1], (8, 8))
    for s in sims + [f32]:
        s.close()
