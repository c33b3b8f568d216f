"""Plain BGK (Eq. (5)) on the fused D3Q19 column sweep.

Both BGK forms - at the node's rate from the mixture viscosity (LBCG_BGK)
and with each colour at its own rate (LBCG_BGK_COLOUR) - relax every
population from its own pulled value, so the sweep keeps the decoded
populations of the plane being collided beside its moments.  The sweep's
pulls, moments and collision are the generic kernel's expressions, so the
two must agree bitwise (FP32 and FP16 storage, periodic and with walls,
inlets and an outlet, two x tiles and ragged edges), the result must not
depend on the z chunking, and the FP32 result must stay within the FP32
bar of the FP64 oracle.
"""
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


def _say(msg):
    print(msg, flush=True)


def _workload(dims, masked, seed, tau=(1.3, 0.7)):
    # random colour densities and velocities (as the FP64 parity tests draw
    # them), with walls on two faces and around one inner node, an inlet and
    # an outlet face when masked
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    rR = rng.uniform(0.05, 1, sh)
    rB = rng.uniform(0.05, 1, sh)
    u = rng.uniform(-0.03, 0.03, (3,) + sh)
    w = W.Workload("random", "D3Q19", dims, rR, rB, u, tau[0], tau[1], 0.01, 0.7)
    if masked:
        m = np.zeros(sh, np.uint8)
        m[:, 0, :] = 1
        m[:, -1, :] = 1
        m[:, 1:-1, 0] = 2
        m[:, 1:-1, -1] = 128
        m[0] = 1
        m[nz // 2, ny // 2, nx // 2] = 1
        w.mask = m
        w.inlets = [{"u": (0.01, 0.002, 0.001), "rho_R": 0.8, "rho_B": 0.2}]
        w.outlets = [{"rho": 1.02}]
    return w


@pytest.mark.parametrize("coll", ["bgk", "bgk_colour"])
@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("masked", [False, True])
def test_bgk_fused_matches_generic_bitwise(L, coll, prec, masked):
    c = {"bgk": L.BGK, "bgk_colour": L.BGK_COLOUR}[coll]
    w = _workload((70, 13, 9), masked, seed=7 + masked)
    fl = np.ones(w.rhoR.shape, bool) if w.mask is None else w.mask == 0
    _say(f"BGK fused {coll} {prec} masked={masked}")
    a = L.Sim.from_workload(w, precision=prec, collision=c)
    info = a.launch_info()
    assert info["kernel"] == L.KERNEL_FUSED and info["rows"] == 8
    b = L.Sim.from_workload(w, precision=prec, collision=c, kernel=L.KERNEL_FUSED, tile=(8, 3, 0))
    g = L.Sim.from_workload(w, precision=prec, collision=c, kernel=L.KERNEL_GENERIC)
    for s in (a, b, g):
        s.step(30)
    pa = a.populations()[..., fl]
    assert np.isfinite(pa).all()
    assert np.array_equal(pa, b.populations()[..., fl])
    assert np.array_equal(pa, g.populations()[..., fl])
    assert a.diagnostics()["step"] == 30


@pytest.mark.parametrize("coll", ["bgk", "bgk_colour"])
def test_bgk_fused_f32_matches_oracle(L, orc, coll):
    c = {"bgk": (L.BGK, orc.BGK), "bgk_colour": (L.BGK_COLOUR, orc.BGK_COLOUR)}[coll]
    # the 27-droplet recipe (u ~ N(0, 1e-3), tau_R = 1, tau_B = 0.6) at 32^3
    w = W.droplets_27(L=32, seed=2)
    s = L.Sim.from_workload(w, precision="f32", collision=c[0])
    assert s.launch_info()["kernel"] == L.KERNEL_FUSED
    s.step(200)
    o = oracle_for(orc, w, threads=8, collision=c[1]).step(200)
    g, f = s.fields(), o.fields()
    ep = rel_l2(g["psi"], f["psi"])
    eu = rel_l2(g["u"], f["u"])
    _say(f"BGK fused {coll} f32 32^3 x200 vs oracle: relL2 psi {ep:.2e} u {eu:.2e} "
         f"(|u|_rms {np.sqrt((f['u'] ** 2).sum(0).mean()):.2e})")
    assert ep < 1e-5 and eu < 1e-5


def test_bgk_fused_limits(L):
    # 8-row tiles only; the batched sweeps, the split step and the compact
    # state stay regularized
    w = _workload((70, 13, 9), True, seed=3)
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(w, precision="f32", collision=L.BGK, kernel=L.KERNEL_FUSED, tile=(4, 0, 0))
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(_workload((16, 16, 16), False, seed=3), precision="f32", collision=L.BGK,
                            kernel=L.KERNEL_COMPACT)
    a = L.Sim.from_workload(w, precision="f32", collision=L.BGK)
    a.step(2)
    with pytest.raises(L.LbcgError):
        L.Batch([a])
    # a sparse lattice whose regularized form takes the split step
    m = np.ones((8, 16, 70), np.uint8)
    m[2:6, 4:12, :] = 0
    sh = m.shape
    ws = W.Workload("channel", "D3Q19", (70, 16, 8), np.full(sh, 0.6), np.full(sh, 0.4), None, 1.0, 0.8, 0.01,
                    0.7, mask=m)
    assert L.Sim.from_workload(ws, precision="f32").launch_info()["rows"] == 0
    b = L.Sim.from_workload(ws, precision="f32", collision=L.BGK)
    assert b.launch_info()["rows"] == 8
    shape = b.tune()
    assert shape["rows"] == 8
    b.step(3)
    assert b.diagnostics()["status"] == 0


@pytest.mark.parametrize("coll", ["bgk", "bgk_colour"])
def test_bgk_fused_largest_lattice_sampled(L, orc, coll):
    # Plain BGK on the fused sweep at the largest cube it takes (304^3 FP32,
    # byte offsets up to 2^32 - 25 MB), in the automatic launch shape: one
    # step at 32 sampled nodes against the oracle on 5^3 cuts
    from tests.test_gpu_parity import _sampled_one_step
    c = {"bgk": (L.BGK, orc.BGK), "bgk_colour": (L.BGK_COLOUR, orc.BGK_COLOUR)}[coll]
    w = W.droplets_27(L=304, seed=2)
    s = L.Sim.from_workload(w, precision="f32", collision=c[0])
    info = s.launch_info()
    _say(f"BGK {coll} 304^3 f32: launch {info}")
    assert info["kernel"] == L.KERNEL_FUSED and info["rows"] == 8
    s.step(3)
    worst = _sampled_one_step(L, orc, w, s, n_samples=32, seed=304, collision=c[1])
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    s.close()
