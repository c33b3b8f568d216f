"""GPU: the fused D2Q9 strip sweep (periodic lattices, FP32 and FP16
storage) against the generic two-pass kernel (bitwise: both run the same
device arithmetic in the same order) and against the FP64 oracle."""
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


def _random_2d(dims, seed):
    rng = np.random.default_rng(seed)
    nx, ny, _ = dims
    sh = (1, ny, nx)
    u = np.zeros((3,) + sh)
    u[:2] = rng.uniform(-0.04, 0.04, (2,) + sh)
    return W.Workload("random2d", "D2Q9", dims, rng.uniform(0.05, 1, sh), rng.uniform(0.05, 1, sh), u,
                      1.3, 0.7, 0.01, 0.7)


@pytest.mark.parametrize("dims", [(64, 64, 1), (100, 37, 1), (130, 9, 1), (5, 3, 1)])
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_fused2d_matches_generic_bitwise(L, dims, prec):
    w = _random_2d(dims, seed=sum(dims))
    _say(f"fused2d vs generic {dims} {prec}")
    a = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_FUSED)
    b = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_GENERIC)
    assert a.launch_info()["kernel"] == L.KERNEL_FUSED
    a.step(50)
    b.step(50)
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


@pytest.mark.parametrize("ychunks", [1, 3, 16])
def test_fused2d_chunk_invariance(L, ychunks):
    w = W.droplets_2d(n=256, seed=6)
    ref = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_GENERIC)
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED, tile=(0, ychunks, 0))
    assert s.launch_info()["zchunks"] == ychunks
    ref.step(20)
    s.step(20)
    assert np.array_equal(s.populations(), ref.populations())


def test_fused2d_f32_matches_oracle_1000_steps(L, orc):
    # 256^2 with 256 droplets (tau_R = 1, tau_B = 0.6, A = 0.005): FP32 strip
    # sweep vs FP64 oracle after 1000 steps, in the tuned launch shape.
    w = W.droplets_2d(n=256, seed=6)
    _say("fused2d f32 256^2 x1000")
    s = L.Sim.from_workload(w, precision="f32")
    assert s.launch_info()["kernel"] == L.KERNEL_FUSED
    s.step(1)
    s.tune()
    o = oracle_for(orc, w, threads=8)
    o.step(1)
    d0 = s.diagnostics(check=True)
    s.step(999)
    o.step(999)
    g, f = s.fields(), o.fields()
    eu, ep = rel_l2(g["u"], f["u"]), rel_l2(g["psi"], f["psi"])
    _say(f"  relL2 u {eu:.3e} psi {ep:.3e} |u|rms {np.sqrt((f['u'] ** 2).mean()):.2e}")
    assert eu < 1e-5 and ep < 1e-5
    d1 = s.diagnostics(check=True)
    assert abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"] < 1e-6


def test_geometry_and_bgk_stay_on_the_generic_kernel(L):
    w = _random_2d((32, 16, 1), seed=1)
    m = np.zeros(w.shape, np.uint8)
    m[:, 0, :] = 1
    w.mask = m
    s = L.Sim.from_workload(w, precision="f32")
    assert s.launch_info()["kernel"] == L.KERNEL_GENERIC
    w.mask = None
    s = L.Sim.from_workload(w, precision="f32", collision=L.BGK)
    assert s.launch_info()["kernel"] == L.KERNEL_GENERIC
