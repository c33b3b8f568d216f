"""The split D3Q19 step for lattices with geometry (launch shape rows 0).

Three kernels (moments and psi of every fluid node; gradient, collision,
store and wall bounce-back; inlet and outlet values) over device-built
lists of the 64 x 4 blocks that hold fluid.  Every value is formed by the
column sweep's expressions in the sweep's order, so the split step must give
bitwise the sweep's state and the generic kernel's, on any geometry: ragged
sizes that leave partial blocks, blocks whose only fluid is one node,
periodic wrap through open faces, inlets, outlets, neutral and wetting walls
and nodes whose non-fluid neighbours mix those codes; and the FP64 oracle's
within the FP32 bar.
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


def _sparse_geometry(dims, seed, fluid=0.4, io=True):
    """Random D3Q19 lattice, at most half fluid: boxes of wall (neutral and
    two wetting codes) scattered over an open lattice until the fluid share
    falls below `fluid`; with io, an inlet face patch at x = 0 and an outlet
    patch at x = nx - 1 (pockets they feed may have no way out: fine for
    bitwise comparisons over a few steps, not for long runs); the other
    faces stay open (periodic)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    m = np.zeros(sh, np.uint8)
    while (m == 0).mean() > fluid:
        code = rng.choice([1, 64, 65])
        z0, y0, x0 = (rng.integers(0, n) for n in sh)
        dz, dy, dx = (rng.integers(1, max(2, n // 3)) for n in sh)
        m[z0:z0 + dz, y0:y0 + dy, x0:x0 + dx] = code
    if io:
        m[:, : ny // 2, 0] = np.where(m[:, : ny // 2, 0] == 0, 2, m[:, : ny // 2, 0])
        m[:, ny // 3:, nx - 1] = np.where(m[:, ny // 3:, nx - 1] == 0, 128, m[:, ny // 3:, nx - 1])
    psi = np.tanh(np.sin(np.arange(nx)[None, None, :] / 3.0) * 3 + rng.normal(0, 0.3, sh))
    rR, rB = W.colour_densities(psi)
    u = rng.uniform(-0.02, 0.02, (3,) + sh)
    w = W.Workload("sparse", "D3Q19", dims, rR, rB, u, 1.2, 0.7, 0.01, 0.7, mask=m)
    w.inlets = [{"u": (0.01, 0.0, 0.002), "rho_R": 0.9, "rho_B": 0.1}]
    w.outlets = [{"rho": 1.01}]
    w.walls = [{"psi": 0.5}, {"psi": -0.3}]
    return w


@pytest.mark.parametrize("dims", [(70, 13, 9), (64, 4, 3), (5, 7, 6), (130, 9, 5)])
@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_split_matches_sweep_and_generic_bitwise(L, dims, prec):
    w = _sparse_geometry(dims, seed=sum(dims))
    fl = w.mask == 0
    _say(f"split {dims} {prec}: {fl.mean():.2f} fluid")
    a = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_FUSED)
    assert a.launch_info()["rows"] == 0
    b = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_FUSED, tile=(8, 2, 0))
    c = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_GENERIC)
    for s in (a, b, c):
        s.step(45)
    pa = a.populations()[..., fl]
    assert np.array_equal(pa, b.populations()[..., fl])
    assert np.array_equal(pa, c.populations()[..., fl])
    assert a.diagnostics()["step"] == 45


def test_split_matches_oracle(L, orc):
    # walls of three codes, periodic elsewhere (inlets and outlets are
    # compared with the oracle on the junction, whose automatic shape is the
    # split step: test_gpu_forms.py)
    w = _sparse_geometry((70, 13, 9), seed=3, io=False)
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    assert s.launch_info()["rows"] == 0
    s.step(200)
    o = oracle_for(orc, w, threads=8).step(200)
    g, f = s.fields(), o.fields()
    fl = w.mask == 0
    ep = rel_l2(g["psi"][fl], f["psi"][fl])
    eu = rel_l2(g["u"][:, fl], f["u"][:, fl])
    _say(f"split vs oracle 70x13x9 x200: relL2 psi {ep:.2e} u {eu:.2e}")
    assert ep < 1e-5 and eu < 1e-5


def test_split_single_fluid_node_and_no_fluid(L):
    # one fluid node in a lattice of walls: one active block, its links all
    # from walls; and a lattice with no fluid node at all, which still
    # advances the step counter
    m = np.ones((4, 6, 70), np.uint8)
    m[2, 3, 66] = 0
    sh = m.shape
    w = W.Workload("one", "D3Q19", (70, 6, 4), np.full(sh, 0.6), np.full(sh, 0.4), None, 1.0, 0.8, 0.01, 0.7,
                   mask=m)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    c = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_GENERIC)
    assert a.launch_info()["rows"] == 0
    a.step(30)
    c.step(30)
    fl = m == 0
    assert np.array_equal(a.populations()[..., fl], c.populations()[..., fl])
    d = a.diagnostics()
    assert d["step"] == 30 and d["status"] == 0
    w.mask = np.ones_like(m)
    e = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    assert e.launch_info()["rows"] == 0
    e.step(7)
    assert e.diagnostics()["step"] == 7
