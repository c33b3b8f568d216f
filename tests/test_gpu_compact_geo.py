"""The compact state on lattices with geometry (D3Q19 FP32 and FP16, the
split step).

Every fluid node stores its 19 new totals and its colour record; a receiver
splits what it pulls with its sender's record, a link from a wall brings back
the node's own total of the opposite direction split with its own record, and
a link from an inlet or an outlet reads the pair the boundary kernel stored
(the pair-state step's value, formed from the node's own new populations).
In exact arithmetic this is the pair-state step, so its fields must stay
within the FP32 bar of the FP64 oracle and close to the pair-state split
step; reads of the state (populations, fields, diagnostics, checkpoints) go
through a conversion to pairs that also writes the walls' values.
"""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, rel_l2
from tests.test_gpu_split import _sparse_geometry

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


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
    # the benchmark's flow-focusing cross at 1/4 size, with faster inlets so
    # that 200 steps move the interface
    return W.flow_focusing(nx=128, ny=48, nz=14, lam=3.0, u_disp=0.02, u_side=0.03, A=0.01)


def test_compact_geometry_matches_oracle(L, orc):
    w = _focusing()
    fl = w.mask == 0
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    info = s.launch_info()
    assert info["kernel"] == L.KERNEL_COMPACT and info["rows"] == 0
    s.step(200)
    o = oracle_for(orc, w, threads=8).step(200)
    g, f = s.fields(), o.fields()
    ep = rel_l2(g["psi"][fl], f["psi"][fl])
    eu = rel_l2(g["u"][:, fl], f["u"][:, fl])
    _say(f"compact geometry vs oracle, focusing 128x48x14 x200: relL2 psi {ep:.2e} u {eu:.2e}")
    assert ep < 1e-5 and eu < 1e-5
    assert s.diagnostics()["step"] == 200


@pytest.mark.parametrize("dims", [(70, 13, 9), (5, 7, 6)])
def test_compact_geometry_walls_matches_oracle(L, orc, dims):
    # walls of three codes (neutral and two wetting), periodic elsewhere,
    # ragged sizes; colour masses kept
    w = _sparse_geometry(dims, seed=sum(dims), io=False)
    fl = w.mask == 0
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    d0 = s.diagnostics()
    s.step(200)
    o = oracle_for(orc, w, threads=8).step(200)
    g, f = s.fields(), o.fields()
    ep = rel_l2(g["psi"][fl], f["psi"][fl])
    eu = rel_l2(g["u"][:, fl], f["u"][:, fl])
    d1 = s.diagnostics()
    dm = max(abs(d1["mass_R"] / d0["mass_R"] - 1), abs(d1["mass_B"] / d0["mass_B"] - 1))
    _say(f"compact geometry, walls {dims} x200: relL2 psi {ep:.2e} u {eu:.2e}, colour mass {dm:.1e}")
    assert ep < 1e-5 and eu < 1e-5
    assert dm < 1e-6


def test_compact_geometry_close_to_pair_state(L):
    # inlets, outlets, walls of three codes and mixed links: the compact and
    # the pair-state split steps agree to FP32 rounding
    w = _sparse_geometry((70, 13, 9), seed=92)
    fl = w.mask == 0
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    assert b.launch_info()["rows"] == 0
    done = 0
    for n in (1, 2, 30):  # step 1 runs the two-pass kernel on both
        a.step(n - done)
        b.step(n - done)
        done = n
        pa, pb = a.populations()[..., fl], b.populations()[..., fl]
        d = float(np.abs(pa - pb).max() / np.abs(pb).max())
        _say(f"  step {n}: max rel difference of the populations {d:.2e}")
        assert d < (4 if n <= 2 else 60) * EPS32


def test_compact_geometry_checkpoint_and_limits(L):
    w = _focusing()
    fl = w.mask == 0
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    a.step(40)
    pa = a.populations()[..., fl]
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b.step(15)
    blob = b.get_state()
    for kernel in (L.KERNEL_COMPACT, L.KERNEL_FUSED):
        c = L.Sim.from_workload(w, precision="f32", kernel=kernel)
        c.set_state(blob)
        c.step(25)
        d = float(np.abs(c.populations()[..., fl] - pa).max() / np.abs(pa).max())
        _say(f"resume on kernel {kernel}: {d:.2e}")
        assert d < 25 * 4 * EPS32
        assert c.diagnostics()["step"] == 40
        c.close()
    # one launch shape; no tile, no batch
    assert a.tune()["rows"] == 0
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(8, 2, 0))
    with pytest.raises(L.LbcgError):
        L.Batch([a])


def test_compact_geometry_f16_within_one_percent(L):
    # FP16 storage (totals, V_axis and R_d rounded stochastically, M in FP32)
    # against FP32 on the flow-focusing junction after 3000 steps: the
    # equivalent radius of the dispersed colour past the junction and the
    # tip of the dispersed thread, as for the FP16 pair state
    w = _focusing()
    nx, ny, nz = w.dims
    xj = nx // 4
    fl = w.mask == 0
    out = {}
    for prec, kernel in (("f32", L.KERNEL_FUSED), ("f16", L.KERNEL_COMPACT), ("f32c", L.KERNEL_COMPACT)):
        s = L.Sim.from_workload(w, precision=prec[:3], kernel=kernel)
        assert s.launch_info()["rows"] == 0
        s.step(3000)
        f = s.fields()
        assert np.isfinite(f["psi"][fl]).all()
        s.close()
        red = np.where(fl, 0.5 * (1.0 + f["psi"]), 0.0)
        vol = red[:, :, xj:].sum()
        out[prec] = ((3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0),
                     int(np.flatnonzero(f["psi"][nz // 2, ny // 2, :] > 0.0).max()))
    (r32, t32) = out["f32"]
    _say(f"focusing 3000 steps: R_eq, tip: pair f32 {out['f32']}, compact f16 {out['f16']}, compact f32 {out['f32c']}")
    assert r32 > 3.0 and t32 > xj
    for k in ("f16", "f32c"):
        r, t = out[k]
        assert abs(r - r32) / r32 < 0.01
        assert abs(t - t32) <= max(1, 0.01 * t32)


def test_compact_geometry_f16_walls_and_reads(L):
    # walls of three codes, periodic elsewhere: colour masses kept to the
    # random walk of the stochastic rounding; a checkpoint resumes on the
    # compact and the pair state
    w = _sparse_geometry((70, 13, 9), seed=92, io=False)
    fl = w.mask == 0
    a = L.Sim.from_workload(w, precision="f16", kernel=L.KERNEL_COMPACT)
    d0 = a.diagnostics()
    a.step(300)
    d1 = a.diagnostics()
    dm = max(abs(d1["mass_R"] / d0["mass_R"] - 1), abs(d1["mass_B"] / d0["mass_B"] - 1))
    _say(f"compact geometry f16, walls, 300 steps: colour mass {dm:.1e}")
    assert dm < 2e-5
    blob = a.get_state()
    a.step(20)
    pa = a.fields()["psi"][fl]
    for kernel in (L.KERNEL_COMPACT, L.KERNEL_FUSED):
        c = L.Sim.from_workload(w, precision="f16", kernel=kernel)
        c.set_state(blob)
        c.step(20)
        d = float(np.abs(c.fields()["psi"][fl] - pa).max())
        _say(f"  f16 resume on kernel {kernel}: max |dpsi| {d:.1e}")
        assert d < 5e-3
        assert c.diagnostics()["step"] == 320
        c.close()
