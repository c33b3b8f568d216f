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


def test_geometry_split_steps_1000_steps_match_oracle(L, orc):
    # the split step on the pair state and on the compact state, FP32, after
    # 1000 steps of driven flow through the quarter-size junction
    w = _focusing()
    fl = w.mask == 0
    f = oracle_for(orc, w, threads=16).step(1000).fields()
    for kernel in (L.KERNEL_FUSED, L.KERNEL_COMPACT):
        s = L.Sim.from_workload(w, precision="f32", kernel=kernel)
        assert s.launch_info()["rows"] == 0
        s.step(1000)
        g = s.fields()
        s.close()
        ep = rel_l2(g["psi"][fl], f["psi"][fl])
        eu = rel_l2(g["u"][:, fl], f["u"][:, fl])
        _say(f"split step (kernel {kernel}) vs oracle, focusing 128x48x14 x1000: relL2 psi {ep:.2e} u {eu:.2e}")
        assert ep < 1e-5 and eu < 1e-5


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


def test_geometry_f32_f16_within_one_percent_of_oracle(L, orc):
    # The split steps on the flow-focusing junction after 3000 steps against
    # the FP64 oracle, FP32 and FP16 storage on the pair and the compact state
    # (FP16 compact: totals, V_axis and R_d rounded stochastically, M in
    # FP32): the equivalent radius of the dispersed colour past the junction
    # and the tip of the dispersed thread within 1 %
    w = _focusing()
    nx, ny, nz = w.dims
    xj = nx // 4
    fl = w.mask == 0

    def measures(f):
        red = np.where(fl, 0.5 * (1.0 + f["psi"]), 0.0)
        vol = red[:, :, xj:].sum()
        return ((3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0),
                int(np.flatnonzero(f["psi"][nz // 2, ny // 2, :] > 0.0).max()))

    out = {"oracle": measures(oracle_for(orc, w, threads=16).step(3000).fields())}
    forms = {"pair f32": ("f32", L.KERNEL_FUSED), "pair f16": ("f16", L.KERNEL_FUSED),
             "compact f32": ("f32", L.KERNEL_COMPACT), "compact f16": ("f16", L.KERNEL_COMPACT)}
    for name, (prec, kernel) in forms.items():
        s = L.Sim.from_workload(w, precision=prec, kernel=kernel)
        assert s.launch_info()["rows"] == 0
        s.step(3000)
        f = s.fields()
        assert np.isfinite(f["psi"][fl]).all()
        s.close()
        out[name] = measures(f)
    r0, t0 = out["oracle"]
    _say("focusing 3000 steps: R_eq, tip: " + ", ".join(f"{k} ({v[0]:.4f}, {v[1]})" for k, v in out.items()))
    assert r0 > 3.0 and t0 > xj
    for k in forms:
        r, t = out[k]
        assert abs(r - r0) / r0 < 0.01
        assert abs(t - t0) <= max(1, 0.01 * t0)


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


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_compact_geometry_single_fluid_node_and_no_fluid(L, prec):
    # one fluid node in a lattice of walls (every link from a wall, so every
    # pull is the node's own total of the opposite direction); and a lattice
    # with no fluid node at all, which still advances the step counter and
    # exports zeros
    m = np.ones((4, 6, 70), np.uint8)
    m[2, 3, 66] = 0
    sh = m.shape
    u = np.zeros((3,) + sh)
    u[:, 2, 3, 66] = (0.02, -0.01, 0.015)
    w = W.Workload("one", "D3Q19", (70, 6, 4), np.full(sh, 0.6), np.full(sh, 0.4), u, 1.0, 0.8, 0.01, 0.7,
                   mask=m)
    fl = m == 0
    a = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_FUSED)
    assert a.launch_info()["rows"] == 0 and b.launch_info()["rows"] == 0
    d0 = a.diagnostics()
    a.step(30)
    b.step(30)
    pa, pb = a.populations()[..., fl], b.populations()[..., fl]
    d = float(np.abs(pa - pb).max() / np.abs(pb).max())
    d1 = a.diagnostics()
    dm = max(abs(d1["mass_R"] / d0["mass_R"] - 1), abs(d1["mass_B"] / d0["mass_B"] - 1))
    _say(f"compact geometry {prec}, one fluid node x30: max rel difference {d:.2e}, colour mass {dm:.1e}")
    assert np.isfinite(pa).all()
    assert d < (60 * EPS32 if prec == "f32" else 5e-3)
    assert dm < (1e-6 if prec == "f32" else 1e-4)
    assert d1["step"] == 30 and d1["status"] == 0
    w.mask = np.ones_like(m)
    e = L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_COMPACT)
    assert e.launch_info()["rows"] == 0
    e.step(7)
    assert e.diagnostics()["step"] == 7
    assert not np.any(e.populations())
    e.step(2)
    assert e.diagnostics()["step"] == 9


def test_compact_geometry_largest_lattice(L):
    # The compact state with geometry takes lattices whose FP32 pair state
    # stays below 4 GiB: 304^3 (pair buffers of 4.27 GB, compact buffers of
    # 2.70 GB, 32-bit byte offsets up to 2^32 - 25 MB) here with a neutral
    # and a wetting wall face, an inlet and an outlet face.  Sampled fluid
    # nodes, those of the last planes among them, agree with the pair state's
    # column sweep to FP32 rounding after 3 steps; at 306^3 the compact kernel
    # is refused.
    edge = 304
    w = W.droplets_27(L=edge, seed=2)
    m = np.zeros((edge,) * 3, np.uint8)
    m[:, 0, :] = 1
    m[:, -1, :] = 64
    m[:, 1:-1, 0] = 2
    m[:, 1:-1, -1] = 128
    w.mask = m
    w.inlets = [{"u": (0.01, 0.0, 0.0), "rho_R": 0.9, "rho_B": 0.1}]
    w.outlets = [{"rho": 1.0}]
    w.walls = [{"psi": 0.5}]
    rng = np.random.default_rng(304)
    x = np.concatenate([rng.integers(1, edge - 1, 200), [1, edge - 2, edge - 2, 1]])
    y = np.concatenate([rng.integers(1, edge - 1, 200), [1, edge - 2, 1, edge - 2]])
    z = np.concatenate([rng.integers(0, edge, 150), np.full(50, edge - 1), [edge - 1, edge - 1, 0, 0]])
    nodes = (x + edge * (y + edge * z)).astype(np.int64)
    assert (m.reshape(-1)[nodes] == 0).all()
    out = {}
    for name, kernel in (("compact", L.KERNEL_COMPACT), ("pair", L.KERNEL_FUSED)):
        _say(f"{edge}^3 f32 with geometry, {name}")
        s = L.Sim.from_workload(w, precision="f32", kernel=kernel)
        assert s.launch_info()["rows"] == (0 if name == "compact" else 8)  # mostly fluid: the column sweep
        s.step(3)
        out[name] = s.populations_at(nodes)
        d = s.diagnostics()
        assert d["step"] == 3 and d["status"] == 0
        s.close()
    pa, pb = out["compact"], out["pair"]
    assert np.isfinite(pa).all()
    diff = float(np.abs(pa - pb).max() / np.abs(pb).max())
    _say(f"  sampled max rel difference compact vs pair {diff:.2e}")
    assert diff < 30 * EPS32
    del w, m
    sh = (306,) * 3
    big = W.Workload("channel", "D3Q19", sh, np.full(sh, 0.6), np.full(sh, 0.4), None, 1.0, 0.8, 0.01, 0.7,
                     mask=np.pad(np.zeros((306, 304, 306), np.uint8), ((0, 0), (1, 1), (0, 0)), constant_values=1))
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(big, precision="f32", kernel=L.KERNEL_COMPACT)
