"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 storage agrees with the oracle to a relative 1e-12 after 100 steps;
FP32 (fused D3Q19) velocity and phase fields within relative L2 1e-5 after
1000 steps; integer/identity properties (tile-shape invariance, determinism,
checkpoint resume) bitwise.
"""
import os

import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, oracle_params, rel_l2

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


def _maxrel(a, b, sel=None):
    a, b = np.asarray(a), np.asarray(b)
    if sel is not None:
        a, b = a[..., sel], b[..., sel]
    return float(np.abs(a - b).max() / np.abs(b).max())


def _random_workload(lat, dims, masked, seed, tau=(1.3, 0.7), A=0.01):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    rR = rng.uniform(0.05, 1, sh)
    rB = rng.uniform(0.05, 1, sh)
    u = rng.uniform(-0.04, 0.04, (3,) + sh)
    if lat == "D2Q9":
        u[2] = 0
    w = W.Workload("random", lat, dims, rR, rB, u, tau[0], tau[1], A, 0.7)
    if masked:
        m = np.zeros(sh, np.uint8)
        m[:, 0, :] = 1
        m[:, -1, :] = 1
        m[:, 1:-1, 0] = 2
        m[:, 1:-1, -1] = 128
        if lat == "D3Q19":
            m[0] = 1
            m[nz // 2, ny // 2, nx // 2] = 1
        w.mask = m
        w.inlets = [{"u": (0.01, 0.002, 0.001 if lat == "D3Q19" else 0.0), "rho_R": 0.8, "rho_B": 0.2}]
        w.outlets = [{"rho": 1.02}]
    return w


@pytest.mark.parametrize("lat,dims", [("D2Q9", (8, 8, 1)), ("D2Q9", (17, 11, 1)),
                                      ("D3Q19", (6, 5, 4)), ("D3Q19", (13, 9, 7))])
@pytest.mark.parametrize("masked", [False, True])
def test_f64_matches_oracle_100_steps(L, orc, lat, dims, masked):
    w = _random_workload(lat, dims, masked, seed=sum(dims) + masked)
    _say(f"f64 parity {lat} {dims} masked={masked}")
    s = L.Sim.from_workload(w, precision="f64", kernel=L.KERNEL_GENERIC)
    o = oracle_for(orc, w)
    fl = np.ones(w.shape, bool) if w.mask is None else w.mask == 0
    assert _maxrel(s.populations(), o.populations(), fl) < 1e-15
    s.step(100)
    o.step(100)
    d = _maxrel(s.populations(), o.populations(), fl)
    _say(f"  max rel diff after 100 steps {d:.2e}")
    assert d < 1e-12


def test_f64_bgk_density_ratio(L, orc):
    # plain BGK (Eq. (5)) with alpha_R != alpha_B (Eq. (7))
    w = _random_workload("D2Q9", (9, 7, 1), False, seed=3)
    s = L.Sim(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.beta, "f64", collision=L.BGK,
              kernel=L.KERNEL_GENERIC, alpha_R=0.3, alpha_B=0.5).init_fields(w.rhoR, w.rhoB, w.u)
    p = oracle_params(orc, w, collision=orc.BGK)
    p.alpha = (0.3, 0.5)
    o = orc.Oracle(p).init(w.rhoR, w.rhoB, w.u)
    s.step(100)
    o.step(100)
    assert _maxrel(s.populations(), o.populations()) < 1e-12


@pytest.mark.parametrize("lat,dims", [("D2Q9", (13, 9, 1)), ("D3Q19", (9, 7, 5))])
def test_f64_regularized_density_ratio(L, orc, lat, dims):
    # regularized collision with alpha_R != alpha_B (Eqs. (7), (8), (11)):
    # the colour equilibria and pressures differ per colour
    w = _random_workload(lat, dims, False, seed=sum(dims) + 7)
    s = L.Sim(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.beta, "f64", kernel=L.KERNEL_GENERIC,
              alpha_R=0.55, alpha_B=0.25).init_fields(w.rhoR, w.rhoB, w.u)
    p = oracle_params(orc, w)
    p.alpha = (0.55, 0.25)
    o = orc.Oracle(p).init(w.rhoR, w.rhoB, w.u)
    s.step(100)
    o.step(100)
    assert _maxrel(s.populations(), o.populations()) < 1e-12


def test_fused_f32_density_ratio_slab(L, orc):
    # FP32 fused kernel, alpha_R = 0.55 (D3Q19: rho^R / rho^B settles at
    # (1 - 1/3) / (1 - 0.55) across a flat interface): the bulk ratio after
    # 10000 steps within 1e-5 of that and of the oracle's.
    nx = 64
    dims = (nx, 8, 4)
    sh = (4, 8, nx)
    psi = np.tanh((16 - np.abs(np.arange(nx) + 0.5 - 32)) / 2.0)
    psi = np.broadcast_to(psi, sh).copy()
    w = W.Workload("slab", "D3Q19", dims, (1 + psi) / 2, (1 - psi) / 2, None, 0.8, 1.2, 0.01, 0.7)
    _say("fused f32 density-ratio slab 64x8x4 x10000")
    s = L.Sim(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.beta, "f32", kernel=L.KERNEL_FUSED,
              alpha_R=0.55).init_fields(w.rhoR, w.rhoB, w.u)
    assert s.launch_info()["kernel"] == L.KERNEL_FUSED
    p = oracle_params(orc, w)
    p.alpha = (0.55, 0.0)
    o = orc.Oracle(p).init(w.rhoR, w.rhoB, w.u)
    s.step(10000)
    o.step(10000)
    g, f = s.fields(), o.fields()
    target = (1 - 1 / 3) / (1 - 0.55)
    rg = g["rhoR"][2, 4, 32] / g["rhoB"][2, 4, 0]
    ro = f["rhoR"][2, 4, 32] / f["rhoB"][2, 4, 0]
    _say(f"  ratio gpu {rg:.7f} oracle {ro:.7f} target {target:.7f}")
    assert abs(rg / target - 1) < 1e-5
    assert abs(rg / ro - 1) < 1e-5
    # bulk densities on both sides (the interfaces themselves may sit ~1e-3
    # apart: FP32 momentum round-off leaves a ~1e-7 drift velocity)
    assert _maxrel(g["rhoR"][..., 26:38], f["rhoR"][..., 26:38]) < 1e-5
    assert _maxrel(g["rhoB"][..., :6], f["rhoB"][..., :6]) < 1e-5


def test_droplet_2d_64_f64(L, orc):
    # D2Q9 static droplet 64x64 (2000 steps): 1e-12 after 100 steps, then
    # per-colour mass conserved to round-off over the whole run (GPU FP64
    # diagnostics).
    w = W.droplet_2d_64()
    s = L.Sim.from_workload(w, precision="f64", kernel=L.KERNEL_GENERIC)
    o = oracle_for(orc, w, threads=8)
    d0 = s.diagnostics()
    s.step(100)
    o.step(100)
    assert _maxrel(s.populations(), o.populations()) < 1e-12
    s.step(w.steps - 100)
    o.step(w.steps - 100)
    g, f = s.fields(), o.fields()
    _say(f"droplet_2d_64 2000 steps: relL2 psi {rel_l2(g['psi'], f['psi']):.2e} u {rel_l2(g['u'], f['u']):.2e}")
    assert rel_l2(g["psi"], f["psi"]) < 1e-10
    d1 = s.diagnostics(check=True)
    eps = np.finfo(float).eps
    assert abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"] < 4 * eps * w.steps
    assert abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"] < 4 * eps * w.steps
    assert d1["p_in"] > d1["p_out"]


@pytest.mark.parametrize("coll", ["reg", "bgk", "bgk_colour"])
def test_fig1_droplet_viscosity_contrast_f64(L, orc, coll):
    # Resting D2Q9 droplet with relaxation time 5 inside and 1 outside (the
    # Fig. 1 set-up) in the three collision forms: regularized and BGK at the
    # node's rate (its mixture viscosity), and BGK with each colour at its
    # own rate.  1e-12 after 100 steps, then the velocity field of step 1000
    # against the oracle's.
    w = W.static_droplet_2d(n=64, R=16.0, noise=0.0)
    w.tau_R, w.tau_B = 5.0, 1.0
    _say(f"fig1 droplet f64 {coll}")
    cl = {"reg": (L.REGULARIZED, orc.REGULARIZED), "bgk": (L.BGK, orc.BGK),
          "bgk_colour": (L.BGK_COLOUR, orc.BGK_COLOUR)}[coll]
    s = L.Sim.from_workload(w, precision="f64", kernel=L.KERNEL_GENERIC, collision=cl[0])
    o = oracle_for(orc, w, threads=8, collision=cl[1])
    s.step(100)
    o.step(100)
    assert _maxrel(s.populations(), o.populations()) < 1e-12
    s.step(900)
    o.step(900)
    g, f = s.fields(), o.fields()
    d = float(np.abs(g["u"] - f["u"]).max() / np.abs(f["u"]).max())
    _say(f"  step 1000 max|u| {np.abs(g['u']).max():.3e}, max rel diff {d:.2e}")
    assert d < 1e-9


def test_fused_f32_droplets_27_recipe_1000_steps(L, orc):
    # The 27-droplet recipe at 48^3 (tau_R = 1, tau_B = 0.6, A = 0.005):
    # FP32 fused kernel vs FP64 oracle after 1000 steps.
    w = W.droplets_27(L=48, seed=2)
    _say("fused f32 48^3 x1000")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    assert s.launch_info()["kernel"] == L.KERNEL_FUSED
    d0 = s.diagnostics()
    s.step(1000)
    g = s.fields()
    d1 = s.diagnostics(check=True)
    # per-colour mass: FP32 rounding is unbiased, so the drift stays far below
    # one FP32 ulp per node-step (a biased reciprocal or codec would not)
    drifts = {k: abs(d1[k] - d0[k]) / d0[k] for k in ("mass_R", "mass_B")}
    _say(f"  mass drift R {drifts['mass_R']:.2e} B {drifts['mass_B']:.2e}")
    o = oracle_for(orc, w, threads=16).step(1000)
    f = o.fields()
    eu, ep = rel_l2(g["u"], f["u"]), rel_l2(g["psi"], f["psi"])
    euf = rel_l2(g["u"], f["u"], floor=1e-4 * np.sqrt(f["u"].size))
    _say(f"  relL2 u {eu:.3e} (floored {euf:.3e}) psi {ep:.3e} |u|rms {np.sqrt((f['u']**2).mean()):.2e}")
    assert eu < 1e-5
    assert ep < 1e-5
    for k, v in drifts.items():
        assert v < 1e-6, (k, v)


def test_fused_matches_generic_ragged(L):
    # nx not a multiple of 64, ny not a multiple of the tile rows
    w = W.droplets_27(L=32, seed=7)
    rng = np.random.default_rng(1)
    nx, ny, nz = 70, 37, 20
    sh = (nz, ny, nx)
    psi = W.droplet_phase((nx, ny, nz), [(20.0, 18.0, 10.0), (50.0, 10.0, 5.0)], [7.0, 5.0])
    rR, rB = W.colour_densities(psi)
    w = W.Workload("ragged", "D3Q19", (nx, ny, nz), rR, rB, rng.normal(0, 1e-3, (3,) + sh), 1.0, 0.6,
                   0.005, 0.7)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_GENERIC)
    a.step(50)
    b.step(50)
    d = _maxrel(a.populations(), b.populations())
    _say(f"fused vs generic ragged 70x37x20 x50: {d:.2e}")
    # Both are FP32 with the same formulas but different instruction order;
    # a few units of FP32 rounding per step accumulate over 50 steps.
    assert d < 50 * 4 * np.finfo(np.float32).eps


@pytest.mark.parametrize("dims", [(96, 40, 24), (64, 16, 9), (5, 3, 2)])
def test_fused_tile_shape_invariance(L, dims):
    # Any tile height and z split gives bitwise the same result (catches LDS
    # halo races and ring/interior mismatches).
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    rng = np.random.default_rng(5)
    psi = W.droplet_phase(dims, [(nx / 3, ny / 2, nz / 2)], [min(dims) / 3 + 1])
    rR, rB = W.colour_densities(psi)
    w = W.Workload("tiles", "D3Q19", dims, rR, rB, rng.normal(0, 1e-3, (3,) + sh), 1.2, 0.7, 0.01, 0.7)
    ref = None
    for tile in ((4, 1, 0), (8, 3, 0), (4, 8, 0), (8, 0, 0)):
        s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED, tile=tile)
        s.step(17)
        p = s.populations()
        if ref is None:
            ref = p
        else:
            assert np.array_equal(p, ref), tile
        s.close()


def test_determinism_and_checkpoint(L):
    w = W.droplets_27(L=40, seed=9)
    a = L.Sim.from_workload(w, precision="f32")
    a.step(40)
    pa = a.populations()
    b = L.Sim.from_workload(w, precision="f32")
    b.step(15)
    blob = b.get_state()
    b.close()
    c = L.Sim.from_workload(w, precision="f32")
    c.set_state(blob)
    c.step(25)
    assert np.array_equal(c.populations(), pa)
    d = L.Sim.from_workload(w, precision="f32")
    d.step(40)
    assert np.array_equal(d.populations(), pa)
    assert c.diagnostics()["step"] == 40


def _sampled_one_step(L, orc, w, s, n_samples=48, seed=0, advance=None, collision=None):
    # Each sampled node's next state depends only on the current state within
    # two nodes, so the oracle steps a periodic 5^3 box cut around it.
    # advance: what takes s one step (default s.step(1); a batch's level);
    # collision: the oracle's relaxation form (default regularized).
    nx, ny, nz = w.dims
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.integers(0, nx, n_samples), rng.integers(0, ny, n_samples),
                        rng.integers(0, nz, n_samples)], 1)
    off = np.arange(-2, 3)
    boxes = []
    for cx, cy, cz in centres:
        zz, yy, xx = np.meshgrid((cz + off) % nz, (cy + off) % ny, (cx + off) % nx, indexing="ij")
        boxes.append((xx + nx * (yy + ny * zz)).reshape(-1))
    nodes = np.concatenate(boxes)
    before = s.populations_at(nodes).reshape(len(centres), 5, 5, 5, 2, 19)
    if advance is None:
        s.step(1)
    else:
        advance()
    after = s.populations_at(np.array([b[62] for b in boxes]))  # 62 = centre of a 5^3 box
    p = orc.Params(lattice=orc.D3Q19, dims=(5, 5, 5), tau=(w.tau_R, w.tau_B), A=(w.A, w.A), beta=w.beta,
                   collision=orc.REGULARIZED if collision is None else collision)
    worst = 0.0
    for j in range(len(centres)):
        o = orc.Oracle(p)
        o.set_populations(np.moveaxis(before[j], (3, 4), (0, 1)))
        o.step(1)
        ref = o.populations()[:, :, 2, 2, 2]
        worst = max(worst, float(np.abs(after[j] - ref).max() / np.abs(ref).max()))
    return worst


def test_full_size_droplets_27_sampled(L, orc):
    # Full 256^3 lattice in the benchmark's launch configuration.
    w = W.droplets_27(L=256, seed=2)
    _say("full size 256^3 fused f32")
    s = L.Sim.from_workload(w, precision="f32")
    info = s.launch_info()
    _say(f"  launch {info}")
    d0 = s.diagnostics(check=True)
    s.step(20)
    worst = _sampled_one_step(L, orc, w, s)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    d1 = s.diagnostics(check=True)
    assert abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"] < 1e-6
    assert abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"] < 1e-6
    s.close()


@pytest.mark.parametrize("edge,kernel", [(304, "fused"), (306, "generic")])
def test_largest_fused_lattice_and_beyond(L, orc, edge, kernel):
    # The fused kernel addresses a state buffer with 32-bit byte offsets:
    # 304^3 FP32 (4.27 GB per buffer) is the largest cube it takes, with
    # offsets up to 2^32 - 25 MB; at 306^3 (4.36 GB) the automatic choice
    # falls back to the generic kernel.  Both stay within the one-step bar.
    w = W.droplets_27(L=edge, seed=2)
    _say(f"{edge}^3 f32, expect {kernel}")
    s = L.Sim.from_workload(w, precision="f32")
    info = s.launch_info()
    _say(f"  launch {info}")
    assert info["kernel"] == (L.KERNEL_FUSED if kernel == "fused" else L.KERNEL_GENERIC)
    s.step(3)
    worst = _sampled_one_step(L, orc, w, s, n_samples=32, seed=edge)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    s.close()


def test_library_loaded_before_torch_in_fresh_process(L):
    # A caller that imports the binding and creates a lattice without ever
    # importing torch itself: the binding must still run on torch's HIP
    # runtime (the one that owns the device memory it hands over).
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, '.');"
            "from paper_1711_02003_amd import lbcg, workloads as W;"
            "w = W.droplets_27(L=16, seed=2);"
            "s = lbcg.Sim.from_workload(w, precision='f32');"
            "s.step(3); f = s.fields();"
            "assert abs(f['rhoR'].sum() + f['rhoB'].sum() - 16 ** 3) < 1e-2;"
            "print('fresh process ok', flush=True)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    _say(r.stdout.strip()[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "fresh process ok" in r.stdout


_LAPLACE_ORACLE = {}


@pytest.mark.parametrize("kernel", ["fused", "compact"])
def test_laplace_law_3d_fused_f32_matches_oracle(L, orc, kernel):
    # Static spheres R in {6, 8, 10} in 32^3 (tau = 1, A = 0.005, 1500 steps):
    # the FP32 fused D3Q19 sweep, on the pair and on the compact state, gives
    # the oracle's effective radii, pressure jumps (p = rho / 3, Eq. (8) for
    # D3Q19 with alpha = w_0) and fitted surface tension of dp = 2 sigma / R.
    n = 32
    zz, yy, xx = np.mgrid[0:n, 0:n, 0:n]
    c = (n - 1) / 2
    r = np.sqrt((xx - c) ** 2 + (yy - c) ** 2 + (zz - c) ** 2)

    def jump(f):
        p = (f["rhoR"] + f["rhoB"]) / 3
        Reff = (3 * ((1 + f["psi"]) / 2).sum() / (4 * np.pi)) ** (1 / 3)
        return Reff, p[r < Reff - 4].mean() - p[r > Reff + 5].mean()

    kid = {"fused": L.KERNEL_FUSED, "compact": L.KERNEL_COMPACT}[kernel]
    res = {"gpu": [], "orc": []}
    for R in (6.0, 8.0, 10.0):
        w = W.static_droplet_3d(n, R=R, A=0.005)
        s = L.Sim.from_workload(w, precision="f32", kernel=kid)
        assert s.launch_info()["kernel"] == kid
        s.step(1500)
        res["gpu"].append(jump(s.fields()))
        s.close()
        if R not in _LAPLACE_ORACLE:
            _LAPLACE_ORACLE[R] = jump(oracle_for(orc, w, threads=16).step(1500).fields())
        res["orc"].append(_LAPLACE_ORACLE[R])
    fits = {}
    for k, v in res.items():
        Rs, dps = np.array(v).T
        M = np.vstack([2 / Rs, np.ones(len(Rs))]).T
        (sigma, c0), *_ = np.linalg.lstsq(M, dps, rcond=None)
        fits[k] = sigma
    _say(f"  radii gpu {[round(x[0], 5) for x in res['gpu']]} oracle {[round(x[0], 5) for x in res['orc']]}; "
         f"sigma gpu {fits['gpu']:.6e} oracle {fits['orc']:.6e}")
    for (Rg, dg), (Ro, do) in zip(res["gpu"], res["orc"]):
        assert abs(Rg - Ro) < 1e-4
        assert abs(dg / do - 1) < 1e-3
    assert abs(fits["gpu"] / fits["orc"] - 1) < 1e-3
