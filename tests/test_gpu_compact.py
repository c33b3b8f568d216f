"""GPU parity of the compact-state sweeps (LBCG_KERNEL_COMPACT), D3Q19 and D2Q9.

The compact state keeps, per node, the 19 total populations and 7 colour
scalars from which the receiver of a population splits it into colours
(Eq. (10) is linear in f_i, with coefficients of the sending node and of the
speed class of c_i).  In exact arithmetic the step is the pair-state step, so
the bars are those of the FP32 pair-state fused kernel: velocity and phase
within relative L2 1e-5 of the FP64 oracle after 1000 steps, colour mass
drift below 1e-6, sampled one-step agreement within 2e-6 at the full
256^3 size, and bitwise invariance under the tile shape and under reads of
the state.
"""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, oracle_params, rel_l2
from tests.test_gpu_parity import _maxrel, _sampled_one_step

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


def _droplets(dims, seed, tau=(1.2, 0.7), A=0.01):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    psi = W.droplet_phase(dims, [(nx / 3, ny / 2, nz / 2), (0.8 * nx, 0.2 * ny, 0.7 * nz)],
                          [min(dims) / 3 + 1, min(dims) / 5 + 1])
    rR, rB = W.colour_densities(psi)
    return W.Workload("compact", "D3Q19", dims, rR, rB, rng.normal(0, 1e-3, (3, nz, ny, nx)), tau[0], tau[1],
                      A, 0.7)


def test_compact_droplets_27_recipe_1000_steps(L, orc):
    # The 27-droplet recipe at 48^3 (tau_R = 1, tau_B = 0.6, A = 0.005).
    w = W.droplets_27(L=48, seed=2)
    _say("compact f32 48^3 x1000")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    assert s.launch_info()["kernel"] == L.KERNEL_COMPACT
    d0 = s.diagnostics()
    s.step(1000)
    g = s.fields()
    d1 = s.diagnostics(check=True)
    drifts = {k: abs(d1[k] - d0[k]) / d0[k] for k in ("mass_R", "mass_B")}
    _say(f"  mass drift R {drifts['mass_R']:.2e} B {drifts['mass_B']:.2e}")
    o = oracle_for(orc, w, threads=16).step(1000)
    f = o.fields()
    eu, ep = rel_l2(g["u"], f["u"]), rel_l2(g["psi"], f["psi"])
    _say(f"  relL2 u {eu:.3e} psi {ep:.3e}")
    assert eu < 1e-5
    assert ep < 1e-5
    for k, v in drifts.items():
        assert v < 1e-6, (k, v)


@pytest.mark.timeout(900)
def test_compact_droplets_27_recipe_128_1000_steps(L, orc):
    # The 27-droplet recipe at 128^3 (two full 64-wide x tiles, 16 row tiles)
    # on the compact kernel in its tuned launch shape, as the benchmark runs
    # it, after 1000 steps against the FP64 oracle: rel-L2 of psi within 1e-5;
    # of u within 1e-5 floored at 1e-4 sqrt(N) (the initial N(0, 1e-3)
    # velocities have decayed to ~1e-5 rms by then, and FP32 forms u to
    # ~2e-10 absolute from momentum sums that cancel, so the plain ratio
    # measures that floor: 2.4e-5 here, bounded by 1e-4).
    w = W.droplets_27(L=128, seed=2)
    _say("compact f32 128^3 x1000 (tuned shape)")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    s.step(1)
    shape = s.tune()
    _say(f"  tuned shape {shape}")
    s.step(999)
    g = s.fields()
    s.close()
    o = oracle_for(orc, w, threads=16).step(1000)
    f = o.fields()
    eu, ep = rel_l2(g["u"], f["u"]), rel_l2(g["psi"], f["psi"])
    euf = rel_l2(g["u"], f["u"], floor=1e-4 * np.sqrt(w.nodes))
    _say(f"  relL2 u {eu:.3e} (floored {euf:.3e}) psi {ep:.3e} (|u|_rms {np.sqrt((f['u'] ** 2).mean()):.2e})")
    assert euf < 1e-5 and eu < 1e-4
    assert ep < 1e-5


def test_compact_density_ratio_slab(L, orc):
    # alpha_R = 0.55 != alpha_B: the colour equilibria differ per colour, so
    # the scalars' class amplitudes carry the phi_i^k terms.  The bulk ratio
    # after 10000 steps within 1e-5 of the flat-interface value and of the
    # oracle's.
    nx = 64
    dims = (nx, 8, 4)
    sh = (4, 8, nx)
    psi = np.tanh((16 - np.abs(np.arange(nx) + 0.5 - 32)) / 2.0)
    psi = np.broadcast_to(psi, sh).copy()
    w = W.Workload("slab", "D3Q19", dims, (1 + psi) / 2, (1 - psi) / 2, None, 0.8, 1.2, 0.01, 0.7)
    _say("compact f32 density-ratio slab 64x8x4 x10000")
    s = L.Sim(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.beta, "f32", kernel=L.KERNEL_COMPACT,
              alpha_R=0.55).init_fields(w.rhoR, w.rhoB, w.u)
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
    assert _maxrel(g["rhoR"][..., 26:38], f["rhoR"][..., 26:38]) < 1e-5
    assert _maxrel(g["rhoB"][..., :6], f["rhoB"][..., :6]) < 1e-5


def test_compact_agrees_with_pair_fused_ragged(L):
    # nx not a multiple of 64, ny not a multiple of the tile rows: the compact
    # and the pair-state sweeps differ only in rounding
    w = _droplets((70, 37, 20), seed=3)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    a.step(50)
    b.step(50)
    d = _maxrel(a.populations(), b.populations())
    _say(f"compact vs fused ragged 70x37x20 x50: {d:.2e}")
    assert d < 50 * 4 * EPS32


@pytest.mark.parametrize("dims", [(96, 40, 24), (64, 16, 9), (5, 3, 2), (33, 17, 12)])
def test_compact_tile_shape_invariance(L, dims):
    # every tile width (64 or 32), z split and automatic shape gives bitwise
    # the same state: ring and interior nodes split the pulled populations by
    # one expression sequence
    w = _droplets(dims, seed=5)
    ref = None
    for tile in ((8, 1, 0), (8, 3, 0), (8, 8, 0), (8, 0, 0), (8, 1, 32), (8, 3, 32), (8, 0, 32)):
        s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=tile)
        s.step(17)
        p = s.populations()
        if ref is None:
            ref = p
        else:
            assert np.array_equal(p, ref), tile
        s.close()


def test_compact_concurrent_streams_match_sequential(L):
    # handles on their own streams stepping at the same time, with chunks
    # down to one plane (every record plane read by other blocks than the
    # one that wrote it): bitwise the result of one handle stepped alone
    w = W.droplets_27(L=64, seed=3)
    ref = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(8, 1, 0))
    ref.step(20)
    ref.synchronize()
    pr = ref.populations()
    for zc, tx in ((64, 64), (8, 32), (2, 64), (64, 32)):
        a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(8, zc, tx))
        b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(8, 1, 96 - tx))
        a.step(20)
        b.step(20)
        assert np.array_equal(a.populations(), pr), zc
        assert np.array_equal(b.populations(), pr), zc
        a.close()
        b.close()


def test_compact_reads_leave_trajectory_unchanged(L):
    # reading the state converts it into the pair buffer but steps go on from
    # the compact state: a run with reads is bitwise the run without
    w = _droplets((64, 24, 16), seed=8)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    for _ in range(3):
        a.step(10)
        a.populations()
        a.diagnostics()
        a.fields()
    b.step(30)
    assert np.array_equal(a.populations(), b.populations())
    assert a.diagnostics()["step"] == 30


def test_compact_checkpoint_resume(L):
    # a checkpoint of a compact handle is a pair state: it resumes on a
    # compact or a pair-state handle, within rounding of the uninterrupted run
    w = W.droplets_27(L=40, seed=9)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    a.step(40)
    pa = a.populations()
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b.step(15)
    blob = b.get_state()
    for kernel in (L.KERNEL_COMPACT, L.KERNEL_FUSED):
        c = L.Sim.from_workload(w, precision="f32", kernel=kernel)
        c.set_state(blob)
        c.step(25)
        d = _maxrel(c.populations(), pa)
        _say(f"resume on kernel {kernel}: {d:.2e}")
        assert d < 25 * 4 * EPS32
        assert c.diagnostics()["step"] == 40
        c.close()


def test_compact_full_size_droplets_27_sampled(L, orc):
    # Full 256^3 lattice: sampled nodes' next state against the oracle's step
    # from the same (converted) state, and colour masses over 20 steps.
    w = W.droplets_27(L=256, seed=2)
    _say("full size 256^3 compact f32")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    _say(f"  launch {s.launch_info()}")
    d0 = s.diagnostics(check=True)
    s.step(20)
    worst = _sampled_one_step(L, orc, w, s)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    d1 = s.diagnostics(check=True)
    assert abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"] < 1e-6
    assert abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"] < 1e-6
    s.close()


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 3), (1, 4, 1), (3, 3, 2)])
def test_compact_degenerate_lattices(L, dims):
    # one node, one-wide dimensions: every neighbour wraps onto the node or
    # its few neighbours; the compact sweep agrees with the pair-state sweep
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    w = W.Workload("tiny", "D3Q19", dims, rng.uniform(0.2, 1, sh), rng.uniform(0.2, 1, sh),
                   rng.uniform(-0.02, 0.02, (3,) + sh), 1.2, 0.7, 0.01, 0.7)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    a.step(30)
    b.step(30)
    d = _maxrel(a.populations(), b.populations())
    _say(f"compact vs fused {dims} x30: {d:.2e}")
    assert d < 30 * 4 * EPS32


def test_compact_largest_lattice_and_beyond(L, orc):
    # The first compact step reads the pair state with 32-bit byte offsets:
    # 304^3 (4.27 GB per pair buffer) is the largest cube the compact kernel
    # takes; 306^3 is refused (the automatic choice would use the generic
    # kernel there).
    w = W.droplets_27(L=304, seed=2)
    _say("304^3 compact f32")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    assert s.launch_info()["kernel"] == L.KERNEL_COMPACT
    s.step(3)
    worst = _sampled_one_step(L, orc, w, s, n_samples=32, seed=304)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    s.close()
    with pytest.raises(L.LbcgError):
        L.Sim("D3Q19", (306, 306, 306), 1.0, 0.6, 0.005, 0.7, "f32", kernel=L.KERNEL_COMPACT)


def test_compact_rejects_what_it_does_not_cover(L):
    w = _droplets((16, 8, 8), seed=1)
    for kw in ({"precision": "f64"}, {"collision": L.BGK}):
        with pytest.raises(L.LbcgError):
            L.Sim.from_workload(w, kernel=L.KERNEL_COMPACT, **kw)
    m = np.zeros(w.shape, np.uint8)
    m[:, 0, :] = 1
    w.mask = m
    # with geometry: D3Q19 FP32 and FP16, on the split step
    for prec in ("f32", "f16"):
        assert L.Sim.from_workload(w, precision=prec, kernel=L.KERNEL_COMPACT).launch_info()["rows"] == 0
    w2 = W.droplets_2d(n=64, seed=1)
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(w2, precision="f16", kernel=L.KERNEL_COMPACT)
    m2 = np.zeros(w2.rhoR.shape, np.uint8)
    m2[:, 0, :] = 1
    w2.mask = m2
    with pytest.raises(L.LbcgError):
        L.Sim.from_workload(w2, precision="f32", kernel=L.KERNEL_COMPACT)
    w.mask = None
    with pytest.raises(L.LbcgError):  # 8-row tiles only
        L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(4, 0, 0))


# ---------------------------------------------------------------- D2Q9

def _random_2d(dims, seed):
    rng = np.random.default_rng(seed)
    nx, ny, _ = dims
    sh = (1, ny, nx)
    u = np.zeros((3,) + sh)
    u[:2] = rng.uniform(-0.04, 0.04, (2,) + sh)
    return W.Workload("random2d", "D2Q9", dims, rng.uniform(0.05, 1, sh), rng.uniform(0.05, 1, sh), u,
                      1.3, 0.7, 0.01, 0.7)


@pytest.mark.parametrize("dims", [(64, 64, 1), (100, 37, 1), (130, 9, 1), (5, 3, 1), (1, 1, 1), (1, 6, 1), (7, 1, 1)])
def test_compact2d_agrees_with_pair_fused(L, dims):
    # several strips, a ragged strip, a lattice narrower than the record halo
    w = _random_2d(dims, seed=sum(dims) + 1)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    assert a.launch_info()["kernel"] == L.KERNEL_COMPACT
    a.step(50)
    b.step(50)
    d = _maxrel(a.populations(), b.populations())
    _say(f"compact2d vs fused2d {dims} x50: {d:.2e}")
    assert d < 50 * 4 * EPS32


@pytest.mark.parametrize("ychunks", [3, 16, 256])
def test_compact2d_chunk_invariance(L, ychunks):
    w = W.droplets_2d(n=256, seed=6)
    ref = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(0, 1, 0))
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(0, ychunks, 0))
    assert s.launch_info()["zchunks"] == ychunks
    ref.step(20)
    ref.synchronize()
    s.step(20)
    assert np.array_equal(s.populations(), ref.populations())


def test_compact2d_concurrent_streams_match_sequential(L):
    # one-row chunks stepping while other handles run on their own streams:
    # every row's records are written in the last stores of a wave, under
    # the memory traffic of the other kernels; bitwise the handle alone
    w = W.droplets_2d(n=256, seed=6)
    ref = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(0, 1, 0))
    ref.step(20)
    ref.synchronize()
    pr = ref.populations()
    for trial in range(3):
        for yc in (256, 64):
            a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(0, yc, 0))
            b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED, tile=(0, 1, 0))
            c = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT, tile=(0, 1, 0))
            b.step(60)
            c.step(60)
            a.step(20)
            assert np.array_equal(a.populations(), pr), (trial, yc)
            for h in (a, b, c):
                h.close()


def test_compact2d_f32_matches_oracle_1000_steps(L, orc):
    # 256^2 with 256 droplets (tau_R = 1, tau_B = 0.6, A = 0.005), tuned shape
    w = W.droplets_2d(n=256, seed=6)
    _say("compact2d f32 256^2 x1000")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    s.step(2)
    s.tune()
    o = oracle_for(orc, w, threads=8)
    o.step(2)
    d0 = s.diagnostics(check=True)
    s.step(998)
    o.step(998)
    g, f = s.fields(), o.fields()
    eu, ep = rel_l2(g["u"], f["u"]), rel_l2(g["psi"], f["psi"])
    _say(f"  relL2 u {eu:.3e} psi {ep:.3e}")
    assert eu < 1e-5 and ep < 1e-5
    d1 = s.diagnostics(check=True)
    assert abs(d1["mass_R"] - d0["mass_R"]) / d0["mass_R"] < 1e-6
    assert abs(d1["mass_B"] - d0["mass_B"]) / d0["mass_B"] < 1e-6


def _sampled_one_step_2d(orc, w, s, n_samples=48, seed=3):
    # A D2Q9 node's next state depends only on the current state within two
    # nodes, so the oracle steps a periodic 5 x 5 box cut around each
    # sampled node; the largest relative difference of its populations.
    nx, ny, _ = w.dims
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.integers(0, nx, n_samples), rng.integers(0, ny, n_samples)], 1)
    off = np.arange(-2, 3)
    boxes = []
    for cx, cy in centres:
        yy, xx = np.meshgrid((cy + off) % ny, (cx + off) % nx, indexing="ij")
        boxes.append((xx + nx * yy).reshape(-1))
    before = s.populations_at(np.concatenate(boxes)).reshape(len(centres), 1, 5, 5, 2, 9)
    s.step(1)
    after = s.populations_at(np.array([b[12] for b in boxes]))  # 12 = centre of a 5 x 5 box
    p = orc.Params(lattice=orc.D2Q9, dims=(5, 5, 1), tau=(w.tau_R, w.tau_B), A=(w.A, w.A), beta=w.beta)
    worst = 0.0
    for j in range(len(centres)):
        o = orc.Oracle(p)
        o.set_populations(np.moveaxis(before[j], (3, 4), (0, 1)))
        o.step(1)
        ref = o.populations()[:, :, 0, 2, 2]
        worst = max(worst, float(np.abs(after[j] - ref).max() / np.abs(ref).max()))
    return worst


def test_compact2d_full_size_sampled(L, orc):
    # the benchmark's 4096^2 D2Q9 lattice in its tuned launch shape
    w = W.droplets_2d(n=4096, seed=6)
    _say("full size 4096^2 compact2d f32")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    s.step(2)
    s.tune()
    s.step(18)
    worst = _sampled_one_step_2d(orc, w, s)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6


@pytest.mark.parametrize("kernel", ["fused", "compact"])
def test_d2q9_largest_lattice_and_beyond(L, orc, kernel):
    # The D2Q9 strip sweeps (pair and compact state) address the pair state
    # with 32-bit byte offsets: 7712^2 FP32 (4.28 GB per pair buffer, offsets
    # up to 2^32 - 13 MB) is the largest square they take, one step at 32
    # sampled nodes against the oracle; at 7744^2 (4.32 GB) both refuse and
    # the automatic choice is the generic kernel.
    k = {"fused": L.KERNEL_FUSED, "compact": L.KERNEL_COMPACT}[kernel]
    w = W.droplets_2d(n=7712, seed=6)
    _say(f"7712^2 D2Q9 f32 {kernel}")
    s = L.Sim.from_workload(w, precision="f32", kernel=k)
    assert s.launch_info()["kernel"] == k
    s.step(3)
    worst = _sampled_one_step_2d(orc, w, s, n_samples=32, seed=7712)
    _say(f"  sampled one-step max rel diff {worst:.2e}")
    assert worst < 2e-6
    s.close()
    del w
    with pytest.raises(L.LbcgError):
        L.Sim("D2Q9", (7744, 7744, 1), 1.0, 0.6, 0.005, 0.7, "f32", kernel=k)
    g = L.Sim("D2Q9", (7744, 7744, 1), 1.0, 0.6, 0.005, 0.7, "f32")
    assert g.launch_info()["kernel"] == L.KERNEL_GENERIC
    g.close()


def test_compact2d_reads_and_resume(L):
    w = W.droplets_2d(n=128, seed=2)
    a = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    b = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    for _ in range(3):
        a.step(10)
        a.populations()
        a.diagnostics()
    b.step(30)
    assert np.array_equal(a.populations(), b.populations())
    c = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_FUSED)
    c.set_state(b.get_state())
    b.step(20)
    c.step(20)
    assert _maxrel(c.populations(), b.populations()) < 20 * 4 * EPS32
