"""GPU FP64 diagnostics (lbcg_diagnostics) against the oracle's
(orc_diagnostics): colour masses (Eq. (2)), momentum (Eq. (3)), max |u|, the
Eq. (8) pressures inside and outside, R_eff and the count of non-finite
nodes; and the LBCG_E_UNSTABLE path.

Bars:
  * FP64 lattices, each side on its own trajectory: relative 1e-12 after 100
    steps (the states themselves agree to 1e-12), integer counts exact;
  * the same state reduced on both sides (the GPU state exported through
    lbcg_populations and loaded into the oracle): both form every node's
    moments in FP64 from the same values in the same order, so only the
    order of the global FP64 sums differs: relative 1e-12 on sums over up to
    2^21 nodes (a node-order sum of n terms errs by at most n eps relative,
    ~4e-10 here; the measured differences are ~1e-15), max |u| to the last
    bit and the counts exactly;
  * the FP32 compact kernel at 256^3 after 10 steps against the oracle's own
    10 steps: masses, pressures and vol_R within 1e-6 relative (FP32 state
    error ~1e-7 per node, unbiased), max |u| within 1e-4 (u ~ 5e-3 is formed
    from momentum sums that cancel to ~1e-8 in FP32), inside/outside counts
    within 1e-4 of each other (nodes within FP32 round-off of psi = +-0.99).
"""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, oracle_params

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


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _compare(g, o, nodes, tol, counts_exact=True, max_u_tol=None, tag=""):
    """g: lbcg diag dict, o: oracle diag dict."""
    worst = {
        "mass_R": _rel(g["mass_R"], o["mass"][0]),
        "mass_B": _rel(g["mass_B"], o["mass"][1]),
        "p_in": _rel(g["p_in"], o["p_in"]) if o["n_in"] else abs(g["p_in"]),
        "p_out": _rel(g["p_out"], o["p_out"]) if o["n_out"] else abs(g["p_out"]),
        "vol_R": _rel(g["vol_R"], o["vol_R"]),
        "R_eff": _rel(g["R_eff"], o["R_eff"]),
        "max_u": _rel(g["max_u"], o["max_u"]),
    }
    # momentum sums cancel: bound their difference by the mass scale
    mom = max(abs(g["momentum"][a] - o["momentum"][a]) for a in range(3)) / (o["mass"][0] + o["mass"][1])
    _say(f"  {tag} diag rel diffs " + " ".join(f"{k} {v:.1e}" for k, v in worst.items()) + f" mom {mom:.1e}")
    for k, v in worst.items():
        if k == "max_u" and max_u_tol is not None:
            assert v <= max_u_tol, (k, v)
        else:
            assert v <= tol, (k, v)
    assert mom <= tol
    assert g["fluid_nodes"] == o["fluid_nodes"] == nodes
    assert g["nonfinite"] == o["nonfinite"]
    if counts_exact:
        assert g["n_in"] == o["n_in"] and g["n_out"] == o["n_out"]
    else:
        assert abs(g["n_in"] - o["n_in"]) <= 1e-4 * max(o["n_in"], 1) + 2
        assert abs(g["n_out"] - o["n_out"]) <= 1e-4 * max(o["n_out"], 1) + 2


def _random_masked(lat, dims, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    rR = rng.uniform(0.05, 1, sh)
    rB = rng.uniform(0.05, 1, sh)
    # a red block and a blue block, so that both bulk pressures have nodes
    rR[..., : nx // 3] = 1.0
    rB[..., : nx // 3] = 0.0
    rR[..., -(nx // 3):] = 0.0
    rB[..., -(nx // 3):] = 1.0
    u = rng.uniform(-0.02, 0.02, (3,) + sh)
    if lat == "D2Q9":
        u[2] = 0
    w = W.Workload("random", lat, dims, rR, rB, u, 1.3, 0.7, 0.01, 0.7)
    m = np.zeros(sh, np.uint8)
    m[:, 0, :] = 1
    m[:, -1, :] = 1
    if lat == "D3Q19":
        m[0] = 1
    w.mask = m
    return w


@pytest.mark.parametrize("case", ["droplet_2d_64", "d2q9_masked", "d3q19_masked", "d3q19_droplet"])
def test_f64_diagnostics_match_oracle(L, orc, case):
    if case == "droplet_2d_64":
        w = W.droplet_2d_64()
    elif case == "d2q9_masked":
        w = _random_masked("D2Q9", (30, 17, 1), 5)
    elif case == "d3q19_masked":
        w = _random_masked("D3Q19", (21, 13, 9), 6)
    else:
        w = W.static_droplet_3d(n=24, R=7.0, tau=(1.2, 0.8), A=0.01)
    _say(f"f64 diagnostics {case} {w.dims}")
    s = L.Sim.from_workload(w, precision="f64", kernel=L.KERNEL_GENERIC)
    o = oracle_for(orc, w, threads=8)
    nodes = int(w.nodes if w.mask is None else (w.mask == 0).sum())
    _compare(s.diagnostics(check=True), o.diagnostics(), nodes, 1e-12, tag="t=0")
    s.step(100)
    o.step(100)
    g = s.diagnostics(check=True)
    assert g["step"] == 100
    _compare(g, o.diagnostics(), nodes, 1e-12, tag="t=100")


@pytest.mark.parametrize("kernel", ["compact", "fused_f16"])
def test_same_state_reduction(L, orc, kernel):
    # The GPU reduction and the oracle's on one and the same state: the
    # 27-droplet recipe at 128^3 on the compact kernel, a 64^3 droplet with
    # FP16 storage.  Per-node moments agree bitwise, so max |u| may differ
    # by the last bit at most (both sides round sqrt and division correctly).
    if kernel == "compact":
        w = W.droplets_27(L=128, seed=2)
        s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    else:
        w = W.static_droplet_3d(n=64, R=16.0, tau=(1.0, 0.7), A=0.005)
        s = L.Sim.from_workload(w, precision="f16")
    _say(f"same-state diagnostics {kernel} {w.dims}")
    s.step(37)
    g = s.diagnostics(check=True)
    f = s.populations()
    o = orc.Oracle(oracle_params(orc, w, threads=8)).set_populations(f)
    _compare(g, o.diagnostics(), w.nodes, 1e-12, max_u_tol=2.3e-16, tag=kernel)


@pytest.mark.timeout(900)
def test_compact_256_diagnostics_vs_oracle_trajectory(L, orc):
    # the benchmark's lattice (27 droplets, 256^3) and kernel, 10 steps
    w = W.droplets_27(L=256, seed=2)
    _say("compact 256^3 x10 diagnostics vs the oracle's own trajectory")
    s = L.Sim.from_workload(w, precision="f32", kernel=L.KERNEL_COMPACT)
    s.step(1)
    s.tune()
    s.step(9)
    g = s.diagnostics(check=True)
    s.close()
    o = oracle_for(orc, w, threads=16).step(10)
    _compare(g, o.diagnostics(), w.nodes, 1e-6, counts_exact=False, max_u_tol=1e-4, tag="256^3")


@pytest.mark.parametrize("prec,kernel", [("f64", "generic"), ("f32", "compact"), ("f16", "fused")])
def test_nonfinite_value_reports_unstable(L, orc, prec, kernel):
    # A NaN written through lbcg_set_state into one population of one node:
    # lbcg_diagnostics returns LBCG_E_UNSTABLE with that node counted, the
    # other sums agree with the oracle's on the same state, and one more
    # step carries the NaN to the node's neighbours.
    w = W.static_droplet_3d(n=20, R=6.0, tau=(1.1, 0.9), A=0.01)
    kind = {"generic": L.KERNEL_GENERIC, "compact": L.KERNEL_COMPACT, "fused": L.KERNEL_FUSED}[kernel]
    s = L.Sim.from_workload(w, precision=prec, kernel=kind)
    s.step(5)
    assert s.diagnostics()["status"] == L.OK
    blob = bytearray(s.get_state())
    elem = {"f64": 8, "f32": 4, "f16": 2}[prec]
    N, i, node = w.nodes, 7, 1234
    off = 64 + (i * N + node) * 2 * elem  # total deviation of direction i at node
    nan = {"f64": np.float64(np.nan), "f32": np.float32(np.nan), "f16": np.float16(np.nan)}[prec]
    blob[off:off + elem] = nan.tobytes()
    s.set_state(bytes(blob))
    d = s.diagnostics()
    _say(f"  {prec} {kernel}: status {d['status']} nonfinite {d['nonfinite']}")
    assert d["status"] == L.E_UNSTABLE and d["nonfinite"] == 1
    with pytest.raises(L.LbcgError) as e:
        s.diagnostics(check=True)
    assert e.value.status == L.E_UNSTABLE
    o = orc.Oracle(oracle_params(orc, w)).set_populations(s.populations())
    od = o.diagnostics()
    assert od["nonfinite"] == 1
    assert _rel(d["mass_R"], od["mass"][0]) < 1e-12 and _rel(d["mass_B"], od["mass"][1]) < 1e-12
    s.step(1)
    d = s.diagnostics()
    assert d["status"] == L.E_UNSTABLE and d["nonfinite"] > 1
