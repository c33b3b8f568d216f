"""Plane Poiseuille flow through a D3Q19 channel on the GPU (FP32, one
colour): a plug velocity inlet at x = 0, a pressure outlet at x = nx - 1 and
half-way bounce-back walls at y = 0 and y = H + 1, periodic in z.  At steady
state the mid-channel profile is the parabola 6 ubar (y + 1/2)(H - 1/2 - y) /
H^2 of half-way walls, and the flux through a cross-section is what the inlet
injects: through its five links with c_x = 1, each inlet node injects
6 u_b (w_axis + 4 w_diag) = u_b, and the two rows beside the walls lose one
diagonal link each (u_b / 6), so u_b (H - 1/3) per z plane.  Checked on the
column sweep, the split step (a lattice at most half fluid: the same channel
with a thick wall region) and the compact state's split step, each also
against the FP64 oracle's steady state."""
import numpy as np
import pytest

from paper_1711_02003_amd import workloads as W
from tests.helpers import oracle_for, rel_l2

pytestmark = pytest.mark.gpu

H, LX, NZ, UB, STEPS = 16, 128, 4, 0.005, 12000


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


def _channel(ny):
    # fluid rows y = 1..H; walls at y = 0 and from y = H + 1 to ny - 1
    mask = np.ones((NZ, ny, LX), np.uint8)
    mask[:, 1:H + 1, :] = 0
    mask[:, 1:H + 1, 0] = 2
    mask[:, 1:H + 1, -1] = 128
    sh = mask.shape
    return W.Workload("poiseuille", "D3Q19", (LX, ny, NZ), np.ones(sh), np.zeros(sh), None, 1.0, 1.0, 0.0, 0.7,
                      mask, [{"u": (UB, 0.0, 0.0), "rho_R": 1.0, "rho_B": 0.0}], [{"rho": 1.0}])


def _profile_and_flux(f):
    y = np.arange(H)
    u = f["u"][0, 1, 1:H + 1, LX // 2]
    ex = 6 * u.mean() * (y + 0.5) * (H - 0.5 - y) / H ** 2
    rho = (f["rhoR"] + f["rhoB"])[1, 1:H + 1, LX // 2]
    return float(np.linalg.norm(u - ex) / np.linalg.norm(ex)), float((rho * u).sum() / (UB * (H - 1 / 3)) - 1)


@pytest.fixture(scope="module")
def steady(orc):
    f = oracle_for(orc, _channel(H + 2), threads=16).step(STEPS).fields()
    prof, flux = _profile_and_flux(f)
    _say(f"oracle Poiseuille: profile {prof:.2e}, flux {flux:+.2e}")
    return f


@pytest.mark.parametrize("form", ["sweep", "split", "compact"])
def test_poiseuille_f32(L, steady, form):
    ny = 2 * H + 8 if form == "split" else H + 2
    w = _channel(ny)
    kernel = L.KERNEL_COMPACT if form == "compact" else L.KERNEL_FUSED
    s = L.Sim.from_workload(w, precision="f32", kernel=kernel)
    assert s.launch_info()["rows"] == (8 if form == "sweep" else 0)
    s.step(STEPS)
    f = s.fields()
    d = s.diagnostics()
    s.close()
    prof, flux = _profile_and_flux(f)
    eu = rel_l2(f["u"][:, :, 1:H + 1], steady["u"][:, :, 1:H + 1])
    _say(f"Poiseuille {form} (ny {ny}): profile {prof:.2e}, flux {flux:+.2e}, relL2 u vs oracle {eu:.2e}")
    assert prof < 0.01 and abs(flux) < 0.002
    assert eu < 1e-5
    assert d["status"] == 0 and d["step"] == STEPS
