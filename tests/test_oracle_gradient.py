"""Closed-form pins of the oracle's colour gradient (orc_gradient), the
isotropic stencil F = (1/c_s^2) sum_i w_i c_i psi~(x + c_i) of the phase
field psi = (rho^R - rho^B) / rho, and of its boundary substitutions.

Plane wave.  For psi = sin(k.x) at rho = 1,
    F = 3 cos(k.x) sum_i w_i c_i sin(k.c_i)
(the cos(k.c_i) part cancels between c_i and -c_i).  Summing over the
velocity sets by hand:
    D2Q9:  F_x = cos(k.x) sin(k_x) (2 + cos k_y) / 3,
    D3Q19: F_x = cos(k.x) sin(k_x) (1 + cos k_y + cos k_z) / 3,
and the other components by permuting the axes; for a wave along x alone
both give F_x = sin(k) cos(k x).  A wrong weight, sign or direction in the
stencil changes these.

Boundary rules, for a profile psi(x) that depends on x only: an interior
node has F_x = (psi(x+1) - psi(x-1)) / 2 (the c_x = +1 weights sum to 1/6),
and a node at x = 1 next to a plane of non-fluid nodes at x = 0 has
F_x = (psi(2) - psi~) / 2, with psi~ = psi(1) at neutral walls and outlets,
the inlet's (rho_R - rho_B) / (rho_R + rho_B) at inlets, and psi_w at a
wetting wall."""
import numpy as np
import pytest


def _wave_state(orc, lat, dims, k, mask=None, inlets=(), outlets=(), walls=(), psi=None):
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if psi is None:
        psi = np.sin(k[0] * xx + k[1] * yy + k[2] * zz)
    p = orc.Params(lattice=orc.D2Q9 if lat == "D2Q9" else orc.D3Q19, dims=dims, mask=mask,
                   inlets=list(inlets), outlets=list(outlets), walls=list(walls))
    o = orc.Oracle(p).init((1 + psi) / 2, (1 - psi) / 2)
    return o, (xx, yy, zz)


@pytest.mark.parametrize("lat,dims", [("D2Q9", (24, 16, 1)), ("D3Q19", (12, 8, 16))])
@pytest.mark.parametrize("axis_wave", [0, 1, 2, "oblique"])
def test_plane_wave_gradient(orc, lat, dims, axis_wave):
    if lat == "D2Q9" and axis_wave == 2:
        pytest.skip("no z axis in 2-D")
    nx, ny, nz = dims
    k = np.zeros(3)
    if axis_wave == "oblique":
        k[:] = (2 * np.pi * 2 / nx, 2 * np.pi * 1 / ny, 0.0 if lat == "D2Q9" else 2 * np.pi * 3 / nz)
    else:
        k[axis_wave] = 2 * np.pi * 2 / dims[axis_wave]
    o, (xx, yy, zz) = _wave_state(orc, lat, dims, k)
    F = o.gradient()
    c = np.cos(k[0] * xx + k[1] * yy + k[2] * zz)
    s, co = np.sin(k), np.cos(k)
    if lat == "D2Q9":
        expect = [c * s[0] * (2 + co[1]) / 3, c * s[1] * (2 + co[0]) / 3, 0 * c]
    else:
        expect = [c * s[0] * (1 + co[1] + co[2]) / 3, c * s[1] * (1 + co[0] + co[2]) / 3,
                  c * s[2] * (1 + co[0] + co[1]) / 3]
    for a in range(3):
        assert np.abs(F[a] - expect[a]).max() < 1e-14, a
    if axis_wave != "oblique":
        a = axis_wave
        assert np.abs(F[a] - np.sin(k[a]) * c).max() < 1e-14


def _profile(nx):
    # a smooth, non-symmetric profile in x with values inside (-1, 1)
    x = np.arange(nx)
    return 0.6 * np.tanh((x - nx / 3) / 2.5) + 0.1 * np.cos(2 * np.pi * x / nx)


@pytest.mark.parametrize("lat,dims", [("D2Q9", (16, 6, 1)), ("D3Q19", (16, 5, 4))])
@pytest.mark.parametrize("kind", ["wall", "outlet", "inlet", "wetting"])
def test_boundary_substitution(orc, lat, dims, kind):
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    prof = _profile(nx)
    psi = np.broadcast_to(prof, sh).copy()
    mask = np.zeros(sh, np.uint8)
    inlets, outlets, walls = [], [], []
    if kind == "wall":
        mask[..., 0] = 1
        sub = prof[1]
    elif kind == "outlet":
        mask[..., 0] = orc.OUTLET0
        outlets = [orc.Outlet(rho=1.0)]
        sub = prof[1]
    elif kind == "inlet":
        mask[..., 0] = orc.INLET0
        inlets = [orc.Inlet(u=(0.01, 0, 0), rho_w=(0.8, 0.2))]
        sub = 0.6
    else:
        mask[..., 0] = orc.WALL0 + 1
        walls = [orc.Wall(psi=0.9), orc.Wall(psi=-0.4)]
        sub = -0.4
    o, _ = _wave_state(orc, lat, dims, None, mask=mask, inlets=inlets, outlets=outlets, walls=walls,
                       psi=psi)
    F = o.gradient()
    Fx = F[0][0, 0]
    assert Fx[0] == 0.0  # non-fluid nodes report no gradient
    assert Fx[1] == pytest.approx((prof[2] - sub) / 2, abs=1e-15)
    for x in range(2, nx - 1):
        assert Fx[x] == pytest.approx((prof[x + 1] - prof[x - 1]) / 2, abs=1e-15)
    # x = nx - 1: its +x neighbour wraps to the boundary plane at x = 0
    assert Fx[nx - 1] == pytest.approx((sub if kind in ("inlet", "wetting") else prof[nx - 1])
                                       / 2 - prof[nx - 2] / 2, abs=1e-15)
    assert np.abs(F[1]).max() < 1e-15 and np.abs(F[2]).max() < 1e-15
    # every row and plane alike
    assert np.abs(F[0] - F[0][:1, :1]).max() == 0.0
