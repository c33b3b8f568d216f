"""Brute force on tiny lattices: the C oracle against the independent
per-equation NumPy version (oracle/literal.py), with and without walls
(neutral and wetting), inlets and outlets; regularized, plain BGK at the
node's rate and Eq. (5) with a rate per colour."""
import numpy as np
import pytest

from oracle import literal as L


def _geometry(orc, lat, sh):
    mask = np.zeros(sh, np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    mask[:, 1:-1, 0] = 2
    mask[:, 1:-1, -1] = 128
    if lat == "D3Q19":
        mask[0, :, :] = 1
        mask[-1, 2, 3] = 1  # an isolated obstacle node
        mask[0, 1:3, 1:4] = orc.WALL0 + 1  # a wetting patch in the z = 0 wall
    else:
        mask[0, 0, 2:5] = orc.WALL0  # wetting patches in the y = 0 wall
        mask[0, -1, 3] = orc.WALL0 + 1
    inlets = [orc.Inlet(u=(0.01, 0.002, 0.001 if lat == "D3Q19" else 0.0), rho_w=(0.8, 0.2))]
    outlets = [orc.Outlet(rho=1.02)]
    walls = [orc.Wall(psi=0.6), orc.Wall(psi=-0.8)]
    return mask, inlets, outlets, walls


@pytest.mark.parametrize("lat,dims", [("D2Q9", (8, 8, 1)), ("D3Q19", (6, 5, 4))])
@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("coll", ["reg", "bgk", "bgk_colour"])
def test_c_oracle_matches_literal(orc, lat, dims, masked, coll):
    rng = np.random.default_rng(sum(map(ord, lat + coll)) + 7 * masked)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    mask, inlets, outlets, walls = _geometry(orc, lat, sh) if masked else (None, [], [], [])
    tau, A, alpha, beta = (1.3, 0.7), (0.01, 0.02), (0.0, 0.0), 0.7
    if coll != "reg":
        alpha = (0.3, 0.5) if lat == "D2Q9" else (0.25, 0.4)
    p = orc.Params(lattice=orc.D2Q9 if lat == "D2Q9" else orc.D3Q19, dims=dims, tau=tau, A=A,
                   alpha=alpha, beta=beta, mask=mask, inlets=inlets, outlets=outlets, walls=walls,
                   collision={"reg": orc.REGULARIZED, "bgk": orc.BGK, "bgk_colour": orc.BGK_COLOUR}[coll])
    rR = rng.uniform(0, 1, sh)
    rB = rng.uniform(0, 1, sh)
    u = rng.uniform(-0.05, 0.05, (3,) + sh)
    if lat == "D2Q9":
        u[2] = 0
    o = orc.Oracle(p).init(rR, rB, u)
    fl = L.init(lat, rR, rB, u, alpha)
    assert np.abs(o.populations() - fl).max() < 1e-16
    fluid = np.ones(sh, bool) if mask is None else mask == 0
    for _ in range(6):
        o.step(1)
        fl = L.step(fl, lat, tau, A, beta, alpha=alpha, mask=mask, inlets=inlets,
                    outlets=outlets, bgk=coll == "bgk", walls=walls, bgk_colour=coll == "bgk_colour")
        d = np.abs((o.populations() - fl)[:, :, fluid]).max()
        assert d < 1e-14, d
