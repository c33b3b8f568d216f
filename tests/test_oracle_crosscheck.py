"""Brute force on tiny lattices: the C oracle against the independent
per-equation NumPy version (oracle/literal.py), with and without walls,
inlets and outlets, regularized and plain BGK."""
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
    inlets = [orc.Inlet(u=(0.01, 0.002, 0.001 if lat == "D3Q19" else 0.0), rho_w=(0.8, 0.2))]
    outlets = [orc.Outlet(rho=1.02)]
    return mask, inlets, outlets


@pytest.mark.parametrize("lat,dims", [("D2Q9", (8, 8, 1)), ("D3Q19", (6, 5, 4))])
@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("bgk", [False, True])
def test_c_oracle_matches_literal(orc, lat, dims, masked, bgk):
    rng = np.random.default_rng(hash((lat, masked, bgk)) % 2 ** 32)
    nx, ny, nz = dims
    sh = (nz, ny, nx)
    mask, inlets, outlets = _geometry(orc, lat, sh) if masked else (None, [], [])
    tau, A, alpha, beta = (1.3, 0.7), (0.01, 0.02), (0.0, 0.0), 0.7
    if bgk:
        alpha = (0.3, 0.5) if lat == "D2Q9" else (0.25, 0.4)
    p = orc.Params(lattice=orc.D2Q9 if lat == "D2Q9" else orc.D3Q19, dims=dims, tau=tau, A=A,
                   alpha=alpha, beta=beta, mask=mask, inlets=inlets, outlets=outlets,
                   collision=orc.BGK if bgk else orc.REGULARIZED)
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
                    outlets=outlets, bgk=bgk)
        d = np.abs((o.populations() - fl)[:, :, fluid]).max()
        assert d < 1e-14, d
