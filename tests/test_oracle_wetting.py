"""Pins of the oracle's wetting walls (mask codes 64 + j): half-way
bounce-back like a neutral wall, with the colour gradient seeing the wall's
own phase value psi_w instead of the fluid node's psi.

The paper states no wall rule; these pins fix the reading from what any
wetting rule of this kind must satisfy: a wall whose psi_w equals the phase
of the fluid beside it acts exactly as a neutral wall; swapping the colours
and the sign of psi_w mirrors the whole evolution; a positive psi_w makes
the red colour wet the wall (contact angle inside red below 90 degrees), a
negative one makes it dewet, and the neutral wall holds a droplet near 90
degrees."""
import numpy as np
import pytest


def _sessile(orc, psi_w, nx=96, ny=40, R=14.0, neutral=False, swap=False, tau=(1.0, 1.0)):
    # red half-disc on the wall row y = 0 (half-way wall plane at y = 0.5),
    # walls at y = 0 and y = ny - 1, periodic in x
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.sqrt((xx - (nx - 1) / 2) ** 2 + (yy - 0.5) ** 2)
    psi = np.tanh((R - r) / 2)
    if swap:
        psi = -psi
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 0, :] = 1 if neutral else orc.WALL0 + 1
    mask[0, -1, :] = 1 if neutral else orc.WALL0 + 1
    p = orc.Params(lattice=orc.D2Q9, dims=(nx, ny, 1), tau=tau, A=(0.01, 0.01), beta=0.7, mask=mask,
                   walls=[orc.Wall(psi=0.3), orc.Wall(psi=psi_w)], threads=8)
    return orc.Oracle(p).init(((1 + psi) / 2)[None], ((1 - psi) / 2)[None])


def _contact_angle(o, nx, ny):
    # circular cap: half base b on the first fluid row and height h on the
    # centre line give theta = 2 atan(h / b) (90 degrees for h = b)
    ps = o.fields()["psi"][0]
    c = nx // 2
    col = (ps[1:-1, c - 1] + ps[1:-1, c]) / 2
    h = np.interp(0.0, -col, np.arange(1, ny - 1)) - 0.5
    b = np.interp(0.0, -ps[1, c:], np.arange(c, nx)) - (nx - 1) / 2
    return 2 * np.degrees(np.arctan(h / b))


def test_contact_angle_follows_psi_w(orc):
    th = {}
    mass = {}
    for key, kw in (("neutral", dict(psi_w=0.0, neutral=True)), ("+0.5", dict(psi_w=0.5)),
                    ("-0.5", dict(psi_w=-0.5))):
        o = _sessile(orc, **kw)
        m0 = o.diagnostics()["mass"]
        o.step(4000)
        mass[key] = (m0, o.diagnostics()["mass"])
        th[key] = _contact_angle(o, 96, 40)
    assert abs(th["neutral"] - 90.0) < 3.0
    assert th["+0.5"] < 80.0 < 100.0 < th["-0.5"]
    for m0, m1 in mass.values():  # walls of either kind keep each colour's mass
        assert abs(m1[0] / m0[0] - 1) < 1e-12 and abs(m1[1] / m0[1] - 1) < 1e-12


def test_colour_swap_mirrors_psi_w(orc):
    # tau_R = tau_B, A_R = A_B, alpha_R = alpha_B: exchanging the colours of
    # the initial state and the sign of every psi_w exchanges the colours of
    # the result (to round-off).
    for psi_w in (0.7, -0.4):
        a = _sessile(orc, psi_w, tau=(0.8, 0.8)).step(200)
        b = _sessile(orc, -psi_w, tau=(0.8, 0.8), swap=True)
        b.p.walls[0].psi = -0.3
        b = type(b)(b.p)
        yy, xx = np.mgrid[0:40, 0:96]
        r = np.sqrt((xx - 47.5) ** 2 + (yy - 0.5) ** 2)
        psi = -np.tanh((14.0 - r) / 2)
        b.init(((1 + psi) / 2)[None], ((1 - psi) / 2)[None]).step(200)
        fa, fb = a.populations(), b.populations()
        assert np.abs(fa[0] - fb[1]).max() < 1e-13
        assert np.abs(fa[1] - fb[0]).max() < 1e-13
        # and a different psi_w does change the result
        assert np.abs(fa[0] - _sessile(orc, 0.0, tau=(0.8, 0.8)).step(200).populations()[0]).max() > 1e-6


def test_wall_at_the_fluid_phase_is_neutral(orc):
    # A blue droplet far from the walls in red fluid: every fluid node next
    # to a wall stays exactly pure red (psi = 1) over these steps, so a
    # wetting wall with psi_w = 1 acts bitwise as a neutral wall.  (The
    # initial blue density rounds to exactly 0 from r ~ 46 on, and a nonzero
    # tail moves at most one node per step.)
    nx, ny = 64, 160
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.sqrt((xx - 31.5) ** 2 + (yy - 79.5) ** 2)
    psi = -np.tanh((8.0 - r) / 2)  # blue inside r < 8
    res = []
    for neutral in (True, False):
        mask = np.zeros((1, ny, nx), np.uint8)
        mask[0, 0, :] = mask[0, -1, :] = 1 if neutral else orc.WALL0
        p = orc.Params(lattice=orc.D2Q9, dims=(nx, ny, 1), tau=(1.2, 0.7), A=(0.01, 0.01), beta=0.7,
                       mask=mask, walls=[orc.Wall(psi=1.0)])
        o = orc.Oracle(p).init(((1 + psi) / 2)[None], ((1 - psi) / 2)[None])
        assert np.all(o.fields()["psi"][0][[1, -2], :] == 1.0)
        o.step(12)
        assert np.all(o.fields()["psi"][0][[1, -2], :] == 1.0)
        res.append(o.populations())
    assert np.array_equal(res[0], res[1])
