"""Per-equation NumPy version of the RCG step, for tiny lattices only.

Test infrastructure (cross-check of the C oracle).  Written independently of
``rcg_oracle.c``: the lattice tables are typed in from their definitions, the
non-equilibrium momentum flux is summed explicitly as sum_i (f_i - f_i^eq)
c_i c_i rather than from a closed form, the perturbation is added to each
colour separately exactly as Eq. (9) is written, streaming is done in pull
form with ``np.roll``, and boundary links are handled by explicit loops.

Populations have shape (2, Q, nz, ny, nx); arXiv:1711.02003 Sec. II.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0


def d2q9():
    # Eq. (7) numbering, started at zero: rest, then axis/diagonal alternating.
    c = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [-1, 1, 0],
                  [-1, 0, 0], [-1, -1, 0], [0, -1, 0], [1, -1, 0]])
    w = np.array([4 / 9] + [1 / 9, 1 / 36] * 4)
    # Perturbation constants of the D2Q9 colour-gradient model.
    Bf = [Fraction(-4, 27)] + [Fraction(2, 27), Fraction(5, 108)] * 4
    return c, w, np.array([float(b) for b in Bf]), 2


def d3q19():
    c = [[0, 0, 0]]
    for a in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[a] = s
            c.append(v)
    for a in range(3):
        for b in range(a + 1, 3):
            for sa in (1, -1):
                for sb in (1, -1):
                    v = [0, 0, 0]
                    v[a], v[b] = sa, sb
                    c.append(v)
    c = np.array(c)
    n2 = (c * c).sum(1)
    w = np.where(n2 == 0, 1 / 3, np.where(n2 == 1, 1 / 18, 1 / 36))
    B = np.where(n2 == 0, -2 / 9, np.where(n2 == 1, 1 / 54, 1 / 27))
    return c, w, B, 3


def tables(lattice: str):
    return d2q9() if lattice == "D2Q9" else d3q19()


def phi(lattice: str, alpha: float):
    """Eq. (7) (and its D3Q19 counterpart: moving share proportional to w_i)."""
    c, w, _, _ = tables(lattice)
    n2 = (c * c).sum(1)
    if lattice == "D2Q9":
        return np.where(n2 == 0, alpha, np.where(n2 == 1, (1 - alpha) / 5, (1 - alpha) / 20))
    return np.where(n2 == 0, alpha, np.where(n2 == 1, (1 - alpha) / 12, (1 - alpha) / 24))


def equilibrium(lattice, rho_k, alpha_k, u):
    """Eq. (6): rho^k [phi_i^k + w_i (c.u/cs2 + (c.u)^2/(2 cs4) - u^2/(2 cs2))]."""
    c, w, _, _ = tables(lattice)
    ph = phi(lattice, alpha_k)
    cu = np.einsum("ia,a...->i...", c.astype(float), u)
    uu = (u * u).sum(0)
    shp = (-1,) + (1,) * rho_k.ndim
    return rho_k[None] * (ph.reshape(shp) + w.reshape(shp) * (cu / CS2 + cu ** 2 / (2 * CS2 ** 2)
                                                             - uu[None] / (2 * CS2)))


def _opp(c):
    return np.array([int(np.where((c == -ci).all(1))[0][0]) for ci in c])


def step(f, lattice, tau, A, beta, alpha=(0.0, 0.0), eps_F=1e-8, mask=None, inlets=(),
         outlets=(), bgk=False, walls=(), bgk_colour=False):
    """One time step.  f: (2, Q, nz, ny, nx) pre-collision; returns the next one.

    Mask codes: 1 neutral wall, 2 + j inlet j, 64 + j wetting wall j (its
    phase value walls[j].psi enters the gradient), 128 + j outlet j.
    bgk: Eq. (5) at the node's rate; bgk_colour: Eq. (5) with each colour at
    its own rate 1/tau_k."""
    c, w, B, D = tables(lattice)
    Q = len(w)
    alpha = [a if a > 0 else w[0] for a in alpha]
    sh = f.shape[2:]
    fluid = np.ones(sh, bool) if mask is None else (mask == 0)
    cf = c.astype(float)

    # Eq. (2), Eq. (3)
    rho_k = f.sum(1)
    rho = rho_k.sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.einsum("kiz...,ia->az...", f, cf) / rho
        psi = (rho_k[0] - rho_k[1]) / rho
    u = np.where(fluid[None], u, 0.0)
    psi = np.where(fluid, psi, 0.0)

    # colour gradient with neighbour substitution at non-fluid nodes
    F = np.zeros((3,) + sh)
    m = np.zeros(sh, np.int64) if mask is None else mask.astype(np.int64)
    for i in range(1, Q):
        shift = (-c[i, 2], -c[i, 1], -c[i, 0])  # value at x + c_i
        pn = np.roll(psi, shift, axis=(0, 1, 2))
        mn = np.roll(m, shift, axis=(0, 1, 2))
        ps = np.where(mn == 0, pn, psi)
        for j, inl in enumerate(inlets):
            rw = inl.rho_w
            ps = np.where(mn == 2 + j, (rw[0] - rw[1]) / (rw[0] + rw[1]), ps)
        for j, wl in enumerate(walls):
            ps = np.where(mn == 64 + j, wl.psi, ps)
        F += (w[i] / CS2) * cf[i][:, None, None, None] * ps[None]
    F = np.where(fluid[None], F, 0.0)
    Fn = np.sqrt((F * F).sum(0))
    hasF = Fn > eps_F

    # each colour relaxed at the node's rate (the mixture viscosity is the
    # colour-fraction-weighted harmonic mean of the component viscosities),
    # then the perturbation added to each colour
    with np.errstate(invalid="ignore", divide="ignore"):
        nu = 1.0 / sum((rho_k[k] / rho) / (CS2 * (tau[k] - 0.5)) for k in range(2))
        om = np.where(fluid, 1.0 / (nu / CS2 + 0.5), 0.0)
    f2k = np.zeros_like(f)
    Qt = np.einsum("ia,ib->iab", cf, cf) - CS2 * np.eye(3)[None]
    Fc = np.einsum("ia,a...->i...", cf, F)
    with np.errstate(invalid="ignore", divide="ignore"):
        pert = np.where(hasF[None], Fn[None] * (w.reshape(-1, 1, 1, 1) * Fc ** 2 / (Fn[None] ** 2)
                                                - B.reshape(-1, 1, 1, 1)), 0.0)
    for k in range(2):
        fe = equilibrium(lattice, rho_k[k], alpha[k], u)
        if bgk_colour:
            f1 = f[k] - (f[k] - fe) / tau[k]
        elif bgk:
            f1 = f[k] - om * (f[k] - fe)
        else:
            Pneq = np.einsum("i...,ia,ib->ab...", f[k] - fe, cf, cf)
            H = np.einsum("iab,ab...->i...", Qt, Pneq) * (w / (2 * CS2 ** 2)).reshape(-1, 1, 1, 1)
            f1 = fe + (1 - om) * H
        f2k[k] = f1 + 0.5 * A[k] * pert

    # Eq. (10) recolouring of the total
    ftot = f2k.sum(0)
    cn = np.sqrt((c * c).sum(1)).astype(float)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosp = np.where(hasF[None] & (cn.reshape(-1, 1, 1, 1) > 0),
                        Fc / (Fn[None] * np.where(cn > 0, cn, 1).reshape(-1, 1, 1, 1)), 0.0)
    zero = np.zeros((3,) + sh)
    e0 = equilibrium(lattice, rho_k[0], alpha[0], zero) + equilibrium(lattice, rho_k[1], alpha[1], zero)
    with np.errstate(invalid="ignore", divide="ignore"):
        seg = beta * rho_k[0] * rho_k[1] / rho ** 2
        post = np.stack([rho_k[0] / rho * ftot + seg * cosp * e0,
                         rho_k[1] / rho * ftot - seg * cosp * e0])
    post = np.where(fluid[None, None], post, 0.0)

    # Eq. (1) streaming, pull form; boundary links by explicit loops
    new = np.zeros_like(f)
    for i in range(Q):
        new[:, i] = np.roll(post[:, i], (c[i, 2], c[i, 1], c[i, 0]), axis=(1, 2, 3))
    if mask is not None:
        opp = _opp(c)
        nz, ny, nx = sh
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if mask[z, y, x] != 0:
                        continue
                    for i in range(Q):
                        uz, uy, ux = (z - c[i, 2]) % nz, (y - c[i, 1]) % ny, (x - c[i, 0]) % nx
                        code = int(mask[uz, uy, ux])
                        if code == 0:
                            continue
                        io = opp[i]
                        if code == 1 or 64 <= code < 128:
                            new[:, i, z, y, x] = post[:, io, z, y, x]
                        elif code < 64:
                            inl = inlets[code - 2]
                            cu = float(np.dot(c[io], inl.u))
                            for k in range(2):
                                new[k, i, z, y, x] = post[k, io, z, y, x] - 2 * w[io] * inl.rho_w[k] * cu / CS2
                        else:
                            # anti-bounce-back pressure outlet, moments of the
                            # node's own post-collision populations
                            rho_out = outlets[code - 128].rho
                            pk = post[:, :, z, y, x]
                            rk = pk.sum(1)
                            uP = (pk.sum(0)[:, None] * cf).sum(0) / rk.sum()
                            ph = [phi(lattice, alpha[0]), phi(lattice, alpha[1])]
                            cu = float(np.dot(c[io], uP))
                            uu = float(np.dot(uP, uP))
                            for k in range(2):
                                rw = rho_out * rk[k] / rk.sum()
                                even = rw * (ph[k][io] + w[io] * (cu * cu / (2 * CS2 ** 2) - uu / (2 * CS2)))
                                new[k, i, z, y, x] = -post[k, io, z, y, x] + 2 * even
        new = np.where(fluid[None, None], new, 0.0)
    return new


def init(lattice, rhoR, rhoB, u=None, alpha=(0.0, 0.0)):
    c, w, _, _ = tables(lattice)
    alpha = [a if a > 0 else w[0] for a in alpha]
    if u is None:
        u = np.zeros((3,) + rhoR.shape)
    return np.stack([equilibrium(lattice, rhoR, alpha[0], u), equilibrium(lattice, rhoB, alpha[1], u)])
