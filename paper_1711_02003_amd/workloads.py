"""Seeded synthetic inputs for the regularized colour-gradient LB step.

This module only draws initial fields, geometry masks and parameter sets; it
holds none of the method's arithmetic, so the GPU library, the oracle and the
tests can all consume the same arrays.  Every generator uses NumPy's PCG64
(``numpy.random.default_rng(seed)``) and documents its draw order.

The paper's own inputs (its flow-focusing and volcano geometries, flow rates
and surface tensions) are not published in usable form, so these shapes stand
in for them: static droplets for the Laplace and conservation checks, a
27-droplet periodic box for throughput, a flow-focusing cross junction shaped
after the paper's Fig. 2 device, and step-emulsifier channels opening onto a
deep reservoir shaped after its Fig. 5 ("volcano") device.

Conventions: scalar fields (nz, ny, nx) float64, x fastest; velocity
(3, nz, ny, nx); masks uint8 (nz, ny, nx) with 0 fluid, 1 wall, 2 + j inlet j,
128 + j outlet j.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

FLUID, WALL, INLET0, OUTLET0 = 0, 1, 2, 128


@dataclass
class Workload:
    """Initial fields + geometry + model parameters of one lattice."""
    name: str
    lattice: str                         # "D2Q9" or "D3Q19"
    dims: tuple                          # (nx, ny, nz)
    rhoR: np.ndarray
    rhoB: np.ndarray
    u: Optional[np.ndarray]
    tau_R: float = 1.0
    tau_B: float = 1.0
    A: float = 0.01
    beta: float = 0.7
    mask: Optional[np.ndarray] = None
    inlets: List[dict] = field(default_factory=list)   # {"u": (3,), "rho_R":, "rho_B":}
    outlets: List[dict] = field(default_factory=list)  # {"rho": outlet density}
    steps: int = 1000
    walls: List[dict] = field(default_factory=list)    # {"psi": phase value of wetting wall j}

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    @property
    def nodes(self) -> int:
        return int(np.prod(self.dims))

    @property
    def fluid_nodes(self) -> int:
        return self.nodes if self.mask is None else int((self.mask == FLUID).sum())


def tanh_profile(dist_inside: np.ndarray, width: float = 2.0) -> np.ndarray:
    """Initial phase profile tanh(d / width), d > 0 inside the droplet."""
    return np.tanh(dist_inside / width)


def _min_image(d: np.ndarray, n: int) -> np.ndarray:
    return d - n * np.round(d / n)


def droplet_phase(dims, centres, radii, width=2.0) -> np.ndarray:
    """psi0 = max over droplets of tanh((R_d - r_d)/width), periodic minimum-image r.

    Beyond r = R + 40 the double-precision tanh is exactly -1, so each droplet
    is evaluated only in its bounding box of that reach.
    """
    nx, ny, nz = dims
    psi = np.full((nz, ny, nx), -1.0)
    reach = 40.0
    for c, R in zip(centres, radii):
        sl = []
        coords = []
        for a, n in enumerate((nx, ny, nz)):
            lo = int(np.floor(c[a] - R - reach))
            hi = int(np.ceil(c[a] + R + reach)) + 1
            if hi - lo >= n:
                idx = np.arange(n)
            else:
                idx = np.arange(lo, hi) % n
            coords.append(idx)
        ix, iy, iz = coords
        dx = _min_image(ix - c[0], nx)
        dy = _min_image(iy - c[1], ny)
        dz = _min_image(iz - c[2], nz) if nz > 1 else np.zeros(1)
        r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = tanh_profile(R - r, width)
        sub = psi[np.ix_(iz, iy, ix)]
        psi[np.ix_(iz, iy, ix)] = np.maximum(sub, val)
    return psi


def colour_densities(psi: np.ndarray):
    """rho_R = (1 + psi)/2, rho_B = (1 - psi)/2 (total density 1)."""
    return 0.5 * (1.0 + psi), 0.5 * (1.0 - psi)


def static_droplet_2d(n: int = 64, R: float = 16.0, width: float = 2.0, noise: float = 1e-6,
                      seed: int = 1, centre=None, tau=(1.0, 1.0), A: float = 0.01,
                      beta: float = 0.7, steps: int = 2000) -> Workload:
    """D2Q9 disc of radius R at the box centre ((n-1)/2, (n-1)/2), periodic.

    Draws: rho_R noise U(-noise, noise) per node, then rho_B noise likewise.
    """
    c = ((n - 1) / 2.0, (n - 1) / 2.0, 0.0) if centre is None else centre
    psi = droplet_phase((n, n, 1), [c], [R], width)
    rR, rB = colour_densities(psi)
    if noise > 0:
        rng = np.random.default_rng(seed)
        rR = rR + rng.uniform(-noise, noise, rR.shape)
        rB = rB + rng.uniform(-noise, noise, rB.shape)
    return Workload("static_droplet_2d", "D2Q9", (n, n, 1), rR, rB, None, tau[0], tau[1], A,
                    beta, steps=steps)


def droplet_2d_64(seed: int = 1) -> Workload:
    """D2Q9 static droplet 64x64 periodic, R = 16, tanh width 2, +-1e-6 noise,
    tau_R = tau_B = 1, A = 0.01, beta = 0.7, 2000 steps."""
    w = static_droplet_2d(64, 16.0, 2.0, 1e-6, seed)
    w.name = "d2q9_static_droplet_64"
    return w


def static_droplet_3d(n: int = 64, R: float = 16.0, width: float = 2.0, tau=(1.0, 1.0),
                      A: float = 0.005, beta: float = 0.7, steps: int = 1000) -> Workload:
    """D3Q19 sphere of radius R at the box centre, periodic, at rest, no noise."""
    c = ((n - 1) / 2.0,) * 3
    psi = droplet_phase((n, n, n), [c], [R], width)
    rR, rB = colour_densities(psi)
    return Workload("static_droplet_3d", "D3Q19", (n, n, n), rR, rB, None, tau[0], tau[1], A,
                    beta, steps=steps)


def droplets_27(L: int = 256, seed: int = 2, steps: int = 1000) -> Workload:
    """D3Q19 periodic box with 27 droplets on a jittered 3x3x3 lattice.

    At L = 256: centres (i + 1/2) L/3 + U(-8, 8) per axis, radii U[12, 24];
    other L scale the jitter and radii by L/256.  Velocity N(0, 1e-3) per
    component per node.  tau_R = 1.0, tau_B = 0.6, A = 0.005, beta = 0.7.
    Draws: 81 jitters (droplet-major, x y z), 27 radii, then u (3, nz, ny, nx).
    """
    rng = np.random.default_rng(seed)
    s = L / 256.0
    jit = rng.uniform(-8.0 * s, 8.0 * s, (27, 3))
    radii = rng.uniform(12.0 * s, 24.0 * s, 27)
    centres = []
    d = 0
    for k in range(3):
        for j in range(3):
            for i in range(3):
                base = np.array([(i + 0.5) * L / 3.0, (j + 0.5) * L / 3.0, (k + 0.5) * L / 3.0])
                centres.append(base + jit[d])
                d += 1
    psi = droplet_phase((L, L, L), centres, radii, 2.0)
    rR, rB = colour_densities(psi)
    u = rng.normal(0.0, 1e-3, (3, L, L, L))
    return Workload(f"d3q19_27_droplets_{L}", "D3Q19", (L, L, L), rR, rB, u, 1.0, 0.6, 0.005, 0.7,
                    steps=steps)


def droplets_2d(n: int = 4096, seed: int = 6, steps: int = 1000) -> Workload:
    """D2Q9 periodic square with 256 droplets on a jittered 16 x 16 lattice
    (the 2-D counterpart of droplets_27).

    At n = 4096: centres (i + 1/2) n/16 + U(-32, 32) per axis, radii
    U[24, 56]; other n scale the jitter and radii by n/4096.  Velocity
    N(0, 1e-3) per in-plane component per node.  tau_R = 1.0, tau_B = 0.6,
    A = 0.005, beta = 0.7.  Draws: 512 jitters (droplet-major, x y), 256
    radii, then u (2, 1, n, n).
    """
    rng = np.random.default_rng(seed)
    s = n / 4096.0
    jit = rng.uniform(-32.0 * s, 32.0 * s, (256, 2))
    radii = rng.uniform(24.0 * s, 56.0 * s, 256)
    centres = []
    d = 0
    for j in range(16):
        for i in range(16):
            centres.append(((i + 0.5) * n / 16.0 + jit[d, 0], (j + 0.5) * n / 16.0 + jit[d, 1], 0.0))
            d += 1
    psi = droplet_phase((n, n, 1), centres, radii, 2.0)
    rR, rB = colour_densities(psi)
    u = np.zeros((3, 1, n, n))
    u[:2] = rng.normal(0.0, 1e-3, (2, 1, n, n))
    return Workload(f"d2q9_256_droplets_{n}", "D2Q9", (n, n, 1), rR, rB, u, 1.0, 0.6, 0.005, 0.7,
                    steps=steps)


def flow_focusing(nx: int = 512, ny: int = 128, nz: int = 64, lam: float = 1.0,
                  u_disp: float = 0.005, u_side: float = 0.01, A: float = 0.01,
                  steps: int = 20000) -> Workload:
    """Flow-focusing cross junction (after the paper's Fig. 2 device).

    Walls at z = 0 and z = nz-1.  Dispersed (red) channel x in [1, nx/4),
    y in [3ny/8, 5ny/8) fed at x = 0 by inlet 0 (u = (u_disp, 0, 0), red).
    Two side channels x in [nx/4, nx/4 + ny/4) fed at y = 0 and y = ny-1 by
    inlets 1 and 2 (u = (0, +-u_side, 0), blue).  Main channel from x = nx/4
    to the outlet plane x = nx-1 (outlet 0, density 1).  Everything else wall.
    tau_B = 1, tau_R = 1/2 + lam/2 (viscosity ratio lam).
    """
    mask = np.full((nz, ny, nx), WALL, np.uint8)
    y0, y1 = 3 * ny // 8, 5 * ny // 8
    xj0, xj1 = nx // 4, nx // 4 + ny // 4
    zs = slice(1, nz - 1)
    mask[zs, y0:y1, 1:nx - 1] = FLUID
    mask[zs, 1:ny - 1, xj0:xj1] = FLUID
    mask[zs, y0:y1, 0] = INLET0 + 0
    mask[zs, 0, xj0:xj1] = INLET0 + 1
    mask[zs, ny - 1, xj0:xj1] = INLET0 + 2
    mask[zs, y0:y1, nx - 1] = OUTLET0 + 0
    x = np.arange(nx)[None, None, :]
    psi = np.broadcast_to(tanh_profile(xj0 - 0.5 - x, 2.0), (nz, ny, nx)).copy()
    psi[:, :y0, :] = -1.0
    psi[:, y1:, :] = -1.0
    psi[mask != FLUID] = -1.0
    rR, rB = colour_densities(psi)
    inlets = [{"u": (u_disp, 0.0, 0.0), "rho_R": 1.0, "rho_B": 0.0},
              {"u": (0.0, u_side, 0.0), "rho_R": 0.0, "rho_B": 1.0},
              {"u": (0.0, -u_side, 0.0), "rho_R": 0.0, "rho_B": 1.0}]
    outlets = [{"rho": 1.0}]
    return Workload(f"d3q19_flow_focusing_{nx}x{ny}x{nz}", "D3Q19", (nx, ny, nz), rR, rB, None,
                    0.5 + lam / 2.0, 1.0, A, 0.7, mask, inlets, outlets, steps)


def flow_focusing_2d(nx: int = 2048, ny: int = 512, lam: float = 3.0, u_disp: float = 0.005,
                     u_side: float = 0.01, A: float = 0.01, steps: int = 20000) -> Workload:
    """D2Q9 flow-focusing cross junction (the paper's 2-D device geometry,
    after its Fig. 2): the D3Q19 junction's cross-section.

    Dispersed (red) channel y in [3ny/8, 5ny/8) from x = 1, fed at x = 0 by
    inlet 0 (u = (u_disp, 0), red).  Two side channels x in [nx/4, nx/4 +
    ny/4) fed at y = 0 and y = ny-1 by inlets 1 and 2 (u = (0, +-u_side),
    blue).  Main channel from x = nx/4 to the outlet column x = nx-1 (outlet
    0, density 1).  Everything else wall.  tau_B = 1, tau_R = 1/2 + lam/2.
    """
    mask = np.full((1, ny, nx), WALL, np.uint8)
    y0, y1 = 3 * ny // 8, 5 * ny // 8
    xj0, xj1 = nx // 4, nx // 4 + ny // 4
    mask[0, y0:y1, 1:nx - 1] = FLUID
    mask[0, 1:ny - 1, xj0:xj1] = FLUID
    mask[0, y0:y1, 0] = INLET0 + 0
    mask[0, 0, xj0:xj1] = INLET0 + 1
    mask[0, ny - 1, xj0:xj1] = INLET0 + 2
    mask[0, y0:y1, nx - 1] = OUTLET0 + 0
    x = np.arange(nx)[None, None, :]
    psi = np.broadcast_to(tanh_profile(xj0 - 0.5 - x, 2.0), (1, ny, nx)).copy()
    psi[:, :y0, :] = -1.0
    psi[:, y1:, :] = -1.0
    psi[mask != FLUID] = -1.0
    rR, rB = colour_densities(psi)
    inlets = [{"u": (u_disp, 0.0, 0.0), "rho_R": 1.0, "rho_B": 0.0},
              {"u": (0.0, u_side, 0.0), "rho_R": 0.0, "rho_B": 1.0},
              {"u": (0.0, -u_side, 0.0), "rho_R": 0.0, "rho_B": 1.0}]
    outlets = [{"rho": 1.0}]
    return Workload(f"d2q9_flow_focusing_{nx}x{ny}", "D2Q9", (nx, ny, 1), rR, rB, None,
                    0.5 + lam / 2.0, 1.0, A, 0.7, mask, inlets, outlets, steps)


def batch_boxes(n_boxes: int = 64, seed: int = 4, edge_lo: int = 32, edge_hi: int = 96,
                steps: int = 1000) -> List[Workload]:
    """Independent periodic D3Q19 droplet boxes of uneven size.

    Per box (in this order): edges U{edge_lo..edge_hi} (x, y, z); droplet count
    U{1..8}; for each droplet, rejection-sampled centre (uniform in the box) and
    radius U[4, 0.2 min edge] until it is at least 6 nodes clear of the others
    (at most 200 tries, then the droplet is dropped); tau_R, tau_B
    U[0.55, 1.2]; A U[0.001, 0.01]; u N(0, 1e-3).  beta = 0.7.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_boxes):
        dims = tuple(int(v) for v in rng.integers(edge_lo, edge_hi + 1, 3))
        nd = int(rng.integers(1, 9))
        rmax = max(4.0, 0.2 * min(dims))
        centres, radii = [], []
        for _ in range(nd):
            for _try in range(200):
                c = rng.uniform(0, 1, 3) * np.array(dims)
                R = rng.uniform(4.0, rmax)
                ok = True
                for c2, R2 in zip(centres, radii):
                    d = _min_image(c - c2, np.array(dims))
                    if np.sqrt((d * d).sum()) < R + R2 + 6.0:
                        ok = False
                        break
                if ok:
                    centres.append(c)
                    radii.append(R)
                    break
        tR, tB = rng.uniform(0.55, 1.2, 2)
        A = rng.uniform(0.001, 0.01)
        psi = droplet_phase(dims, centres, radii, 2.0)
        rR, rB = colour_densities(psi)
        nx, ny, nz = dims
        u = rng.normal(0.0, 1e-3, (3, nz, ny, nx))
        out.append(Workload(f"box{b}_{nx}x{ny}x{nz}", "D3Q19", dims, rR, rB, u, float(tR),
                            float(tB), float(A), 0.7, steps=steps))
    return out


def step_emulsifier(Lc: int, W: int, H: int, k: int, u_in: float, steps: int,
                    A: float = 0.01, tau: float = 1.0) -> Workload:
    """Shallow channel (length Lc, width W, height H) opening onto a deep
    reservoir (2W long, 2W wide, k*H tall): the paper's Fig. 5 step
    emulsifier ("volcano" nozzle) shape.

    Box: nx = Lc + 2W + 2, ny = 2W + 2, nz = k*H + 2 (one wall layer around).
    The channel is centred in y and sits on the reservoir floor.  Inlet 0 at
    x = 0 (red, u = (u_in, 0, 0)); outlet 0 on the reservoir's far face
    x = nx-1 (density 1).  The channel starts filled with red, the reservoir
    with blue.
    """
    nx, ny, nz = Lc + 2 * W + 2, 2 * W + 2, k * H + 2
    mask = np.full((nz, ny, nx), WALL, np.uint8)
    cy0 = 1 + (2 * W - W) // 2
    mask[1:1 + H, cy0:cy0 + W, 1:1 + Lc] = FLUID
    mask[1:nz - 1, 1:ny - 1, 1 + Lc:nx - 1] = FLUID
    mask[1:1 + H, cy0:cy0 + W, 0] = INLET0
    mask[1:nz - 1, 1:ny - 1, nx - 1] = OUTLET0
    x = np.arange(nx)[None, None, :]
    psi = np.broadcast_to(tanh_profile(Lc + 0.5 - x, 2.0), (nz, ny, nx)).copy()
    psi[mask != FLUID] = -1.0
    rR, rB = colour_densities(psi)
    return Workload(f"d3q19_step_emulsifier_{Lc}x{W}x{H}k{k}", "D3Q19", (nx, ny, nz), rR, rB,
                    None, tau, tau, A, 0.7, mask,
                    [{"u": (u_in, 0.0, 0.0), "rho_R": 1.0, "rho_B": 0.0}],
                    [{"rho": 1.0}], steps)


def served_requests(n: int = 256, seed: int = 5, rate: float = 1.0, steps_lo: int = 5000,
                    steps_hi: int = 20000, scale: float = 1.0) -> List[dict]:
    """Poisson stream of step-emulsifier requests.

    Per request (in this order): exponential inter-arrival gap with mean
    1/rate seconds; Lc U{64..256}, W U{32..64}, H U{8..16}, k U{2..4};
    inlet u U[0.002, 0.01]; steps U{steps_lo..steps_hi}.  ``scale`` shrinks
    the lengths (for tests).  Returns dicts with the arrival time and the
    generator arguments; ``step_emulsifier(**r["args"])`` builds the lattice.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(n):
        t += rng.exponential(1.0 / rate)
        Lc = int(rng.integers(64, 257))
        W = int(rng.integers(32, 65))
        H = int(rng.integers(8, 17))
        k = int(rng.integers(2, 5))
        u_in = float(rng.uniform(0.002, 0.01))
        st = int(rng.integers(steps_lo, steps_hi + 1))
        if scale != 1.0:
            Lc, W, H = max(4, int(Lc * scale)), max(4, int(W * scale)), max(3, int(H * scale))
        out.append({"id": j, "arrival": t,
                    "args": {"Lc": Lc, "W": W, "H": H, "k": k, "u_in": u_in, "steps": st}})
    return out
