"""Test-infrastructure oracle for the regularized colour-gradient LB step.

Plain FP64 CPU code (``rcg_oracle.c``) behind ctypes, plus an independent
per-equation NumPy version (``literal.py``) for tiny lattices.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does.  Method: arXiv:1711.02003, Sec. II,
Eqs. (1)-(11).

Array conventions of this binding: scalar fields have shape (nz, ny, nx)
(x fastest), vector fields (3, nz, ny, nx); populations are stored
array-of-structures as (nz, ny, nx, 2, Q) = [node][colour][direction].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcg_oracle.so")
SRC = os.path.join(HERE, "rcg_oracle.c")

D2Q9, D3Q19 = 0, 1
REGULARIZED, BGK, BGK_COLOUR = 0, 1, 2
INLET0, WALL0, OUTLET0 = 2, 64, 128  # mask codes: inlet j, wetting wall j, outlet j


def build(force: bool = True) -> str:
    """Compile the C oracle in-tree with gcc (-O3, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Inlet(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("rho_w", C.c_double * 2)]


class _Outlet(C.Structure):
    _fields_ = [("rho", C.c_double)]


class _Wall(C.Structure):
    _fields_ = [("psi", C.c_double)]


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("collision", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("tau", C.c_double * 2), ("A", C.c_double * 2), ("alpha", C.c_double * 2),
        ("beta", C.c_double), ("eps_F", C.c_double),
        ("mask", C.POINTER(C.c_uint8)),
        ("n_inlets", C.c_int), ("inlets", C.POINTER(_Inlet)),
        ("n_outlets", C.c_int), ("outlets", C.POINTER(_Outlet)),
        ("n_walls", C.c_int), ("walls", C.POINTER(_Wall)),
        ("n_threads", C.c_int),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("mass", C.c_double * 2), ("momentum", C.c_double * 3), ("max_u", C.c_double),
        ("p_in", C.c_double), ("p_out", C.c_double), ("n_in", C.c_long), ("n_out", C.c_long),
        ("vol_R", C.c_double), ("R_eff", C.c_double), ("nonfinite", C.c_long),
        ("fluid_nodes", C.c_long),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_Params)
        lib.orc_lattice.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_int), dp, dp, dp,
                                    C.POINTER(C.c_int)]
        lib.orc_init.argtypes = [P, dp, dp, dp, dp]
        lib.orc_step.argtypes = [P, dp, C.c_int]
        lib.orc_fields.argtypes = [P, dp, dp, dp, dp, dp]
        lib.orc_gradient.argtypes = [P, dp, dp]
        lib.orc_diagnostics.argtypes = [P, dp, C.POINTER(_Diag)]
        lib.orc_collide_node.argtypes = [P, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lattice_tables(lattice: int, alpha: float = 0.0) -> dict:
    """Velocity set, weights, phi(alpha), B and opposite index as the C oracle builds them."""
    lib = _load()
    Q = 9 if lattice == D2Q9 else 19
    c = np.zeros(3 * Q, dtype=np.int32)
    w, phi, B = (np.zeros(Q) for _ in range(3))
    opp = np.zeros(Q, dtype=np.int32)
    q = lib.orc_lattice(lattice, alpha, c.ctypes.data_as(C.POINTER(C.c_int)), _dp(w), _dp(phi),
                        _dp(B), opp.ctypes.data_as(C.POINTER(C.c_int)))
    assert q == Q
    return {"c": c.reshape(Q, 3), "w": w, "phi": phi, "B": B, "opp": opp}


@dataclass
class Inlet:
    u: Sequence[float]
    rho_w: Sequence[float]  # (rho_R, rho_B) injected


@dataclass
class Outlet:
    rho: float = 1.0  # prescribed outlet density


@dataclass
class Wall:
    psi: float = 0.0  # phase value the colour gradient sees at this wetting wall


@dataclass
class Params:
    """Model parameters, named as in the paper (Eqs. (5), (7), (9), (10))."""
    lattice: int
    dims: Sequence[int]             # (nx, ny, nz); nz = 1 for D2Q9
    tau: Sequence[float] = (1.0, 1.0)
    A: Sequence[float] = (0.0, 0.0)
    alpha: Sequence[float] = (0.0, 0.0)   # 0 -> w_0 (equal densities)
    beta: float = 0.7
    eps_F: float = 1e-8
    mask: Optional[np.ndarray] = None     # uint8 (nz, ny, nx)
    inlets: Sequence[Inlet] = field(default_factory=list)
    outlets: Sequence[Outlet] = field(default_factory=list)
    walls: Sequence[Wall] = field(default_factory=list)   # mask codes WALL0 + j
    collision: int = REGULARIZED
    threads: int = 0

    @property
    def Q(self) -> int:
        return 9 if self.lattice == D2Q9 else 19

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)


class Oracle:
    """FP64 CPU reference simulation (pre-collision state S_t)."""

    def __init__(self, p: Params):
        self.p = p
        self._lib = _load()
        nx, ny, nz = (int(v) for v in p.dims)
        self.N = nx * ny * nz
        self._keep = []
        cp = _Params()
        cp.lattice, cp.collision = p.lattice, p.collision
        cp.nx, cp.ny, cp.nz = nx, ny, nz
        cp.tau[:] = list(p.tau)
        cp.A[:] = list(p.A)
        cp.alpha[:] = list(p.alpha)
        cp.beta, cp.eps_F = p.beta, p.eps_F
        if p.mask is not None:
            m = np.ascontiguousarray(p.mask, dtype=np.uint8).reshape(-1)
            assert m.size == self.N
            self._keep.append(m)
            cp.mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
        ins = (_Inlet * max(1, len(p.inlets)))()
        for j, inl in enumerate(p.inlets):
            ins[j].u[:] = [float(v) for v in inl.u]
            ins[j].rho_w[:] = [float(v) for v in inl.rho_w]
        outs = (_Outlet * max(1, len(p.outlets)))()
        for j, o in enumerate(p.outlets):
            outs[j].rho = float(o.rho)
        wls = (_Wall * max(1, len(p.walls)))()
        for j, wl in enumerate(p.walls):
            wls[j].psi = float(wl.psi)
        self._keep += [ins, outs, wls]
        cp.n_inlets, cp.inlets = len(p.inlets), ins
        cp.n_outlets, cp.outlets = len(p.outlets), outs
        cp.n_walls, cp.walls = len(p.walls), wls
        cp.n_threads = p.threads
        self._cp = cp
        self.f = np.zeros((nz, ny, nx, 2, p.Q), dtype=np.float64)

    def _pp(self):
        return C.byref(self._cp)

    def init(self, rhoR, rhoB, u=None):
        rR = np.ascontiguousarray(rhoR, dtype=np.float64).reshape(-1)
        rB = np.ascontiguousarray(rhoB, dtype=np.float64).reshape(-1)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        rc = self._lib.orc_init(self._pp(), _dp(rR), _dp(rB), _dp(uu), _dp(self.f))
        if rc:
            raise ValueError(f"orc_init failed ({rc})")
        return self

    def step(self, n: int = 1):
        rc = self._lib.orc_step(self._pp(), _dp(self.f), int(n))
        if rc:
            raise ValueError(f"orc_step failed ({rc})")
        return self

    def fields(self):
        sh = self.p.shape
        rR, rB, psi = np.zeros(sh), np.zeros(sh), np.zeros(sh)
        u = np.zeros((3,) + sh)
        rc = self._lib.orc_fields(self._pp(), _dp(self.f), _dp(rR), _dp(rB), _dp(u), _dp(psi))
        if rc:
            raise ValueError(f"orc_fields failed ({rc})")
        return {"rhoR": rR, "rhoB": rB, "u": u, "psi": psi}

    def gradient(self):
        F = np.zeros((3,) + self.p.shape)
        rc = self._lib.orc_gradient(self._pp(), _dp(self.f), _dp(F))
        if rc:
            raise ValueError(f"orc_gradient failed ({rc})")
        return F

    def diagnostics(self) -> dict:
        """FP64 diagnostics of the current state (mass, momentum, max |u|,
        Eq. (8) pressures inside and outside, R_eff, non-finite count)."""
        d = _Diag()
        rc = self._lib.orc_diagnostics(self._pp(), _dp(self.f), C.byref(d))
        if rc:
            raise ValueError(f"orc_diagnostics failed ({rc})")
        out = {k: getattr(d, k) for k, _ in _Diag._fields_}
        out["mass"] = list(d.mass)
        out["momentum"] = list(d.momentum)
        return out

    def collide_node(self, fin: np.ndarray, F: Sequence[float]):
        """Collision + perturbation + recolouring at one node: returns (post[2,Q], f2[Q])."""
        Q = self.p.Q
        fi = np.ascontiguousarray(fin, dtype=np.float64).reshape(2 * Q)
        Fa = np.ascontiguousarray(F, dtype=np.float64).reshape(3)
        out = np.zeros(2 * Q)
        f2 = np.zeros(Q)
        rc = self._lib.orc_collide_node(self._pp(), _dp(fi), _dp(Fa), _dp(out), _dp(f2))
        if rc:
            raise ValueError("orc_collide_node failed")
        return out.reshape(2, Q), f2

    def populations(self) -> np.ndarray:
        """Pre-collision populations as (2, Q, nz, ny, nx)."""
        return np.ascontiguousarray(np.moveaxis(self.f, (3, 4), (0, 1)))

    def set_populations(self, f_kq: np.ndarray):
        self.f[...] = np.moveaxis(np.asarray(f_kq, dtype=np.float64), (0, 1), (3, 4))
        return self
