"""Python binding of the lbcg C ABI (include/lbcg.h): argument marshalling only.

Every step of the method runs in the HIP library ``liblbcg.so``; this module
converts NumPy arrays and Python parameters into the C structures, and uses
PyTorch (when present) only for device memory and the current HIP stream.
There is no CPU fallback: if the library or a gfx950 device is missing, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBCG_LIBRARY", os.path.join(HERE, "liblbcg.so"))

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSTABLE, E_STATE = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19 = 0, 1
F64, F32, F16 = 0, 1, 2
REGULARIZED, BGK, BGK_COLOUR = 0, 1, 2
INLET0, WALL0, OUTLET0 = 2, 64, 128  # mask codes: inlet j, wetting wall j, outlet j
KERNEL_AUTO, KERNEL_GENERIC, KERNEL_FUSED, KERNEL_COMPACT = 0, 1, 2, 3
PRECISIONS = {"f64": F64, "f32": F32, "f16": F16}
LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19}


class LbcgError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class _Inlet(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("rho_R", C.c_double), ("rho_B", C.c_double)]


class _Outlet(C.Structure):
    _fields_ = [("rho", C.c_double)]


class _Wall(C.Structure):
    _fields_ = [("psi", C.c_double)]


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("precision", C.c_int32), ("collision", C.c_int32),
        ("kernel", C.c_int32), ("dims", C.c_int64 * 3), ("mask", C.POINTER(C.c_uint8)),
        ("tau_R", C.c_double), ("tau_B", C.c_double), ("A_R", C.c_double), ("A_B", C.c_double),
        ("beta", C.c_double), ("alpha_R", C.c_double), ("alpha_B", C.c_double),
        ("eps_F", C.c_double), ("n_inlets", C.c_int32), ("n_outlets", C.c_int32),
        ("inlets", C.POINTER(_Inlet)), ("outlets", C.POINTER(_Outlet)),
        ("n_walls", C.c_int32), ("walls", C.POINTER(_Wall)), ("tile", C.c_int32 * 3),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("mass_R", C.c_double), ("mass_B", C.c_double), ("momentum", C.c_double * 3),
        ("max_u", C.c_double), ("p_in", C.c_double), ("p_out", C.c_double),
        ("vol_R", C.c_double), ("R_eff", C.c_double), ("nonfinite", C.c_int64),
        ("n_in", C.c_int64), ("n_out", C.c_int64), ("fluid_nodes", C.c_int64),
        ("step", C.c_int64),
    ]


# Every exported symbol of include/lbcg.h, with its ctypes signature.
_P = C.POINTER
_SIGS = {
    "lbcg_footprint": (C.c_int, [_P(_Params), _P(C.c_size_t)]),
    "lbcg_create": (C.c_int, [_P(_Params), C.c_void_p, C.c_size_t, C.c_void_p, _P(C.c_void_p)]),
    "lbcg_init_fields": (C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
    "lbcg_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbcg_fields": (C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_double), _P(C.c_double),
                              _P(C.c_double)]),
    "lbcg_populations": (C.c_int, [C.c_void_p, _P(C.c_double)]),
    "lbcg_populations_at": (C.c_int, [C.c_void_p, _P(C.c_int64), C.c_int64, _P(C.c_double)]),
    "lbcg_diagnostics": (C.c_int, [C.c_void_p, _P(_Diag)]),
    "lbcg_state_bytes": (C.c_int, [C.c_void_p, _P(C.c_size_t)]),
    "lbcg_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbcg_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbcg_synchronize": (C.c_int, [C.c_void_p]),
    "lbcg_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbcg_destroy": (None, [C.c_void_p]),
    "lbcg_strerror": (C.c_char_p, [C.c_int]),
    "lbcg_launch_info": (C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)]),
    "lbcg_tune": (C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_int32)]),
    "lbcg_batch_create": (C.c_int, [_P(C.c_void_p), C.c_int32, _P(C.c_int32), _P(C.c_void_p)]),
    "lbcg_batch_step": (C.c_int, [C.c_void_p, _P(C.c_int64)]),
    "lbcg_batch_launch_info": (C.c_int, [C.c_void_p, _P(C.c_int32), _P(C.c_int32), _P(C.c_int64)]),
    "lbcg_batch_destroy": (None, [C.c_void_p]),
    "lbcg_batch_step_noalloc": (C.c_int, [_P(C.c_void_p), C.c_int32, _P(C.c_int32), _P(C.c_int64)]),
}
NOALLOC_MAX_LATTICES, NOALLOC_MAX_BLOCKS = 256, 65536

_lib = None


def load_library() -> C.CDLL:
    """Load liblbcg.so (built in-tree by ``paper_1711_02003_amd.build``)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime and hands this library its device
        # memory and streams: load torch first so that liblbcg.so binds to
        # that same runtime (loading it first would bring in a second runtime,
        # and every call with torch's pointers would then fail).
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:  # pragma: no cover
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1711_02003_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load_library().lbcg_strerror(int(status)).decode()


def _check(rc: int, what: str):
    if rc != OK:
        raise LbcgError(rc, what)


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Inlet:
    u: Sequence[float]
    rho_R: float
    rho_B: float


@dataclass
class Outlet:
    rho: float = 1.0


@dataclass
class Wall:
    psi: float = 0.0  # phase value the colour gradient sees at a wetting wall


def make_params(lattice, dims, tau_R, tau_B, A_R, A_B, beta, precision=F32, collision=REGULARIZED,
                kernel=KERNEL_AUTO, mask=None, inlets=(), outlets=(), alpha_R=0.0, alpha_B=0.0,
                eps_F=-1.0, tile=(0, 0, 0), walls=()):
    """Build the C parameter block; returns (params, keep-alive list)."""
    p = _Params()
    p.lattice = LATTICES.get(lattice, lattice)
    p.precision = PRECISIONS.get(precision, precision)
    p.collision, p.kernel = int(collision), int(kernel)
    p.dims[:] = [int(d) for d in dims]
    keep = []
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        keep.append(m)
        p.mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
    p.tau_R, p.tau_B, p.A_R, p.A_B, p.beta = float(tau_R), float(tau_B), float(A_R), float(A_B), float(beta)
    p.alpha_R, p.alpha_B, p.eps_F = float(alpha_R), float(alpha_B), float(eps_F)
    ins = (_Inlet * max(1, len(inlets)))()
    for j, i in enumerate(inlets):
        d = i if isinstance(i, dict) else i.__dict__
        ins[j].u[:] = [float(v) for v in d["u"]]
        ins[j].rho_R, ins[j].rho_B = float(d["rho_R"]), float(d["rho_B"])
    outs = (_Outlet * max(1, len(outlets)))()
    for j, o in enumerate(outlets):
        d = o if isinstance(o, dict) else o.__dict__
        outs[j].rho = float(d["rho"])
    wls = (_Wall * max(1, len(walls)))()
    for j, wl in enumerate(walls):
        d = wl if isinstance(wl, dict) else wl.__dict__
        wls[j].psi = float(d["psi"])
    keep += [ins, outs, wls]
    p.n_inlets, p.inlets = len(inlets), ins
    p.n_outlets, p.outlets = len(outlets), outs
    p.n_walls, p.walls = len(walls), wls
    p.tile[:] = [int(t) for t in tile]
    return p, keep


def footprint(params) -> int:
    b = C.c_size_t(0)
    _check(load_library().lbcg_footprint(C.byref(params), C.byref(b)), "lbcg_footprint")
    return int(b.value)


def _torch_device_buffer(nbytes: int):
    """Device memory from PyTorch's caching allocator (None if torch is absent)."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        return None, None
    if not torch.cuda.is_available():
        return None, None
    t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    return t, (stream or None)


class Sim:
    """One lattice simulated by the HIP library."""

    def __init__(self, lattice="D3Q19", dims=(64, 64, 64), tau_R=1.0, tau_B=1.0, A=0.01,
                 beta=0.7, precision="f32", collision=REGULARIZED, kernel=KERNEL_AUTO, mask=None,
                 inlets=(), outlets=(), alpha_R=0.0, alpha_B=0.0, eps_F=-1.0, A_B=None,
                 tile=(0, 0, 0), use_torch=True, stream=None, dev_buf=None, walls=()):
        self._lib = load_library()
        self.lattice = LATTICES.get(lattice, lattice)
        self.Q = 9 if self.lattice == D2Q9 else 19
        self.dims = tuple(int(d) for d in dims)
        self.N = int(np.prod(self.dims))
        self.precision = PRECISIONS.get(precision, precision)
        self.params, self._keep = make_params(
            self.lattice, self.dims, tau_R, tau_B, A, A if A_B is None else A_B, beta,
            self.precision, collision, kernel, mask, inlets, outlets, alpha_R, alpha_B, eps_F, tile, walls)
        self.footprint = footprint(self.params)
        self._buf = None
        dev_ptr, strm = None, stream
        if dev_buf is not None:
            # caller-owned device memory: (address, bytes), at least the footprint
            dev_ptr, nbytes = int(dev_buf[0]), int(dev_buf[1])
            if nbytes < self.footprint:
                raise ValueError(f"device buffer of {nbytes} bytes < footprint {self.footprint}")
        elif use_torch:
            self._buf, tstream = _torch_device_buffer(self.footprint)
            if self._buf is not None:
                dev_ptr = self._buf.data_ptr()
                if strm is None:
                    strm = tstream
        h = C.c_void_p()
        _check(self._lib.lbcg_create(C.byref(self.params), dev_ptr,
                                     self.footprint if dev_ptr else 0, strm, C.byref(h)),
               "lbcg_create")
        self._h = h

    @classmethod
    def from_workload(cls, w, precision="f32", kernel=KERNEL_AUTO, **kw):
        s = cls(w.lattice, w.dims, w.tau_R, w.tau_B, w.A, w.beta, precision, kernel=kernel,
                mask=w.mask, inlets=w.inlets, outlets=w.outlets, walls=getattr(w, "walls", ()), **kw)
        s.init_fields(w.rhoR, w.rhoB, w.u)
        return s

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def _handle(self):
        if self._h is None:
            raise RuntimeError("simulation already closed")
        return self._h

    def init_fields(self, rhoR, rhoB, u=None):
        rR = np.ascontiguousarray(rhoR, dtype=np.float64).reshape(-1)
        rB = np.ascontiguousarray(rhoB, dtype=np.float64).reshape(-1)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        assert rR.size == self.N and rB.size == self.N and (uu is None or uu.size == 3 * self.N)
        _check(self._lib.lbcg_init_fields(self._handle(), _dp(rR), _dp(rB), _dp(uu)), "lbcg_init_fields")
        return self

    def step(self, n: int = 1):
        _check(self._lib.lbcg_step(self._handle(), int(n)), "lbcg_step")
        return self

    def synchronize(self):
        _check(self._lib.lbcg_synchronize(self._handle()), "lbcg_synchronize")

    def set_stream(self, stream):
        """Queue later work on `stream` (a hipStream_t as int, or None for the
        library's own); the caller orders earlier work before it."""
        _check(self._lib.lbcg_set_stream(self._handle(), stream), "lbcg_set_stream")
        return self

    def fields(self):
        sh = self.shape
        rR, rB, psi = np.empty(sh), np.empty(sh), np.empty(sh)
        u = np.empty((3,) + sh)
        _check(self._lib.lbcg_fields(self._handle(), _dp(rR), _dp(rB), _dp(u), _dp(psi)), "lbcg_fields")
        return {"rhoR": rR, "rhoB": rB, "u": u, "psi": psi}

    def populations(self):
        """Pre-collision populations of S_t as (2, Q, nz, ny, nx) float64."""
        f = np.empty((2, self.Q) + self.shape)
        _check(self._lib.lbcg_populations(self._handle(), _dp(f)), "lbcg_populations")
        return f

    def populations_at(self, nodes) -> np.ndarray:
        """Pre-collision populations at listed node indices as (count, 2, Q)."""
        idx = np.ascontiguousarray(nodes, dtype=np.int64).reshape(-1)
        f = np.empty((idx.size, 2, self.Q))
        _check(self._lib.lbcg_populations_at(self._handle(), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                             idx.size, _dp(f)), "lbcg_populations_at")
        return f

    def diagnostics(self, check: bool = False) -> dict:
        d = _Diag()
        rc = self._lib.lbcg_diagnostics(self._handle(), C.byref(d))
        if rc not in (OK, E_UNSTABLE) or (check and rc != OK):
            _check(rc, "lbcg_diagnostics")
        out = {k: getattr(d, k) for k, _ in _Diag._fields_}
        out["momentum"] = list(d.momentum)
        out["status"] = rc
        return out

    def get_state(self) -> bytes:
        n = C.c_size_t(0)
        _check(self._lib.lbcg_state_bytes(self._handle(), C.byref(n)), "lbcg_state_bytes")
        buf = (C.c_char * n.value)()
        _check(self._lib.lbcg_get_state(self._handle(), buf, n.value), "lbcg_get_state")
        return bytes(buf)

    def set_state(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        _check(self._lib.lbcg_set_state(self._handle(), buf, len(blob)), "lbcg_set_state")
        return self

    def launch_info(self):
        k, r, z, t = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.lbcg_launch_info(self._handle(), C.byref(k), C.byref(r), C.byref(z), C.byref(t)),
               "lbcg_launch_info")
        return {"kernel": k.value, "rows": r.value, "zchunks": z.value, "tile_width": t.value}

    def tune(self):
        """Time candidate launch shapes of the fused kernel and keep the fastest."""
        r, z = C.c_int32(), C.c_int32()
        _check(self._lib.lbcg_tune(self._handle(), C.byref(r), C.byref(z)), "lbcg_tune")
        return {"rows": r.value, "zchunks": z.value, "tile_width": self.launch_info()["tile_width"]}

    def close(self):
        if self._h is not None:
            self._lib.lbcg_destroy(self._h)
            self._h = None
            self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Sim handles (all on the fused or all on the compact kernel, one
    precision, one stream) stepped together.

    ``tile`` = (rows per block, z planes per chunk); None = chosen by timing on
    the batch.  The batch keeps references to its handles.
    """

    def __init__(self, sims, tile=None):
        self._lib = load_library()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._handle().value for s in self.sims])
        t = None if tile is None else (C.c_int32 * 2)(*[int(v) for v in tile])
        h = C.c_void_p()
        _check(self._lib.lbcg_batch_create(arr, len(self.sims), t, C.byref(h)), "lbcg_batch_create")
        self._h = h

    def step(self, nsteps):
        """Advance lattice j by nsteps[j] steps (an int applies to every lattice)."""
        if np.isscalar(nsteps):
            nsteps = [int(nsteps)] * len(self.sims)
        n = np.ascontiguousarray(nsteps, dtype=np.int64)
        assert n.size == len(self.sims)
        if self._h is None:
            raise RuntimeError("batch already closed")
        _check(self._lib.lbcg_batch_step(self._h, n.ctypes.data_as(C.POINTER(C.c_int64))), "lbcg_batch_step")
        return self

    def synchronize(self):
        self.sims[0].synchronize()

    def launch_info(self):
        r, z, b = C.c_int32(), C.c_int32(), C.c_int64()
        _check(self._lib.lbcg_batch_launch_info(self._h, C.byref(r), C.byref(z), C.byref(b)),
               "lbcg_batch_launch_info")
        return {"rows": r.value, "zplanes": z.value, "blocks": b.value}

    def close(self):
        if self._h is not None:
            self._lib.lbcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_noalloc(sims, nsteps, tile):
    """lbcg_batch_step_noalloc: advance sims[j] by nsteps[j] steps (an int
    applies to every lattice) in the launch shape tile = (rows, z planes per
    chunk), with no batch object and no allocation."""
    lib = load_library()
    sims = list(sims)
    if np.isscalar(nsteps):
        nsteps = [int(nsteps)] * len(sims)
    n = np.ascontiguousarray(nsteps, dtype=np.int64)
    assert n.size == len(sims)
    arr = (C.c_void_p * len(sims))(*[s._handle().value for s in sims])
    t = (C.c_int32 * 2)(*[int(v) for v in tile])
    _check(lib.lbcg_batch_step_noalloc(arr, len(sims), t, n.ctypes.data_as(C.POINTER(C.c_int64))),
           "lbcg_batch_step_noalloc")
