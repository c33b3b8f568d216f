"""Shared test helpers: map seeded workloads onto the oracle's parameters and
compare fields.  Test infrastructure only."""
import numpy as np


def oracle_params(orc, w, threads=0, collision=None):
    """Oracle parameters for a workloads.Workload (A_R = A_B = A)."""
    return orc.Params(
        lattice=orc.D2Q9 if w.lattice == "D2Q9" else orc.D3Q19,
        dims=w.dims, tau=(w.tau_R, w.tau_B), A=(w.A, w.A), alpha=(0.0, 0.0), beta=w.beta,
        eps_F=1e-8, mask=w.mask,
        inlets=[orc.Inlet(u=i["u"], rho_w=(i["rho_R"], i["rho_B"])) for i in w.inlets],
        outlets=[orc.Outlet(rho=o["rho"]) for o in w.outlets],
        walls=[orc.Wall(psi=wl["psi"]) for wl in getattr(w, "walls", [])],
        collision=orc.REGULARIZED if collision is None else collision, threads=threads)


def oracle_for(orc, w, threads=0, collision=None):
    return orc.Oracle(oracle_params(orc, w, threads, collision)).init(w.rhoR, w.rhoB, w.u)


def rel_l2(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))
