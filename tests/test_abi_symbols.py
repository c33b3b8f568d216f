"""The C-ABI library loads and exports every function include/lbcg.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbcg.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbcg_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1711_02003_amd import lbcg
    if not os.path.exists(lbcg.LIB_PATH):
        from paper_1711_02003_amd import build
        build.build()
    return ctypes.CDLL(lbcg.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("lbcg_create", "lbcg_step", "lbcg_fields", "lbcg_footprint", "lbcg_diagnostics",
              "lbcg_destroy", "lbcg_batch_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1711_02003_amd import lbcg
    assert sorted(lbcg._SIGS) == declared()


def test_strerror_and_validation_without_device(lib):
    # lbcg_strerror and lbcg_footprint make no device calls.
    from paper_1711_02003_amd import lbcg
    lbcg._lib = None
    assert lbcg.strerror(0) == "ok"
    assert "invalid" in lbcg.strerror(-1)
    p, keep = lbcg.make_params("D3Q19", (256, 256, 256), 1.0, 0.6, 0.005, 0.005, 0.7)
    b = lbcg.footprint(p)
    assert b >= 2 * 38 * 256 ** 3 * 4
    for bad in (dict(tau_R=0.5), dict(dims=(0, 4, 4)), dict(beta=1.5)):
        kw = dict(lattice="D3Q19", dims=(8, 8, 8), tau_R=1.0, tau_B=1.0, A_R=0.0, A_B=0.0, beta=0.7)
        kw.update(bad)
        p, keep = lbcg.make_params(**kw)
        with pytest.raises(lbcg.LbcgError) as e:
            lbcg.footprint(p)
        assert e.value.status == lbcg.E_INVAL
    # D2Q9 needs nz = 1; mask codes must name a declared inlet/outlet
    p, keep = lbcg.make_params("D2Q9", (8, 8, 2), 1.0, 1.0, 0.0, 0.0, 0.7)
    with pytest.raises(lbcg.LbcgError):
        lbcg.footprint(p)
    import numpy as np
    m = np.zeros((1, 8, 8), np.uint8)
    m[0, 0, 0] = 2
    p, keep = lbcg.make_params("D2Q9", (8, 8, 1), 1.0, 1.0, 0.0, 0.0, 0.7, mask=m)
    with pytest.raises(lbcg.LbcgError):
        lbcg.footprint(p)


def test_compact_footprint_adds_two_compact_buffers(lib):
    # LBCG_KERNEL_COMPACT keeps two compact states (19 x 4 B of totals and
    # 20 B of colour scalars per pitch node) beside the two pair buffers
    from paper_1711_02003_amd import lbcg
    lbcg._lib = None
    dims = (70, 37, 20)
    pitch = -(-70 * 37 * 20 // 64) * 64
    f, keep = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, kernel=lbcg.KERNEL_FUSED)
    c, keep2 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, kernel=lbcg.KERNEL_COMPACT)
    extra = lbcg.footprint(c) - lbcg.footprint(f)
    one = -(-(19 * 4 + 20) * pitch // 256) * 256
    assert one * 2 - 512 <= extra <= one * 2 + 512, (extra, one)
    # FP16: 19 x 2 B of totals, 12 B of colour scalars (M in FP32)
    f16, keep4 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, "f16", kernel=lbcg.KERNEL_FUSED)
    c16, keep5 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, "f16", kernel=lbcg.KERNEL_COMPACT)
    extra = lbcg.footprint(c16) - lbcg.footprint(f16)
    one = -(-(19 * 2 + 12) * pitch // 256) * 256
    assert one * 2 - 512 <= extra <= one * 2 + 512, (extra, one)
    # 8-row tiles only; 32-wide tiles on the compact D3Q19 sweep only
    t, keep3 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, kernel=lbcg.KERNEL_COMPACT,
                                tile=(4, 0, 0))
    with pytest.raises(lbcg.LbcgError):
        lbcg.footprint(t)
    t, keep3 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, kernel=lbcg.KERNEL_COMPACT,
                                tile=(8, 0, 32))
    assert lbcg.footprint(t) > 0
    for bad in (dict(kernel=lbcg.KERNEL_FUSED, tile=(8, 0, 32)), dict(kernel=lbcg.KERNEL_COMPACT, tile=(8, 0, 48))):
        t, keep3 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, **bad)
        with pytest.raises(lbcg.LbcgError):
            lbcg.footprint(t)


def test_wall_and_collision_validation(lib):
    # Wetting walls: mask codes 64 + j need j < n_walls and psi_w in [-1, 1];
    # at most 62 inlets (codes 2..63); the three collision forms.
    import numpy as np

    from paper_1711_02003_amd import lbcg
    lbcg._lib = None
    m = np.zeros((1, 8, 8), np.uint8)
    m[0, 0, :] = lbcg.WALL0 + 1
    p, keep = lbcg.make_params("D2Q9", (8, 8, 1), 1.0, 1.0, 0.0, 0.0, 0.7, mask=m,
                               walls=[{"psi": 0.2}, {"psi": -1.0}])
    assert lbcg.footprint(p) > 0
    for walls in ([{"psi": 0.2}], [{"psi": 0.2}, {"psi": 1.5}], [{"psi": 0.2}, {"psi": float("nan")}]):
        p, keep = lbcg.make_params("D2Q9", (8, 8, 1), 1.0, 1.0, 0.0, 0.0, 0.7, mask=m, walls=walls)
        with pytest.raises(lbcg.LbcgError) as e:
            lbcg.footprint(p)
        assert e.value.status == lbcg.E_INVAL
    inl = [{"u": (0.0, 0.0, 0.0), "rho_R": 1.0, "rho_B": 0.0}]
    p, keep = lbcg.make_params("D2Q9", (8, 8, 1), 1.0, 1.0, 0.0, 0.0, 0.7, inlets=inl * 62)
    assert lbcg.footprint(p) > 0
    p, keep = lbcg.make_params("D2Q9", (8, 8, 1), 1.0, 1.0, 0.0, 0.0, 0.7, inlets=inl * 63)
    with pytest.raises(lbcg.LbcgError):
        lbcg.footprint(p)
    for coll in (lbcg.REGULARIZED, lbcg.BGK, lbcg.BGK_COLOUR):
        p, keep = lbcg.make_params("D3Q19", (8, 8, 8), 1.0, 0.7, 0.0, 0.0, 0.7, collision=coll)
        assert lbcg.footprint(p) > 0
    p, keep = lbcg.make_params("D3Q19", (8, 8, 8), 1.0, 0.7, 0.0, 0.0, 0.7, collision=3)
    with pytest.raises(lbcg.LbcgError):
        lbcg.footprint(p)


def test_geometry_compact_and_bgk_validation(lib):
    # The compact state with a mask runs the split step: its footprint adds
    # the split step's scratch (12 moments and a node-list entry per node,
    # block lists), it takes no launch shape, and plain BGK takes 8-row tiles
    # on the fused D3Q19 sweep (any on the generic kernel); BGK lattices
    # carry no split-step scratch.
    import numpy as np

    from paper_1711_02003_amd import lbcg
    lbcg._lib = None
    dims = (70, 13, 9)
    pitch = -(-70 * 13 * 9 // 64) * 64
    m = np.zeros((9, 13, 70), np.uint8)
    m[:, 0, :] = 1
    kw = dict(mask=m)
    per = dict(kernel=lbcg.KERNEL_COMPACT)
    c, k1 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, kernel=lbcg.KERNEL_COMPACT)
    cm, k2 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, **per, **kw)
    extra = lbcg.footprint(cm) - lbcg.footprint(c)
    # mask (1 B), link words (4 B), moments (48 B) and node list (4 B) per node
    assert (1 + 4 + 48 + 4) * pitch <= extra <= (1 + 4 + 48 + 4) * pitch + 64 * 1024, extra
    for prec in ("f32", "f16"):
        p, k3 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, prec, **per, **kw)
        assert lbcg.footprint(p) > 0
        p, k3 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, prec, **per, **kw, tile=(8, 2, 0))
        with pytest.raises(lbcg.LbcgError):
            lbcg.footprint(p)
    for kernel, ok in ((lbcg.KERNEL_FUSED, False), (lbcg.KERNEL_AUTO, False), (lbcg.KERNEL_GENERIC, True)):
        p, k4 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, collision=lbcg.BGK, kernel=kernel,
                                 tile=(4, 0, 0))
        if ok:
            assert lbcg.footprint(p) > 0
        else:
            with pytest.raises(lbcg.LbcgError):
                lbcg.footprint(p)
    p, k5 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, "f64", collision=lbcg.BGK, tile=(4, 0, 0))
    assert lbcg.footprint(p) > 0
    reg, k6 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, **kw)
    bgk, k7 = lbcg.make_params("D3Q19", dims, 1.0, 0.6, 0.005, 0.005, 0.7, collision=lbcg.BGK, **kw)
    assert lbcg.footprint(reg) - lbcg.footprint(bgk) >= (48 + 4) * pitch
