"""Pins of the oracle's lattice tables against what the paper and the
mathematics fix (Sec. II, Eqs. (6)-(9))."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

CS2 = 1.0 / 3.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_velocity_set_isotropy(orc, lat):
    t = orc.lattice_tables(orc.D2Q9 if lat == "D2Q9" else orc.D3Q19)
    c, w, opp = t["c"].astype(float), t["w"], t["opp"]
    D = 2 if lat == "D2Q9" else 3
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    # odd moments vanish, second moment c_s^2 I, fourth moment c_s^4 (dd + dd + dd)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2[:D, :D], CS2 * np.eye(D), atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    I = np.eye(D)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                      + np.einsum("ad,bc->abcd", I, I))
    assert np.allclose(m4[:D, :D, :D, :D], iso, atol=1e-15)
    # opposite directions
    assert np.array_equal(c[opp], -c)
    assert len(set(map(tuple, t["c"]))) == len(w)


def test_d2q9_numbering_follows_eq7(orc):
    # Eq. (7): rest first, then nearest neighbours and diagonals alternate.
    t = orc.lattice_tables(orc.D2Q9)
    n2 = (t["c"] ** 2).sum(1)
    assert list(n2) == [0, 1, 2, 1, 2, 1, 2, 1, 2]


@pytest.mark.parametrize("alpha", [4 / 9, 0.2, 0.7, 0.9])
def test_phi_d2q9_eq7_and_pressure_eq8(orc, alpha):
    g = json.load(open(GOLDEN))
    assert "(1-alpha)/5" in g["phi_d2q9"]["axis"]
    t = orc.lattice_tables(orc.D2Q9, alpha)
    n2 = (t["c"] ** 2).sum(1)
    expect = np.where(n2 == 0, alpha, np.where(n2 == 1, (1 - alpha) / 5, (1 - alpha) / 20))
    assert np.allclose(t["phi"], expect, atol=1e-16)
    assert np.isclose(t["phi"].sum(), 1.0)
    # Eq. (8): p^k / rho^k = 3 (1 - alpha_k) / 5 = sum_i phi_i c_ix^2
    assert np.isclose((t["phi"] * t["c"][:, 0] ** 2).sum(), 3 * (1 - alpha) / 5)


@pytest.mark.parametrize("alpha", [1 / 3, 0.1, 0.6])
def test_phi_d3q19(orc, alpha):
    t = orc.lattice_tables(orc.D3Q19, alpha)
    assert np.isclose(t["phi"].sum(), 1.0)
    assert np.isclose((t["phi"] * t["c"][:, 0] ** 2).sum(), (1 - alpha) / 2)
    assert np.allclose((t["phi"][:, None] * t["c"]).sum(0), 0)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_equal_density_alpha_gives_weights(orc, lat):
    # alpha_k = w_0 makes phi = w and the colour pressure rho/3 (density ratio 1).
    L = orc.D2Q9 if lat == "D2Q9" else orc.D3Q19
    t = orc.lattice_tables(L, 0.0)
    assert np.allclose(t["phi"], t["w"], atol=1e-16)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_perturbation_constants(orc, lat):
    # sum_i B_i = c_s^2 (mass conservation of Eq. (9)) and
    # sum_i B_i c_i c_i = 3 c_s^4 I (stress proportional to I - nn).
    L = orc.D2Q9 if lat == "D2Q9" else orc.D3Q19
    D = 2 if lat == "D2Q9" else 3
    t = orc.lattice_tables(L)
    c, B = t["c"].astype(float), t["B"]
    assert np.isclose(B.sum(), CS2, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", B, c, c)[:D, :D], 3 * CS2 ** 2 * np.eye(D), atol=1e-16)
    n2 = (t["c"] ** 2).sum(1)
    known = ({0: Fraction(-4, 27), 1: Fraction(2, 27), 2: Fraction(5, 108)} if D == 2 else
             {0: Fraction(-2, 9), 1: Fraction(1, 54), 2: Fraction(1, 27)})
    assert np.allclose(B, [float(known[int(v)]) for v in n2], atol=1e-17)
