"""Closed-form pins of the oracle's collision at a single node.

The expected values are moment identities that follow from the paper's
operators (Sec. II, Eqs. (5), (6), (9), (10), (11)), not re-typings of the
oracle's per-population formulas: a dropped term, a wrong sign or a swapped
index in the oracle changes at least one of these moments.
"""
import numpy as np
import pytest

CS2 = 1.0 / 3.0


def _setup(orc, lat, tau=(1.3, 0.7), A=(0.01, 0.03), alpha=(0.0, 0.0), beta=0.7,
           collision=None):
    L = orc.D2Q9 if lat == "D2Q9" else orc.D3Q19
    p = orc.Params(lattice=L, dims=(1, 1, 1), tau=tau, A=A, alpha=alpha, beta=beta,
                   collision=orc.REGULARIZED if collision is None else collision)
    o = orc.Oracle(p)
    t = orc.lattice_tables(L)
    return o, t, (2 if lat == "D2Q9" else 3)


def _random_node(rng, t, D, lo=0.05):
    Q = len(t["w"])
    fin = t["w"][None, :] * rng.uniform(lo, 1.0, (2, 1)) * (1 + 0.2 * rng.uniform(-1, 1, (2, Q)))
    F = np.zeros(3)
    F[:D] = rng.normal(0, 0.3, D)
    return fin, F


def _phat(lat, alpha):
    # Eq. (8) for D2Q9; the same sum of phi_i c_ix^2 for D3Q19.
    return 3 * (1 - alpha) / 5 if lat == "D2Q9" else (1 - alpha) / 2


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("collision", ["reg", "bgk"])
def test_moments_of_collision_and_perturbation(orc, lat, collision):
    rng = np.random.default_rng(11)
    tau, A, beta = (1.3, 0.7), (0.01, 0.03), 0.7
    o, t, D = _setup(orc, lat, tau, A, collision=orc.BGK if collision == "bgk" else orc.REGULARIZED)
    c = t["c"].astype(float)
    w0 = t["w"][0]
    for _ in range(20):
        fin, F = _random_node(rng, t, D)
        post, f2 = o.collide_node(fin, F)
        rk = fin.sum(1)
        rho = rk.sum()
        j = np.einsum("ki,ia->a", fin, c)
        u = j / rho
        # per-colour mass after recolouring (Eq. (10) with Eq. (2))
        assert np.allclose(post.sum(1), rk, rtol=0, atol=1e-15)
        # total momentum (Eq. (3)): kept by the relaxation (one rate per
        # node, both forms), the perturbation and the recolouring.
        assert np.allclose(np.einsum("ki,ia->a", post, c), j, atol=1e-15)
        assert np.isclose(f2.sum(), rho, atol=1e-15)
        assert np.allclose(f2 @ c, j, atol=1e-15)
        # second moment: relaxed momentum flux plus the perturbation stress
        # -2 Abar c_s^4 |F| (I - n n), Abar = sum_k A_k / 2
        Fn = np.linalg.norm(F)
        n = F / Fn
        I = np.eye(3)
        I[D:, D:] = 0
        # the node relaxes at the mixture viscosity, the harmonic mean of
        # nu_k = (tau_k - 1/2)/3 weighted by the colour fractions
        nu = 1 / sum(rk[k] / rho / ((tau[k] - 0.5) / 3) for k in range(2))
        om = 1 / (3 * nu + 0.5)
        Pi_eq = rho * (_phat(lat, w0) * I + np.outer(u, u))
        Pi = np.einsum("ki,ia,ib->ab", fin, c, c)
        expect = Pi_eq + (1 - om) * (Pi - Pi_eq)
        Abar = 0.5 * (A[0] + A[1])
        expect += -2 * Abar * CS2 ** 2 * Fn * (I - np.outer(n, n))
        assert np.allclose(np.einsum("i,ia,ib->ab", f2, c, c), expect, atol=2e-15)
        # recolouring: the two colours add up to the perturbed total
        assert np.allclose(post.sum(0), f2, atol=1e-16)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("alpha", [(0.0, 0.0), (0.3, 0.55)])
def test_recolouring_moves_red_along_gradient(orc, lat, alpha):
    # sum_i (f_i^R* - rho^R/rho f_i) c_i = beta rho^R rho^B / rho^2 *
    #     sum_k rho^k (1 - alpha_k)/(1 - w_0) * kappa * F/|F|,
    # kappa = sum_i w_i c_ix^2 / |c_i|.
    rng = np.random.default_rng(5)
    beta = 0.7
    o, t, D = _setup(orc, lat, alpha=alpha, beta=beta)
    c = t["c"].astype(float)
    w0 = t["w"][0]
    al = [a if a > 0 else w0 for a in alpha]
    kappa = 2 / 9 + 1 / (9 * np.sqrt(2)) if lat == "D2Q9" else 1 / 9 + 2 / (9 * np.sqrt(2))
    for _ in range(10):
        fin, F = _random_node(rng, t, D)
        post, f2 = o.collide_node(fin, F)
        rk = fin.sum(1)
        rho = rk.sum()
        lhs = (post[0] - rk[0] / rho * f2) @ c
        scale = sum(rk[k] * (1 - al[k]) / (1 - w0) for k in range(2))
        rhs = beta * rk[0] * rk[1] / rho ** 2 * scale * kappa * F / np.linalg.norm(F)
        assert np.allclose(lhs, rhs, atol=1e-15)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_regularized_ignores_non_hydrodynamic_content(orc, lat):
    # Eq. (11): the regularized post-collision state depends on rho^k, rho u
    # and Pi^k only.  Adding a vector with zero density, momentum and momentum
    # flux (a ghost mode) to a colour leaves the output unchanged; plain BGK
    # (Eq. (5)) passes it on scaled by (1 - omega).
    rng = np.random.default_rng(7)
    o, t, D = _setup(orc, lat)
    ob, _, _ = _setup(orc, lat, collision=orc.BGK)
    c = t["c"].astype(float)
    rows = [np.ones(len(c))] + [c[:, a] for a in range(D)] + \
           [c[:, a] * c[:, b] for a in range(D) for b in range(a, D)]
    M = np.array(rows)
    for _ in range(5):
        fin, F = _random_node(rng, t, D)
        r = rng.normal(0, 1e-3, len(c))
        g = r - M.T @ np.linalg.solve(M @ M.T, M @ r)
        assert np.abs(M @ g).max() < 1e-15
        fin2 = fin.copy()
        fin2[1] += g
        a, _ = o.collide_node(fin, F)
        b, _ = o.collide_node(fin2, F)
        assert np.abs(a - b).max() < 1e-15
        a, _ = ob.collide_node(fin, F)
        b, _ = ob.collide_node(fin2, F)
        assert np.abs(a - b).max() > 1e-6


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_tau_one_regularized_equals_bgk(orc, lat):
    # With omega = 1 both Eq. (5) and Eq. (11) return the equilibrium.
    rng = np.random.default_rng(3)
    o, t, D = _setup(orc, lat, tau=(1.0, 1.0))
    ob, _, _ = _setup(orc, lat, tau=(1.0, 1.0), collision=orc.BGK)
    for _ in range(5):
        fin, F = _random_node(rng, t, D)
        a, fa = o.collide_node(fin, F)
        b, fb = ob.collide_node(fin, F)
        assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_single_phase_and_zero_gradient(orc, lat):
    # rho^B = 0: the blue output is exactly zero and red carries the whole
    # perturbed total (recolouring is the identity).  F = 0: no perturbation
    # and colour is split in proportion to density.
    rng = np.random.default_rng(9)
    o, t, D = _setup(orc, lat)
    for _ in range(5):
        fin, F = _random_node(rng, t, D)
        fin[1] = 0.0
        post, f2 = o.collide_node(fin, F)
        assert np.all(post[1] == 0.0)
        assert np.array_equal(post[0], f2)
        fin, _ = _random_node(rng, t, D)
        post, f2 = o.collide_node(fin, np.zeros(3))
        rk = fin.sum(1)
        assert np.allclose(post[0], rk[0] / rk.sum() * f2, atol=1e-17)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("collision", ["reg", "bgk"])
def test_pure_components_relax_at_their_own_rate(orc, lat, collision):
    # A node holding one colour only relaxes its momentum flux by exactly
    # 1 - 1/tau_k of that component (the mixture rule reduces to tau_k).
    rng = np.random.default_rng(13)
    tau = (1.3, 0.7)
    o, t, D = _setup(orc, lat, tau, collision=orc.BGK if collision == "bgk" else orc.REGULARIZED)
    c = t["c"].astype(float)
    w0 = t["w"][0]
    I = np.eye(3)
    I[D:, D:] = 0
    for k in range(2):
        fin, _ = _random_node(rng, t, D)
        fin[1 - k] = 0.0
        post, _ = o.collide_node(fin, np.zeros(3))
        rho = fin.sum()
        u = fin[k] @ c / rho
        Pi_eq = rho * (_phat(lat, w0) * I + np.outer(u, u))
        Pi = np.einsum("i,ia,ib->ab", fin[k], c, c)
        got = np.einsum("i,ia,ib->ab", post[k], c, c)
        assert np.allclose(got, Pi_eq + (1 - 1 / tau[k]) * (Pi - Pi_eq), atol=2e-15)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("alpha", [(0.0, 0.0), (0.3, 0.55)])
def test_moments_of_per_colour_bgk(orc, lat, alpha):
    # Eq. (5) as written: colour k relaxes towards its own equilibrium
    # f^{k,eq}(rho^k, u) (Eq. (6), common u of Eq. (3)) at omega_k = 1/tau_k.
    # Zeroth and first moments of the relaxed total (F = 0: no perturbation):
    #   sum_i f_i = rho,
    #   sum_i f_i c_i = sum_k (1 - omega_k) j^k + omega_k rho^k u,
    # so momentum is not kept when tau_R != tau_B (j^k != rho^k u); second
    # moment sum_k (1 - omega_k) Pi^k + omega_k rho^k (phat_k I + u u).
    rng = np.random.default_rng(17)
    tau = (1.6, 0.6)
    o, t, D = _setup(orc, lat, tau, alpha=alpha, collision=orc.BGK_COLOUR)
    c = t["c"].astype(float)
    w0 = t["w"][0]
    al = [a if a > 0 else w0 for a in alpha]
    I = np.eye(3)
    I[D:, D:] = 0
    for _ in range(10):
        fin, _ = _random_node(rng, t, D)
        post, f2 = o.collide_node(fin, np.zeros(3))
        rk = fin.sum(1)
        rho = rk.sum()
        jk = fin @ c
        u = jk.sum(0) / rho
        om = [1 / tau[0], 1 / tau[1]]
        assert np.isclose(f2.sum(), rho, atol=1e-15)
        expect_j = sum((1 - om[k]) * jk[k] + om[k] * rk[k] * u for k in range(2))
        assert np.allclose(f2 @ c, expect_j, atol=1e-15)
        assert np.abs(f2 @ c - jk.sum(0)).max() > 1e-6  # momentum changes
        Pk = np.einsum("ki,ia,ib->kab", fin, c, c)
        expect_P = sum((1 - om[k]) * Pk[k] + om[k] * rk[k] * (_phat(lat, al[k]) * I + np.outer(u, u))
                       for k in range(2))
        assert np.allclose(np.einsum("i,ia,ib->ab", f2, c, c), expect_P, atol=2e-15)
        assert np.allclose(post.sum(1), rk, atol=1e-15)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_per_colour_bgk_at_equal_rates_is_node_rate_bgk(orc, lat):
    # With tau_R = tau_B both readings of Eq. (5) relax at the same rate.
    rng = np.random.default_rng(19)
    a_o, t, D = _setup(orc, lat, tau=(0.9, 0.9), collision=orc.BGK_COLOUR)
    b_o, _, _ = _setup(orc, lat, tau=(0.9, 0.9), collision=orc.BGK)
    for _ in range(5):
        fin, F = _random_node(rng, t, D)
        a, _ = a_o.collide_node(fin, F)
        b, _ = b_o.collide_node(fin, F)
        assert np.abs(a - b).max() < 1e-15
