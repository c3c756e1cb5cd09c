"""Pins of the oracle's lattice tables and node-level algebra against what the
paper prints and against textbook lattice Boltzmann identities (CPU only)."""
import itertools

import numpy as np
import pytest

from conftest import load_matrix

# Standard D3Q19 equilibrium weights (textbook, e.g. Qian, d'Humieres &
# Lallemand 1992): rest 1/3, axis 1/18, diagonal 1/36.
CS2 = 1.0 / 3.0


def std_weights(e):
    e2 = (e * e).sum(axis=1)
    return np.where(e2 == 0, 1 / 3, np.where(e2 == 1, 1 / 18, 1 / 36))


def std_feq(rho, u, e):
    """Textbook second-order D3Q19 equilibrium."""
    w = std_weights(e)
    eu = e @ u
    return w * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))


def guo_forcing(F, u, e):
    """Textbook discrete forcing term of Guo, Zheng & Shi (2002) without the
    (1 - 1/2tau) prefactor: w [(e - u).F/cs^2 + (e.u)(e.F)/cs^4]."""
    w = std_weights(e)
    return w * (((e - u) @ F) / CS2 + (e @ u) * (e @ F) / CS2 ** 2)


@pytest.fixture(scope="module")
def T(oracle_lib):
    return oracle_lib.tables()


def test_d3q19_velocities_match_eq2(T):
    printed = load_matrix("d3q19_velocities.txt").astype(int)
    assert printed.shape == (3, 19)
    np.testing.assert_array_equal(T["e19"].T, printed)
    # opposite pairs (1,2), (3,4), ..., (17,18)
    for a in range(1, 19, 2):
        np.testing.assert_array_equal(T["e19"][a], -T["e19"][a + 1])


def test_d3q7_velocities_match_eq21(T):
    printed = load_matrix("d3q7_velocities.txt").astype(int)
    np.testing.assert_array_equal(T["e7"].T, printed)


def test_force_weights_eq7_isotropy(T):
    e = T["e19"].astype(float)
    om = T["omega"]
    assert om[0] == 0.0
    np.testing.assert_allclose(sorted(set(om[1:])), [1 / 12, 1 / 6])
    # second order: sum omega e_i e_j = delta_ij (so the stencil is a consistent gradient)
    np.testing.assert_allclose(np.einsum("a,ai,aj->ij", om, e, e), np.eye(3), atol=1e-15)
    # odd moments vanish, fourth order isotropic: sum w ex^4 = 3 sum w ex^2 ey^2
    np.testing.assert_allclose(np.einsum("a,ai->i", om, e), 0, atol=1e-15)
    np.testing.assert_allclose((om * e[:, 0] ** 4).sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(3 * (om * e[:, 0] ** 2 * e[:, 1] ** 2).sum(), 1.0, atol=1e-15)


def test_d3q7_weights_eq22(T):
    e = T["e7"].astype(float)
    w = T["wT"]
    d = 0.95
    np.testing.assert_allclose(w.sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(w @ e, 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("a,ai,aj->ij", w, e, e), d / 3 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(w[0], 1 - d)


def test_moment_matrix_invertible(T):
    M, Minv = T["M"], T["Minv"]
    assert np.linalg.matrix_rank(M) == 19
    np.testing.assert_allclose(M @ Minv, np.eye(19), atol=1e-14)
    np.testing.assert_allclose(Minv @ M, np.eye(19), atol=1e-14)


def test_equilibrium_moments_0_to_9_are_textbook(oracle_lib, T):
    """Eq. (5): the hydrodynamic moments (density, momentum, stress) equal
    the moments of the textbook D3Q19 equilibrium under M."""
    rng = np.random.default_rng(1)
    e = T["e19"].astype(float)
    for _ in range(20):
        rho = rng.uniform(0.1, 8)
        u = rng.uniform(-0.1, 0.1, 3)
        meq = oracle_lib.equilibrium_moments(rho, u)
        np.testing.assert_allclose(meq[:10], (T["M"] @ std_feq(rho, u, e))[:10], rtol=0, atol=1e-13)


def test_rest_equilibrium_is_weighted_density(oracle_lib, T):
    """M^-1 m_eq(rho, 0) must be the textbook rest equilibrium w_alpha rho."""
    e = T["e19"].astype(float)
    for rho in (0.38, 1.0, 6.5):
        f = T["Minv"] @ oracle_lib.equilibrium_moments(rho, np.zeros(3))
        np.testing.assert_allclose(f, std_weights(e) * rho, atol=1e-14)


def test_eq46_moment_groupings(T):
    """Eq. (46) groups m1+m11+m13, m2+m10+m15, m3+m12+m14: they must be the
    third-order moments sum e_i |e|^2 f."""
    e = T["e19"].astype(float)
    e2 = (e * e).sum(axis=1)
    f = np.random.default_rng(2).uniform(0, 1, 19)
    m = T["M"] @ f
    np.testing.assert_allclose(m[1] + m[11] + m[13], (e[:, 0] * e2 * f).sum(), atol=1e-14)
    np.testing.assert_allclose(m[2] + m[10] + m[15], (e[:, 1] * e2 * f).sum(), atol=1e-14)
    np.testing.assert_allclose(m[3] + m[12] + m[14], (e[:, 2] * e2 * f).sum(), atol=1e-14)
    # and m4 is the energy moment sum |e|^2 f
    np.testing.assert_allclose(m[4], (e2 * f).sum(), atol=1e-14)


def test_forcing_moments_match_guo_projection(oracle_lib, T):
    """Eq. (9) with sigma = 0: rows 0-15 equal M applied to the textbook
    discrete forcing term (rows 16-18 are the paper's own choice)."""
    rng = np.random.default_rng(3)
    e = T["e19"].astype(float)
    for _ in range(20):
        F = rng.uniform(-0.05, 0.05, 3)
        u = rng.uniform(-0.1, 0.1, 3)
        S = oracle_lib.forcing_moments(F, F, u, 1.0, sigma=0.0)
        np.testing.assert_allclose(S[:16], (T["M"] @ guo_forcing(F, u, e))[:16], atol=1e-15)


def test_forcing_and_equilibrium_worked_example(oracle_lib):
    """Hand-evaluated Eq. (5) and Eq. (9) at rho = 3, u = (0.1, 0, 0),
    F = F_m = (0.3, 0, 0), psi = 1, sigma = 0.1, tau_e = 1.25:
      varphi = 3/9 (1 - 0.015) = 0.328333..., m16 = m17 = varphi + 3/3*0.01,
      m18 = varphi, m10 = m12 = m14 = m15 = 0, m11 = m13 = 3(1/3)(0.1) = 0.1;
      S4 = 2*0.03 + 6*0.1*0.09/(1*0.75) = 0.132, S16 = S17 = 2/3*0.03 = 0.02,
      S18 = 0, S11 = S13 = 0.1."""
    meq = oracle_lib.equilibrium_moments(3.0, [0.1, 0.0, 0.0])
    vphi = 3.0 / 9.0 * (1 - 0.015)
    np.testing.assert_allclose(meq[[16, 17, 18]], [vphi + 0.01, vphi + 0.01, vphi], atol=1e-15)
    np.testing.assert_allclose(meq[[10, 11, 12, 13, 14, 15]], [0, 0.1, 0, 0.1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(meq[4], 3.03, atol=1e-15)
    S = oracle_lib.forcing_moments([0.3, 0, 0], [0.3, 0, 0], [0.1, 0, 0], 1.0, sigma=0.1, tau_e=1.25)
    np.testing.assert_allclose(S[4], 0.132, atol=1e-15)
    np.testing.assert_allclose(S[[16, 17, 18]], [0.02, 0.02, 0.0], atol=1e-15)
    np.testing.assert_allclose(S[[11, 13]], [0.1, 0.1], atol=1e-15)


def test_d3q7_N_and_inverse_match_eq38_eq41(T):
    np.testing.assert_array_equal(T["N"], load_matrix("d3q7_N.txt"))
    np.testing.assert_allclose(T["Ninv"] * 6.0, load_matrix("d3q7_Ninv_times6.txt"), atol=1e-13)


def test_d3q7_equilibrium_moments_eq42(T):
    """N (w T) = (T, 0, 0, 0, 3 c_sT^2 T, 0, 0) with c_sT^2 = d/3."""
    for Tv in (0.05, 0.07, 1.0):
        n = T["N"] @ (T["wT"] * Tv)
        np.testing.assert_allclose(n, [Tv, 0, 0, 0, 0.95 * Tv, 0, 0], atol=1e-15)


def test_cubic_group_maps_lattice_onto_itself(T):
    """Every one of the 48 cube symmetries permutes the D3Q19 velocity set;
    the symmetry test of the full solver relies on this."""
    e = [tuple(v) for v in T["e19"]]
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            img = {tuple(signs[i] * v[perm[i]] for i in range(3)) for v in e}
            assert img == set(e)
