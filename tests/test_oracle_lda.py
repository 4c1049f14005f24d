"""Pins of the LDA-exchange oracle (oracle/lda.py) to things fixed by
mathematics rather than by the oracle itself: closed-form radial and
angular integrals, the Becke partition's defining properties, the analytic
overlap matrix, the exact exchange energy of one Gaussian, the derivative
relation V_x = dE_x/dD, translation invariance, and the closed-form LDA
energy of a one-function atom."""
import math

import numpy as np
import pytest

from mess_inputs import generators as G
from oracle import core, lda, scf


def test_radial_rule_gaussian_moments():
    r, w = lda.radial_rule()
    for a in (0.1, 1.0, 10.0):
        exact = math.sqrt(math.pi) / (4.0 * a ** 1.5)  # int_0^inf r^2 exp(-a r^2) dr
        assert abs(np.sum(w * np.exp(-a * r * r)) / exact - 1.0) < 1e-10
    # int_0^inf r^2 exp(-r) dr = 2
    assert abs(np.sum(w * np.exp(-r)) - 2.0) < 1e-8


def _sphere_monomial(a, b, c):
    """int over the unit sphere of x^a y^b z^c."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    return 2.0 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)


def test_angular_rule_exact_on_monomials():
    d, w = lda.angular_rule()
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    for a in range(0, 9):
        for b in range(0, 9 - a):
            for c in range(0, 9 - a - b):
                got = np.sum(w * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c)
                assert abs(got - _sphere_monomial(a, b, c)) < 1e-13, (a, b, c)


def test_becke_partition():
    mol = G.random_small_molecule(1)
    centres = np.asarray(mol.xyz).reshape(-1, 3)
    rng = np.random.Generator(np.random.PCG64(5))
    pts = rng.uniform(-6, 6, size=(300, 3))
    tot = sum(lda.becke_weight(pts, centres, a) for a in range(len(centres)))
    assert np.abs(tot - 1.0).max() < 1e-14
    # a nucleus belongs wholly to its own cell
    for a in range(len(centres)):
        assert abs(lda.becke_weight(centres[a:a + 1], centres, a)[0] - 1.0) < 1e-15
    # cell function: s(-mu) = 1 - s(mu), s(-1) = 1, s(1) = 0
    mu = np.linspace(-1, 1, 41)
    assert np.abs(lda.becke_s(-mu) - (1.0 - lda.becke_s(mu))).max() < 1e-15
    assert lda.becke_s(np.array([-1.0]))[0] == 1.0 and lda.becke_s(np.array([1.0]))[0] == 0.0


def test_grid_order_and_subset():
    mol = G.random_small_molecule(2, n_atoms=3)
    pts, w = lda.grid_points(mol)
    assert pts.shape == (lda.n_points(mol), 3)
    idx = np.array([0, 1, 577, 578, 43349, 43350, 2 * 43350 + 12345, lda.n_points(mol) - 1])
    p2, w2 = lda.grid_points(mol, idx)
    assert np.array_equal(p2, pts[idx]) and np.array_equal(w2, w[idx])
    # first point of atom 0: largest radius, first theta node, azimuth 0
    r, _ = lda.radial_rule()
    dirs, _ = lda.angular_rule()
    assert np.allclose(pts[0], np.asarray(mol.xyz).reshape(-1, 3)[0] + r[0] * dirs[0], rtol=0, atol=1e-12)


def test_overlap_on_grid_matches_analytic():
    mol = G.random_small_molecule(1)
    S, _, _ = core.one_electron(mol)
    Sg = lda.overlap_on_grid(mol)
    # grid error: tight exponents (up to 5000) limit the 75-node radial rule
    assert np.abs(Sg - S).max() < 1e-5


def test_exchange_energy_of_one_gaussian_closed_form():
    for alpha in (0.5, 1.0, 2.0):
        mol = G.single_gaussian_system("He", alpha)
        D = np.array([[2.0]])
        Ex, V, rho = lda.lda_x(mol, D)
        # rho = 2 phi^2, phi = (2a/pi)^(3/4) exp(-a r^2):
        # int rho^(4/3) = 2^(4/3) (2a/pi)^2 (3 pi / (8 a))^(3/2)
        exact = -lda.C_X * 2 ** (4 / 3) * (2 * alpha / math.pi) ** 2 * (3 * math.pi / (8 * alpha)) ** 1.5
        assert abs(Ex / exact - 1.0) < 1e-10, alpha
        # V_11 = int v_x phi^2 = (4/3) E_x / 2 for this one-function density
        assert abs(V[0, 0] / (2.0 / 3.0 * exact) - 1.0) < 1e-10


def _psd_density(n, nocc, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    C = rng.normal(size=(n, nocc)) / math.sqrt(n)
    return 2.0 * C @ C.T


def test_potential_is_derivative_of_energy():
    mol = G.random_small_molecule(4, n_atoms=3)
    grid = lda.grid_points(mol)
    D = _psd_density(mol.n_bf, 4, 1)
    _, V, _ = lda.lda_x(mol, D, grid=grid)
    for (i, j) in ((0, 0), (2, 5), (7, 3)):
        E1 = np.zeros_like(D)
        E1[i, j] += 1.0
        if i != j:
            E1[j, i] += 1.0
        h = 1e-4
        ep = lda.lda_x(mol, D + h * E1, grid=grid)[0]
        em = lda.lda_x(mol, D - h * E1, grid=grid)[0]
        fd = (ep - em) / (2 * h)
        want = V[i, j] * (1 if i == j else 2)
        assert abs(fd - want) <= 1e-7 * max(1.0, abs(want)), (i, j, fd, want)


def test_translation_invariance():
    mol = G.random_small_molecule(4, n_atoms=3)
    D = _psd_density(mol.n_bf, 4, 2)
    E0, V0, _ = lda.lda_x(mol, D)
    m2 = mol.copy()
    m2.xyz = np.asarray(mol.xyz, np.float64) + np.array([0.3, -0.2, 0.7])
    E1, V1, _ = lda.lda_x(m2, D)
    assert abs(E1 - E0) < 1e-11 * abs(E0)
    assert np.abs(V1 - V0).max() < 1e-11 * np.abs(V0).max()


def test_electron_count_on_grid():
    mol = G.random_small_molecule(1)
    rhf = scf.RHF(mol)
    D = rhf.core_guess()
    assert abs(np.sum(D * rhf.S) - mol.n_electrons) < 1e-10
    pts, w = lda.grid_points(mol)
    _, _, rho = lda.lda_x(mol, D, grid=(pts, w))
    assert abs(np.sum(w * rho) - mol.n_electrons) < 1e-4


def test_lda_scf_one_function_atom_closed_form():
    alpha, Z = 0.8, 2
    mol = G.single_gaussian_system("He", alpha)
    r = scf.RHF(mol, xc="lda", conv_tol=1e-12, max_iter=5).run()
    T = 1.5 * alpha
    Vn = -Z * 2.0 * math.sqrt(2 * alpha / math.pi)
    J11 = 2.0 * math.sqrt(alpha / math.pi)
    Ex = -lda.C_X * 2 ** (4 / 3) * (2 * alpha / math.pi) ** 2 * (3 * math.pi / (8 * alpha)) ** 1.5
    exact = 2.0 * (T + Vn) + 2.0 * J11 + Ex  # Tr[DH] + 1/2 Tr[DJ] + E_x, D = [[2]]
    assert abs(r["energies"][0] - exact) < 1e-10
    assert r["converged"]
