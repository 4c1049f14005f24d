"""Pins of the oracle's PBE exchange-correlation (CPU).

What the PBE construction and the electron-gas limits fix, independently of
how the oracle evaluates the formulas:

* exchange: F_x(0) = 1 (the gradient-free limit is the Dirac-Slater exchange
  of the LDA oracle), F_x -> 1 + kappa for large s (the Lieb-Oxford cap the
  construction imposes), F_x = 1 + mu s^2 + O(s^4) with mu = beta pi^2 / 3;
* Perdew-Wang correlation: c0 = (1 - ln 2)/pi^2 = 0.0310907 and c1 = 0.046644
  in the high-density limit eps = c0 ln r_s - c1, and -d0 / r_s with
  d0 = 0.4335 at low density (the constants the parametrisation is built
  from);
* gradient correction: H = beta t^2 + O(t^4) for slowly varying densities,
  and H -> -eps_c^unif for rapidly varying ones (correlation vanishes);
* the complex-step partial derivatives agree with central differences;
* V_xc = dE_xc/dD: E_xc along a symmetric density direction agrees with
  Tr[V_xc Delta] to central-difference accuracy, on a water molecule with
  s, p and d functions; V_xc symmetric; the grid integrates rho to N_e.
"""
import numpy as np
import pytest

from mess_inputs import generators as G
from oracle import lda as olda
from oracle import pbe
from oracle import scf as oscf


def test_exchange_limits():
    assert pbe.fx(0.0) == 1.0
    assert abs(pbe.fx(1e30) - (1.0 + pbe.KAPPA)) < 1e-15
    for s2 in (1e-6, 1e-8):
        assert abs((pbe.fx(s2) - 1.0) / s2 - pbe.MU) < 1e-5 * pbe.MU
    assert abs(pbe.MU - 0.2195149727645171) < 1e-15
    # sigma = 0: PBE exchange is the LDA oracle's Dirac-Slater exchange
    rho = np.array([1e-6, 3e-3, 0.2, 7.0, 450.0])
    rs = (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)
    ex = pbe.energy_density(rho, np.zeros_like(rho)) - rho * pbe.pw92(rs)
    ex_lda, _ = olda.exchange_terms(rho)
    assert np.max(np.abs(ex - ex_lda) / np.abs(ex_lda)) < 1e-14


def test_pw92_limits():
    assert abs(pbe.PW_A - (1.0 - np.log(2.0)) / np.pi ** 2) < 1e-6
    for rs in (1e-7, 1e-9):
        assert abs(pbe.pw92(rs) - pbe.PW_A * np.log(rs) - (-0.046644)) < 2e-6
    rs = 1e9
    assert abs(pbe.pw92(rs) * rs + 0.4335) < 1e-4
    # negative and increasing toward zero with r_s
    r = np.geomspace(1e-3, 1e3, 50)
    e = pbe.pw92(r)
    assert np.all(e < 0) and np.all(np.diff(e) > 0)


def test_gradient_correction_limits():
    for ec in (-0.1, -0.03, -0.005):
        for t2 in (1e-8, 1e-10):
            assert abs(pbe.pbe_h(ec, t2) / t2 - pbe.BETA) < 1e-6
        assert abs(pbe.pbe_h(ec, 1e12) + ec) < 1e-9
        t = np.geomspace(1e-3, 1e3, 40)
        h = pbe.pbe_h(ec, t * t)
        assert np.all(h > 0) and np.all(np.diff(h) > 0) and np.all(h < -ec)


def test_complex_step_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(3))
    rho = 10.0 ** rng.uniform(-8, 2, 40)
    sigma = rho ** (8.0 / 3.0) * 10.0 ** rng.uniform(-3, 2, 40)
    f, fr, fs = pbe.derivatives(rho, sigma)
    # fourth-order central differences in extended precision (the
    # sigma-dependent part can be a small share of f, so FP64 differences
    # would be dominated by rounding)
    def d4(fun, x, h):
        x, h = np.longdouble(x), np.longdouble(h)
        return float((8 * (fun(x + h) - fun(x - h)) - (fun(x + 2 * h) - fun(x - 2 * h))) / (12 * h))

    for i in range(40):
        r0, s0 = np.longdouble(rho[i]), np.longdouble(sigma[i])
        d = d4(lambda r: pbe.energy_density(r, s0), r0, 1e-3 * r0)
        assert abs(d - fr[i]) < 1e-8 * abs(fr[i]), i
        d = d4(lambda s: pbe.energy_density(r0, s), s0, 1e-2 * s0)
        assert abs(d - fs[i]) < 1e-7 * abs(fs[i]), i
    # below the density cut-off: nothing
    f0, fr0, fs0 = pbe.derivatives(np.array([5e-11, 0.0, -1e-3]), np.array([1.0, 0.0, 2.0]))
    assert not np.any(f0) and not np.any(fr0) and not np.any(fs0)


def test_basis_gradients_by_differences():
    mol = G.water_cluster(0, n_waters=1)
    rng = np.random.Generator(np.random.PCG64(5))
    pts = np.asarray(mol.xyz).reshape(-1, 3)[0] + rng.normal(0.0, 1.0, (25, 3))
    phi, dphi = pbe.basis_gradients(mol, pts)
    assert np.array_equal(phi, olda.basis_values(mol, pts))
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (olda.basis_values(mol, pts + e) - olda.basis_values(mol, pts - e)) / (2 * h)
        assert np.max(np.abs(fd - dphi[k])) < 1e-6 * max(1.0, np.max(np.abs(dphi[k])))


@pytest.fixture(scope="module")
def water():
    mol = G.water_cluster(0, n_waters=1)
    D = oscf.RHF(mol, jk="dense", conv_tol=1e-9).run()["D"]
    grid = olda.grid_points(mol)
    return mol, D, grid


def test_vxc_is_the_energy_derivative(water):
    mol, D, grid = water
    E, V, rho, grad = pbe.pbe_xc(mol, D, grid=grid)
    assert np.max(np.abs(V - V.T)) < 1e-12 * np.max(np.abs(V))
    assert abs(np.sum(grid[1] * rho) - mol.n_electrons) < 1e-4
    assert E < 0
    rng = np.random.Generator(np.random.PCG64(9))
    A = rng.normal(size=D.shape)
    Delta = 0.5 * (A + A.T) * 1e-2
    eps = 1e-4
    Ep = pbe.pbe_xc(mol, D + eps * Delta, grid=grid)[0]
    Em = pbe.pbe_xc(mol, D - eps * Delta, grid=grid)[0]
    fd = (Ep - Em) / (2 * eps)
    an = float(np.sum(V * Delta))
    assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
