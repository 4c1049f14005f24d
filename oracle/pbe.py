"""PBE exchange-correlation on the molecular grid (FP64, NumPy).

Test infrastructure only.  The paper selects the PBE generalised-gradient
functional (Perdew, Burke and Ernzerhof 1996) through its Hamiltonian's
exchange-correlation option (section 5) and evaluates the density gradient
it needs by automatic differentiation.  Here the functional is written out
for a closed-shell (spin-unpolarised) density, in Hartree atomic units, from
its published definition:

* k_F = (3 pi^2 rho)^(1/3), r_s = (3 / (4 pi rho))^(1/3), sigma = |grad rho|^2.
* Exchange: e_x = rho eps_x^unif F_x(s), eps_x^unif = -3 k_F / (4 pi),
  s^2 = sigma / (4 k_F^2 rho^2), F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa),
  kappa = 0.804, mu = beta pi^2 / 3.
* Correlation: e_c = rho (eps_c^unif(r_s) + H), with eps_c^unif the
  Perdew-Wang (1992) parametrisation of the paramagnetic electron gas,
  G(r_s) = -2 A (1 + a1 r_s) ln(1 + 1 / (2 A (b1 r_s^(1/2) + b2 r_s
  + b3 r_s^(3/2) + b4 r_s^2))), A = 0.031091, a1 = 0.21370, b1 = 7.5957,
  b2 = 3.5876, b3 = 1.6382, b4 = 0.49294; and
  H = gamma ln(1 + (beta/gamma) t^2 (1 + A' t^2) / (1 + A' t^2 + A'^2 t^4)),
  A' = (beta/gamma) / (exp(-eps_c^unif / gamma) - 1), t^2 = sigma / (4 k_s^2 rho^2),
  k_s^2 = 4 k_F / pi, gamma = (1 - ln 2) / pi^2, beta = 0.06672455060314922.
* Readings (restated in the design notes): points with rho < 1e-10 add
  nothing (the gradient terms of the far tails are not evaluated); the grid
  is the one of ``lda.py``; grad rho = 2 sum_{mu nu} D_{mu nu} phi_mu grad phi_nu
  with the basis gradients written out analytically.

E_xc = sum_g w_g f(rho_g, sigma_g), and the Kohn-Sham matrix is
V_{mu nu} = dE_xc / dD_{mu nu}
          = sum_g w_g [f_rho phi_mu phi_nu + 2 f_sigma grad rho . grad(phi_mu phi_nu)].
The partial derivatives f_rho, f_sigma are taken by complex-step
differentiation of f (f(x + i h) = f(x) + i h f'(x) + O(h^2), no
subtraction), so the oracle needs no hand-derived derivative formulas.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import lda as olda

KAPPA = 0.804
BETA = 0.06672455060314922
MU = BETA * np.pi ** 2 / 3.0
GAMMA = (1.0 - np.log(2.0)) / np.pi ** 2
PW_A, PW_A1 = 0.031091, 0.21370
PW_B = (7.5957, 3.5876, 1.6382, 0.49294)
RHO_MIN = 1e-10


def pw92(rs):
    """Perdew-Wang correlation energy per electron of the paramagnetic gas."""
    q = 2.0 * PW_A * (PW_B[0] * np.sqrt(rs) + PW_B[1] * rs + PW_B[2] * rs ** 1.5 + PW_B[3] * rs * rs)
    return -2.0 * PW_A * (1.0 + PW_A1 * rs) * np.log1p(1.0 / q)


def fx(s2):
    """PBE exchange enhancement factor as a function of s^2."""
    return 1.0 + KAPPA - KAPPA / (1.0 + MU * s2 / KAPPA)


def pbe_h(ec, t2):
    """PBE gradient correction to the correlation energy per electron."""
    a = (BETA / GAMMA) / np.expm1(-ec / GAMMA)
    y = a * t2
    return GAMMA * np.log1p((BETA / GAMMA) * t2 * (1.0 + y) / (1.0 + y + y * y))


def energy_density(rho, sigma):
    """f(rho, sigma) = e_x + e_c per unit volume (real or complex arguments;
    callers pass only rho >= RHO_MIN)."""
    kf = (3.0 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    rs = (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)
    s2 = sigma / (4.0 * kf * kf * rho * rho)
    ex = rho * (-3.0 * kf / (4.0 * np.pi)) * fx(s2)
    ec_unif = pw92(rs)
    ks2 = 4.0 * kf / np.pi
    t2 = sigma / (4.0 * ks2 * rho * rho)
    return ex + rho * (ec_unif + pbe_h(ec_unif, t2))


def derivatives(rho, sigma):
    """(f, df/drho, df/dsigma) per point by complex step; zero below RHO_MIN."""
    rho = np.asarray(rho, np.float64)
    sigma = np.asarray(sigma, np.float64)
    f = np.zeros_like(rho)
    fr = np.zeros_like(rho)
    fs = np.zeros_like(rho)
    ok = rho >= RHO_MIN
    r, s = rho[ok], sigma[ok]
    hr = 1e-30 * r
    hs = 1e-30 * np.maximum(s, r ** (8.0 / 3.0))
    f[ok] = energy_density(r, s)
    fr[ok] = np.imag(energy_density(r + 1j * hr, s.astype(np.complex128))) / hr
    fs[ok] = np.imag(energy_density(r.astype(np.complex128), s + 1j * hs)) / hs
    return f, fr, fs


def basis_gradients(mol, pts: np.ndarray):
    """(Phi[g, mu], dPhi[3, g, mu]): values and Cartesian gradients of every
    contracted function; d/dx (x^l e^{-a r^2}) = (l x^{l-1} - 2 a x^{l+1}) e^{-a r^2}."""
    coef = core.coefficients(mol)
    centres = np.asarray(mol.xyz, np.float64).reshape(-1, 3)
    G = pts.shape[0]
    phi = np.zeros((G, mol.n_bf))
    dphi = np.zeros((3, G, mol.n_bf))
    p0 = bf = 0
    for s in range(len(mol.shell_l)):
        l, npr = int(mol.shell_l[s]), int(mol.shell_nprim[s])
        d = pts - centres[mol.shell_atom[s]]
        r2 = np.sum(d * d, axis=1)
        for c, lmn in enumerate(olda._components(l)):
            rad = np.zeros(G)
            drad = np.zeros(G)  # sum c a e^{-a r^2}
            for p in range(npr):
                e = np.exp(-mol.exps[p0 + p] * r2)
                rad += coef[p0 + p, c] * e
                drad += coef[p0 + p, c] * mol.exps[p0 + p] * e
            mono = d[:, 0] ** lmn[0] * d[:, 1] ** lmn[1] * d[:, 2] ** lmn[2]
            phi[:, bf + c] = mono * rad
            for k in range(3):
                lower = np.zeros(G)
                if lmn[k] > 0:
                    e = list(lmn)
                    e[k] -= 1
                    lower = lmn[k] * d[:, 0] ** e[0] * d[:, 1] ** e[1] * d[:, 2] ** e[2]
                dphi[k, :, bf + c] = lower * rad - 2.0 * d[:, k] * mono * drad
        p0 += npr
        bf += len(olda._components(l))
    return phi, dphi


def density_and_gradient(D, phi, dphi):
    """rho[g] and grad rho[3, g] for a symmetric density D."""
    U = phi @ D
    rho = np.sum(U * phi, axis=1)
    grad = 2.0 * np.einsum("gn,kgn->kg", U, dphi)
    return rho, grad


def pbe_xc(mol, D: np.ndarray, chunk: int = 20000, grid=None):
    """(E_xc, V_xc, rho, grad rho) for density D on the molecular grid."""
    pts, w = olda.grid_points(mol) if grid is None else grid
    N = mol.n_bf
    V = np.zeros((N, N))
    E = 0.0
    rho_all = np.empty(pts.shape[0])
    grad_all = np.empty((3, pts.shape[0]))
    for g0 in range(0, pts.shape[0], chunk):
        sl = slice(g0, g0 + chunk)
        phi, dphi = basis_gradients(mol, pts[sl])
        rho, grad = density_and_gradient(D, phi, dphi)
        sigma = np.sum(grad * grad, axis=0)
        f, fr, fs = derivatives(rho, sigma)
        wg = w[sl]
        E += float(np.sum(wg * f))
        # Z_nu(g) = w (f_rho phi_nu / 2 + 2 f_sigma grad rho . grad phi_nu); V = Phi^T Z + Z^T Phi
        Z = (0.5 * wg * fr)[:, None] * phi + np.einsum("kg,kgn->gn", (2.0 * wg * fs)[None, :] * grad, dphi)
        M = phi.T @ Z
        V += M + M.T
        rho_all[sl] = rho
        grad_all[:, sl] = grad
    return E, V, rho_all, grad_all
