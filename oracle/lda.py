"""LDA exchange on an atom-centred molecular grid (FP64, NumPy).

Test infrastructure only.  The paper names the local density approximation
as one choice of the exchange-correlation energy of the Kohn-Sham
Hamiltonian (section 5, batched H2 example); it does not fix the functional
or the grid.  Readings taken here (all restated in the design notes):

* Functional: Dirac-Slater exchange only, no correlation.  Energy density
  e_x(rho) = -C_x rho^(4/3) with C_x = (3/4)(3/pi)^(1/3); potential
  v_x = de_x/drho = -(3/pi)^(1/3) rho^(1/3).  Points where rho <= 0
  contribute nothing.
* Grid per atom: radial Gauss-Chebyshev quadrature of the second kind with
  75 nodes, x_i = cos(i pi / 76), mapped by r = r_m (1 + x) / (1 - x) with
  r_m = 1 bohr; angular product rule of 17 Gauss-Legendre nodes in
  cos(theta) times 34 equally spaced azimuths (578 directions).
* Becke fuzzy-cell partition: cell function s(mu) = (1 - f(f(f(mu)))) / 2,
  f(x) = (3x - x^3) / 2, mu_AB = (|r - A| - |r - B|) / |A - B|; the weight of
  atom A's point r is P_A(r) / sum_C P_C(r) with P_C = prod_{B != C} s(mu_CB);
  no atomic size adjustment.
* Point order: atom, then radial node i = 1..75, then theta node, then
  azimuth; point weight = radial weight x angular weight x Becke weight.

Matrices: rho_g = sum_{mu nu} Phi_{g mu} D_{mu nu} Phi_{g nu},
E_x = sum_g w_g e_x(rho_g), V_x = Phi^T diag(w v_x(rho)) Phi.
"""
from __future__ import annotations

import numpy as np

from . import core

N_RADIAL = 75
N_THETA = 17
N_PHI = 34
R_M = 1.0
C_X = 0.75 * (3.0 / np.pi) ** (1.0 / 3.0)


def radial_rule(n: int = N_RADIAL, rm: float = R_M):
    """Nodes r_i and weights for integrals int_0^inf F(r) r^2 dr.

    Second-kind Chebyshev: int_{-1}^{1} g(x) dx = sum_i pi/(n+1) sin(t_i) g(x_i)
    (the sin^2 weight of the rule divided by sqrt(1 - x^2)), t_i = i pi/(n+1);
    then r = rm (1+x)/(1-x), dr/dx = 2 rm / (1-x)^2.
    """
    i = np.arange(1, n + 1, dtype=np.float64)
    t = i * np.pi / (n + 1)
    x = np.cos(t)
    r = rm * (1.0 + x) / (1.0 - x)
    w = np.pi / (n + 1) * np.sin(t) * 2.0 * rm / (1.0 - x) ** 2 * r ** 2
    return r, w


def angular_rule(ntheta: int = N_THETA, nphi: int = N_PHI):
    """Unit directions [ntheta*nphi, 3] and weights summing to 4 pi."""
    u, a = np.polynomial.legendre.leggauss(ntheta)  # nodes in cos(theta)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - u * u)
    dirs = np.empty((ntheta, nphi, 3))
    dirs[:, :, 0] = st[:, None] * np.cos(phi)[None, :]
    dirs[:, :, 1] = st[:, None] * np.sin(phi)[None, :]
    dirs[:, :, 2] = u[:, None]
    w = np.repeat(a * (2.0 * np.pi / nphi), nphi)
    return dirs.reshape(-1, 3), w


def becke_s(mu):
    f = mu
    for _ in range(3):
        f = 1.5 * f - 0.5 * f ** 3
    return 0.5 * (1.0 - f)


def becke_weight(points: np.ndarray, centres: np.ndarray, owner: int) -> np.ndarray:
    """Becke weight of atom `owner` at each point [n, 3]."""
    d = np.linalg.norm(points[:, None, :] - centres[None, :, :], axis=2)  # [n, nat]
    nat = centres.shape[0]
    P = np.ones((points.shape[0], nat))
    for c in range(nat):
        for b in range(nat):
            if b == c:
                continue
            R = np.linalg.norm(centres[c] - centres[b])
            P[:, c] *= becke_s((d[:, c] - d[:, b]) / R)
    return P[:, owner] / P.sum(axis=1)


def n_points(mol) -> int:
    return len(mol.Z) * N_RADIAL * N_THETA * N_PHI


def grid_points(mol, index=None):
    """Points [n, 3] and weights [n] of the molecular grid (all, or the
    given point indices in the order described above)."""
    centres = np.asarray(mol.xyz, np.float64).reshape(-1, 3)
    r, wr = radial_rule()
    dirs, wa = angular_rule()
    nang = dirs.shape[0]
    per_atom = N_RADIAL * nang
    if index is None:
        index = np.arange(n_points(mol))
    index = np.asarray(index, np.int64)
    atom, rest = index // per_atom, index % per_atom
    ir, ia = rest // nang, rest % nang
    pts = centres[atom] + r[ir][:, None] * dirs[ia]
    w = wr[ir] * wa[ia]
    for a in np.unique(atom):
        sel = atom == a
        w[sel] *= becke_weight(pts[sel], centres, int(a))
    return pts, w


def _components(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def basis_values(mol, pts: np.ndarray) -> np.ndarray:
    """Phi[g, mu]: every contracted Cartesian function at every point."""
    coef = core.coefficients(mol)  # [nprim, 6], per component
    centres = np.asarray(mol.xyz, np.float64).reshape(-1, 3)
    out = np.zeros((pts.shape[0], mol.n_bf))
    p0 = 0
    bf = 0
    for s in range(len(mol.shell_l)):
        l, npr = int(mol.shell_l[s]), int(mol.shell_nprim[s])
        d = pts - centres[mol.shell_atom[s]]
        r2 = np.sum(d * d, axis=1)
        for c, (lx, ly, lz) in enumerate(_components(l)):
            radial = np.zeros(pts.shape[0])
            for p in range(npr):
                radial += coef[p0 + p, c] * np.exp(-mol.exps[p0 + p] * r2)
            out[:, bf + c] = d[:, 0] ** lx * d[:, 1] ** ly * d[:, 2] ** lz * radial
        p0 += npr
        bf += len(_components(l))
    return out


def exchange_terms(rho: np.ndarray):
    """(e_x, v_x) per point; zero where rho <= 0."""
    pos = rho > 0.0
    c = np.zeros_like(rho)
    c[pos] = np.cbrt(rho[pos])
    return -C_X * rho * c * pos, -(3.0 / np.pi) ** (1.0 / 3.0) * c


def lda_x(mol, D: np.ndarray, chunk: int = 20000, grid=None):
    """(E_x, V_x, rho) for density D (N x N); grid = (points, weights) or None."""
    pts, w = grid_points(mol) if grid is None else grid
    N = mol.n_bf
    V = np.zeros((N, N))
    E = 0.0
    rho_all = np.empty(pts.shape[0])
    for g0 in range(0, pts.shape[0], chunk):
        Phi = basis_values(mol, pts[g0:g0 + chunk])
        rho = np.einsum("gm,mn,gn->g", Phi, D, Phi, optimize=True)
        ex, vx = exchange_terms(rho)
        E += float(np.sum(w[g0:g0 + chunk] * ex))
        V += Phi.T @ ((w[g0:g0 + chunk] * vx)[:, None] * Phi)
        rho_all[g0:g0 + chunk] = rho
    return E, V, rho_all


def overlap_on_grid(mol, chunk: int = 20000, grid=None) -> np.ndarray:
    """S_grid = Phi^T diag(w) Phi (checks the grid against the analytic S)."""
    pts, w = grid_points(mol) if grid is None else grid
    S = np.zeros((mol.n_bf, mol.n_bf))
    for g0 in range(0, pts.shape[0], chunk):
        Phi = basis_values(mol, pts[g0:g0 + chunk])
        S += Phi.T @ (w[g0:g0 + chunk][:, None] * Phi)
    return S
