"""Restricted Hartree-Fock SCF oracle (FP64, NumPy/LAPACK).

Test infrastructure only.  Follows paper section 3: the Roothaan equation
F(C) C = S C eps (eq. 2) is solved by fixed-point (self-consistent field)
iteration until the energy stops changing; C holds the LCAO coefficients of
eq. 1, orthonormal in the metric S (eq. 5).  Readings where the paper is
silent (all restated in the design notes):

* Fock and energy (closed shell, total density D = 2 C_occ C_occ^T):
  F = H + J - K/2,  E = 1/2 Tr[D (H + F)] + E_nuc  (E_nuc added to the
  electronic energy as in the paper's examples).
* Orthogonaliser: canonical, X = U s^{-1/2} over eigenpairs of S with
  s > 1e-7.
* Initial guess: core Hamiltonian (diagonalise X^T H X), or a supplied D0.
* Acceleration: optional Pulay DIIS over at most 8 Fock matrices, applied
  once two are stored, error vector X^T (F D S - S D F) X.
* Convergence: |E_k - E_{k-1}| < conv_tol, or a fixed iteration count.
* Divergence guard (on by default): from the 12th iteration on (index
  k >= 12, so that DIIS may overshoot while it settles), a rise of the
  energy by more than 1e-6 Ha counts against the current stage; the second such rise since the
  stage began moves to the next stage, and a non-finite energy jumps to the
  last.  Every stage change clears the DIIS history.  Stages: 0 DIIS;
  1 DIIS afresh; 2 DIIS with damping 0.5 (the next density mixed half and
  half with the current one); 3 restart from the core-Hamiltonian guess,
  damped as in stage 2 (the last stage).  The first energy after a restart
  is compared with nothing.
* LDA (xc="lda"): exchange from the Dirac-Slater functional on the
  molecular grid of ``lda.py`` instead of K:  F = H + J + V_x,
  E = Tr[D H] + 1/2 Tr[D J] + E_x + E_nuc.
* PBE (xc="pbe"): the PBE exchange-correlation of ``pbe.py`` on the same
  grid:  F = H + J + V_xc,  E = Tr[D H] + 1/2 Tr[D J] + E_xc + E_nuc.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import lda as olda
from . import pbe as opbe


def canonical_orthogonaliser(S: np.ndarray, thresh: float = 1e-7) -> np.ndarray:
    s, U = np.linalg.eigh(S)
    keep = s > thresh
    return U[:, keep] / np.sqrt(s[keep])


def density_from_fock(F: np.ndarray, X: np.ndarray, n_occ: int):
    """Solve eq. 2 for fixed F in the orthonormal basis; aufbau occupation."""
    eps, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    Cocc = C[:, :n_occ]
    return 2.0 * Cocc @ Cocc.T, C, eps


def fock_and_energy(H, J, K, D, e_nuc):
    F = H + J - 0.5 * K
    E = 0.5 * float(np.sum(D * (H + F))) + e_nuc
    return F, E


def diis_extrapolate(focks, errors):
    m = len(focks)
    B = np.zeros((m + 1, m + 1))
    for i in range(m):
        for j in range(m):
            B[i, j] = float(np.sum(errors[i] * errors[j]))
    B[:m, m] = B[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(B, rhs)[:m]
    return sum(ci * Fi for ci, Fi in zip(c, focks))


class RHF:
    """Closed-shell SCF driven by oracle integrals.

    jk: 'dense' (full tensor + the defining einsums; small systems) or
    'unique' (8-fold unique quartets, optional Schwarz threshold tau).
    """

    def __init__(self, mol, jk: str = "dense", tau: float = 0.0, diis: bool = True,
                 diis_size: int = 8, conv_tol: float = 1e-8, max_iter: int = 100,
                 fixed_iters: int | None = None, xc: str = "hf", guard: bool = True):
        if mol.n_electrons % 2:
            raise ValueError("closed-shell SCF needs an even electron count")
        self.mol = mol
        self.S, self.T, self.V = core.one_electron(mol)
        self.H = self.T + self.V
        self.e_nuc = core.nuclear_repulsion(mol)
        self.X = canonical_orthogonaliser(self.S)
        self.n_occ = mol.n_electrons // 2
        self.jk_mode, self.tau = jk, tau
        self.diis, self.diis_size = diis, diis_size
        self.guard = guard
        self.conv_tol, self.max_iter, self.fixed_iters = conv_tol, max_iter, fixed_iters
        self._eri = core.eri_dense(mol) if jk == "dense" else None
        if xc not in ("hf", "lda", "pbe"):
            raise ValueError(xc)
        self.xc = xc
        self._grid = olda.grid_points(mol) if xc in ("lda", "pbe") else None

    def fock(self, D):
        """(F, E) at density D for the chosen exchange."""
        J, K = self.jk(D)
        if self.xc == "hf":
            return fock_and_energy(self.H, J, K, D, self.e_nuc)
        if self.xc == "pbe":
            Ex, Vx = opbe.pbe_xc(self.mol, D, grid=self._grid)[:2]
        else:
            Ex, Vx, _ = olda.lda_x(self.mol, D, grid=self._grid)
        F = self.H + J + Vx
        E = float(np.sum(D * self.H)) + 0.5 * float(np.sum(D * J)) + Ex + self.e_nuc
        return F, E

    def jk(self, D):
        if self.jk_mode == "dense":
            return core.jk_from_dense(self._eri, D)
        J, K, _ = core.jk_unique(self.mol, D, self.tau)
        return J, K

    def core_guess(self):
        return density_from_fock(self.H, self.X, self.n_occ)[0]

    def step(self, D):
        """One undamped Roothaan step: D_k -> (F_k, E_k, D_{k+1})."""
        F, E = self.fock(D)
        Dn = density_from_fock(F, self.X, self.n_occ)[0]
        return F, E, Dn

    def commutator(self, F, D):
        return self.X.T @ (F @ D @ self.S - self.S @ D @ F) @ self.X

    RISE_TOL = 1e-6
    RISES_PER_STAGE = 2
    GUARD_FROM = 12
    DAMP = 0.5

    def run(self, D0=None, record=False):
        D = self.core_guess() if D0 is None else np.array(D0, dtype=np.float64)
        energies, focks, errors = [], [], []
        densities, fock_hist, stages = [], [], []
        converged = False
        n_iter = self.fixed_iters if self.fixed_iters is not None else self.max_iter
        F = None
        stage, rises, e_prev = 0, 0, None
        for k in range(n_iter):
            F, E = self.fock(D)
            D_used = D
            energies.append(E)
            stages.append(stage)
            if record:
                densities.append(D)
                fock_hist.append(F)
            if self.fixed_iters is None and e_prev is not None and abs(E - e_prev) < self.conv_tol:
                converged = True
                break
            if self.guard:
                up = 0
                if not np.isfinite(E):
                    up = 3 - stage
                elif e_prev is not None and k >= self.GUARD_FROM and E > e_prev + self.RISE_TOL:
                    rises += 1
                    if rises >= self.RISES_PER_STAGE:
                        up = 1
                if up > 0 and stage < 3:
                    stage, rises = min(3, stage + up), 0
                    focks, errors = [], []
                    if stage == 3:
                        D, e_prev = self.core_guess(), None
                        continue
                elif not np.isfinite(E):
                    raise FloatingPointError("SCF energy is not finite after a restart")
            e_prev = E
            Fx = F
            if self.diis:
                focks.append(F)
                errors.append(self.commutator(F, D))
                if len(focks) > self.diis_size:
                    focks.pop(0)
                    errors.pop(0)
                if len(focks) >= 2:
                    Fx = diis_extrapolate(focks, errors)
            Dn, C, eps = density_from_fock(Fx, self.X, self.n_occ)
            D = Dn if stage < 2 else (1.0 - self.DAMP) * Dn + self.DAMP * D
        if self.fixed_iters is not None:
            converged = True
        return {"energy": energies[-1], "energies": energies, "D": D_used, "D_next": D, "F": F,
                "converged": converged, "iterations": len(energies), "stages": stages,
                "e_nuc": self.e_nuc, "densities": densities, "focks": fock_hist}
