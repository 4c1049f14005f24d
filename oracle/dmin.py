"""Direct minimisation of the closed-shell energy over orthonormal orbitals
(oracle, FP64 NumPy).  Test infrastructure only.

Follows paper section 3 (direct minimisation of E(C) subject to the
orthonormality constraint of eq. 5, C^T S C = 1) with the constraint
enforced by QR orthonormalisation of an unconstrained trial matrix Z, and
the first-order Adam optimiser of section 5.1 (Z = 1 initially).  Reading of
the parts the paper leaves open (restated in the design notes):

* C = X Q with X = S^{-1/2} (Loewdin; X^T S X = 1) and Z = Q R the QR
  decomposition of the square trial matrix, so C^T S C = Q^T Q = 1 for any
  non-singular Z.  The occupied orbitals are the first n_occ columns of C;
  D = 2 C_occ C_occ^T; E(Z) = 1/2 Tr[D (H + F)] + E_nuc with F = H + J - K/2.
* Gradient: dE/dC_occ = 4 F C_occ (F is dE/dD for D = 2 C C^T); through
  C = X Q, Qbar = X^T Cbar; through Z = Q R (R upper triangular, any sign
  convention) with no dependence on R, Zbar = Q tril(B^T - B, -1) R^{-T}
  with B = Qbar^T Q (derived from dZ = dQ R + Q dR with Q^T dQ
  antisymmetric and dR R^{-1} upper triangular).
* Adam: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  Z <- Z - lr mhat / (sqrt(vhat) + eps), bias-corrected, b1 = 0.9,
  b2 = 0.999, eps = 1e-8.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import scf as oscf


def lowdin(S: np.ndarray) -> np.ndarray:
    s, U = np.linalg.eigh(S)
    return (U / np.sqrt(s)) @ U.T


def qr_grad(Q: np.ndarray, R: np.ndarray, Qbar: np.ndarray) -> np.ndarray:
    """Gradient with respect to Z of a function of Q alone, Z = Q R square."""
    B = Qbar.T @ Q
    W = np.tril(B.T - B, -1)
    return np.linalg.solve(R, (Q @ W).T).T   # (Q W) R^{-T}


class DirectMin:
    """E(Z) and its gradient for one molecule; J/K from the dense tensor
    (small systems) or unique quartets."""

    def __init__(self, mol, jk: str = "dense", tau: float = 0.0):
        self.mol = mol
        self.S, T, V = core.one_electron(mol)
        self.H = T + V
        self.e_nuc = core.nuclear_repulsion(mol)
        self.X = lowdin(self.S)
        self.n_occ = mol.n_electrons // 2
        self.jk_mode, self.tau = jk, tau
        self._eri = core.eri_dense(mol) if jk == "dense" else None

    def jk(self, D):
        if self.jk_mode == "dense":
            return core.jk_from_dense(self._eri, D)
        J, K, _ = core.jk_unique(self.mol, D, self.tau)
        return J, K

    def energy_and_grad(self, Z: np.ndarray):
        Q, R = np.linalg.qr(Z)
        C = self.X @ Q
        Co = C[:, :self.n_occ]
        D = 2.0 * Co @ Co.T
        J, K = self.jk(D)
        F, E = oscf.fock_and_energy(self.H, J, K, D, self.e_nuc)
        Cbar = np.zeros_like(C)
        Cbar[:, :self.n_occ] = 4.0 * F @ Co
        Qbar = self.X.T @ Cbar
        return E, qr_grad(Q, R, Qbar), D

    def energy(self, Z: np.ndarray) -> float:
        return self.energy_and_grad(Z)[0]


class Adam:
    def __init__(self, shape, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(shape)
        self.v = np.zeros(shape)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, Z, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return Z - self.lr * mh / (np.sqrt(vh) + self.eps)


def minimise(mol, steps: int = 200, lr: float = 0.1, jk: str = "dense", tau: float = 0.0, Z0=None):
    """Adam on E(Z) from Z = 1; returns the energies of every step (before
    its update), the final Z and density."""
    dm = DirectMin(mol, jk=jk, tau=tau)
    N = mol.n_bf
    Z = np.eye(N) if Z0 is None else np.array(Z0, dtype=np.float64)
    opt = Adam(Z.shape, lr)
    energies = []
    D = None
    for _ in range(steps):
        E, g, D = dm.energy_and_grad(Z)
        energies.append(E)
        Z = opt.step(Z, g)
    return {"energies": energies, "Z": Z, "D": D, "energy": energies[-1]}
