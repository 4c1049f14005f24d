"""Nuclear gradient of the closed-shell Hartree-Fock energy (oracle, FP64).
Test infrastructure only.

The paper lists atomic-force evaluation among the uses of its end-to-end
differentiable energy (section 1; its gradient transformation, section 4).
The oracle takes the plainest route to dE/dR_A that needs no derivative
integrals at all: central differences of the converged oracle energy,
with the basis functions moving with their atoms,

  dE/dx ~ [8 (E(x + h) - E(x - h)) - (E(x + 2h) - E(x - 2h))] / (12 h),

h = 5e-3 bohr (truncation O(h^4)), every displaced SCF converged to
|dE| < 1e-12 Ha from the undisplaced converged density (the converged
energy does not depend on the starting point).  The nuclear repulsion part
has the closed form -sum_B Z_A Z_B (R_A - R_B) / |R_A - R_B|^3, given for
tests.
"""
from __future__ import annotations

import numpy as np

from . import core
from . import scf as oscf

STEP = 5e-3


def displaced(mol, atom: int, axis: int, h: float):
    m = mol.copy()
    m.xyz = np.array(mol.xyz, dtype=np.float64).reshape(-1, 3).copy()
    m.xyz[atom, axis] += h
    return m


def energy(mol, D0=None, conv_tol: float = 1e-12) -> float:
    r = oscf.RHF(mol, jk="dense", conv_tol=conv_tol, max_iter=300).run(D0=D0)
    if not r["converged"]:
        raise RuntimeError("oracle SCF did not converge")
    return r["energy"]


def fd_gradient(mol, h: float = STEP, conv_tol: float = 1e-12) -> np.ndarray:
    """[n_atoms, 3] dE/dR by fourth-order central differences."""
    ref = oscf.RHF(mol, jk="dense", conv_tol=conv_tol, max_iter=300).run()
    D0 = ref["D"]
    nat = len(mol.Z)
    g = np.zeros((nat, 3))
    for a in range(nat):
        for k in range(3):
            e = {s: energy(displaced(mol, a, k, s * h), D0, conv_tol) for s in (-2, -1, 1, 2)}
            g[a, k] = (8.0 * (e[1] - e[-1]) - (e[2] - e[-2])) / (12.0 * h)
    return g


def nuclear_repulsion_gradient(mol) -> np.ndarray:
    xyz = np.asarray(mol.xyz, np.float64).reshape(-1, 3)
    Z = np.asarray(mol.Z, np.float64)
    g = np.zeros_like(xyz)
    for a in range(len(Z)):
        for b in range(len(Z)):
            if a != b:
                d = xyz[a] - xyz[b]
                g[a] -= Z[a] * Z[b] * d / np.linalg.norm(d) ** 3
    return g


def converged(mol, conv_tol: float = 1e-12):
    """(D, F, E) of the converged oracle SCF (inputs for gradient parity);
    a second run from the first one's density tightens the stationarity
    that the analytic gradient formula assumes."""
    rhf = oscf.RHF(mol, jk="dense", conv_tol=conv_tol, max_iter=300)
    r = rhf.run()
    r = rhf.run(D0=r["D"])
    return r["D"], r["F"], r["energy"]
