"""Pins of the oracle's nuclear gradient (central differences of the
converged RHF energy), on the CPU:

* minimal-basis H2 (one s Gaussian per atom): the force along the bond is
  the derivative of the textbook closed-form energy E(R) (differentiated
  here by a high-order difference of the closed form itself), and the
  perpendicular components vanish;
* a water molecule with s, p and d functions: the forces sum to zero
  (translation) and exert no torque (rotation), as an energy invariant
  under rigid motions requires;
* the nuclear-repulsion closed form against differences of E_nuc.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(__file__))
from closed_forms import h2_minimal_energy  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402
from oracle import grad as ograd  # noqa: E402


def test_h2_force_is_the_closed_form_derivative():
    alpha, R = 0.42, 1.3
    mol = G.single_gaussian_system("H2", alpha, bond=R)
    g = ograd.fd_gradient(mol)
    h = 1e-3
    dE = (8 * (h2_minimal_energy(alpha, R + h) - h2_minimal_energy(alpha, R - h))
          - (h2_minimal_energy(alpha, R + 2 * h) - h2_minimal_energy(alpha, R - 2 * h))) / (12 * h)
    # atom 1 sits at +R on z: dE/dz_1 = dE/dR, dE/dz_0 = -dE/dR
    assert abs(g[1, 2] - dE) < 1e-8 and abs(g[0, 2] + dE) < 1e-8
    assert np.abs(g[:, :2]).max() < 1e-9


def test_water_forces_are_translation_and_rotation_invariant():
    mol = G.water_cluster(0, n_waters=1)
    g = ograd.fd_gradient(mol)
    xyz = np.asarray(mol.xyz).reshape(-1, 3)
    assert np.abs(g).max() > 1e-3
    assert np.abs(g.sum(axis=0)).max() < 2e-8
    # (torque: gradient error ~5e-9 times lever arms of several bohr)
    assert np.abs(np.cross(xyz, g).sum(axis=0)).max() < 2e-8 * max(1.0, np.abs(xyz).max())


def test_nuclear_repulsion_gradient():
    mol = G.water_cluster(0, n_waters=1)
    g = ograd.nuclear_repulsion_gradient(mol)
    h = 1e-4
    for a in range(len(mol.Z)):
        for k in range(3):
            ep = core.nuclear_repulsion(ograd.displaced(mol, a, k, h))
            em = core.nuclear_repulsion(ograd.displaced(mol, a, k, -h))
            assert abs((ep - em) / (2 * h) - g[a, k]) < 1e-7
