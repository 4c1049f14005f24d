"""Pins of the direct-minimisation oracle (oracle/dmin.py).

* The QR backward formula against central finite differences of a linear
  function of Q (the formula is derived, not looked up, so it is checked on
  its own).
* The energy gradient with respect to the trial matrix against central
  finite differences of the energy along random directions.
* The minimum over orbitals is the self-consistent solution: Adam reaches
  the minimal-basis H2 closed-form energy, and the oracle SCF's converged
  energy of a 6-atom molecule.
* Orthonormality C^T S C = 1 for any non-singular trial matrix.
"""
import numpy as np

from mess_inputs import generators as G
from oracle import dmin, scf


def test_qr_backward_matches_finite_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    for n in (3, 7):
        Z = np.eye(n) + 0.4 * rng.normal(size=(n, n))
        W0 = rng.normal(size=(n, n))
        Q, R = np.linalg.qr(Z)
        g = dmin.qr_grad(Q, R, W0)
        f = lambda Zz: float(np.sum(W0 * np.linalg.qr(Zz)[0]))  # noqa: E731
        for _ in range(4):
            V = rng.normal(size=Z.shape)
            h = 1e-6
            fd = (f(Z + h * V) - f(Z - h * V)) / (2 * h)
            assert abs(fd - float(np.sum(g * V))) < 1e-7 * max(1.0, abs(fd))


def test_energy_gradient_matches_finite_differences():
    mol = G.random_small_molecule(1)
    dm = dmin.DirectMin(mol)
    rng = np.random.Generator(np.random.PCG64(2))
    Z = np.eye(mol.n_bf) + 0.05 * rng.normal(size=(mol.n_bf, mol.n_bf))
    E, g, _ = dm.energy_and_grad(Z)
    for _ in range(3):
        V = rng.normal(size=Z.shape)
        h = 1e-5
        fd = (dm.energy(Z + h * V) - dm.energy(Z - h * V)) / (2 * h)
        assert abs(fd - float(np.sum(g * V))) < 2e-7 * max(1.0, abs(fd))


def test_orthonormal_orbitals():
    mol = G.random_small_molecule(2)
    dm = dmin.DirectMin(mol)
    rng = np.random.Generator(np.random.PCG64(3))
    Z = rng.normal(size=(mol.n_bf, mol.n_bf))
    Q, R = np.linalg.qr(Z)
    C = dm.X @ Q
    assert np.max(np.abs(C.T @ dm.S @ C - np.eye(mol.n_bf))) < 1e-10


def test_minimum_is_the_scf_solution():
    # minimal-basis H2 (one s Gaussian per atom, alpha 0.5, R 1.4 bohr):
    # Szabo-Ostlund closed form
    r = dmin.minimise(G.single_gaussian_system("H2", 0.5, 1.4), steps=200, lr=0.1)
    assert abs(r["energy"] - (-0.9552136651016611)) < 1e-9
    mol = G.random_small_molecule(1)
    ref = scf.RHF(mol, conv_tol=1e-11).run()
    r = dmin.minimise(mol, steps=600, lr=0.1)
    assert abs(r["energy"] - ref["energy"]) < 1e-6, r["energy"] - ref["energy"]
    # and the density is the SCF one (its projector up to the energy error)
    assert np.max(np.abs(r["D"] - ref["D"])) < 1e-2
