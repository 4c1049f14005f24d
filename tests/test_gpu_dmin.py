"""GPU direct minimisation (mess_dmin_step) against the oracle
(oracle/dmin.py): the same Adam trajectory step by step from Z = 1, the
minimal-basis H2 closed form, and the converged SCF energy of a 6-atom
molecule reached by minimisation alone."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from gpu_common import announce, host, need_gpu, zeros  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import dmin, scf as oscf  # noqa: E402

pytestmark = pytest.mark.gpu


def test_energy_and_gradient_match_oracle():
    """One evaluation at a fixed trial matrix (identity, and a random one):
    E within 1e-10 * max(1, |E|), dE/dZ within 1e-9 of its largest element.
    (An Adam trajectory is not compared step by step: Adam divides each
    gradient component by its own running magnitude, so rounding-level
    differences in the components that vanish exactly (rotations among
    occupied or among virtual orbitals leave E unchanged) change later steps
    by far more than rounding; measured on the oracle alone, a relative
    gradient perturbation of 1e-15 moves its 40-step trajectory by 1e-4 Ha.)"""
    mess = need_gpu()
    import torch
    for mol in (G.random_small_molecule(1), G.water_cluster(0, n_waters=2, box=7.0)):
        dm = dmin.DirectMin(mol)
        B = mess.basis_from_molecule(mol)
        st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=0.0, diis_size=0)
        rng = np.random.Generator(np.random.PCG64(4))
        for Z in (np.eye(mol.n_bf), np.eye(mol.n_bf) + 0.05 * rng.normal(size=(mol.n_bf, mol.n_bf))):
            Eo, go, _ = dm.energy_and_grad(Z)
            Gd = zeros(B.nbf, B.nbf)
            e = mess.mess_dmin_eval(st, torch.tensor(Z, dtype=torch.float64, device="cuda"), Gd)
            gd = host(Gd)
            announce(f"dmin eval {mol.name}: |dE| {abs(e - Eo):.2e}, max |dG| {np.abs(gd - go).max():.2e} "
                     f"(max |G| {np.abs(go).max():.2e})")
            assert abs(e - Eo) < 1e-10 * max(1.0, abs(Eo))
            assert np.abs(gd - go).max() < 1e-9 * np.abs(go).max()


def test_minimisation_reaches_closed_form_and_scf():
    mess = need_gpu()
    h2 = G.single_gaussian_system("H2", 0.5, 1.4)
    B = mess.basis_from_molecule(h2)
    st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=0.0, diis_size=0)
    for _ in range(200):
        e, g = mess.mess_dmin_step(st, lr=0.1)
    assert abs(e - (-0.9552136651016611)) < 1e-9
    mol = G.random_small_molecule(1)
    ref = oscf.RHF(mol, conv_tol=1e-11).run()
    B = mess.basis_from_molecule(mol)
    st = mess.mess_scf_create(B, schwarz_tol=1e-10, conv_tol=0.0, diis_size=0)
    for _ in range(600):
        e, g = mess.mess_dmin_step(st, lr=0.1)
    announce(f"dmin 600 steps: E - E_scf = {e - ref['energy']:.2e}, max |grad| {g:.2e}")
    assert abs(e - ref["energy"]) < 1e-6


def test_dmin_rejections():
    mess = need_gpu()
    mol = G.random_small_molecule(1)
    B = mess.basis_from_molecule(mol)
    st = mess.mess_scf_create(B)
    with pytest.raises(mess.MessError) as ei:
        mess.mess_dmin_step(st, lr=0.0)
    assert ei.value.code == mess.MESS_E_ARG
    with pytest.raises(mess.MessError) as ei:
        mess.mess_dmin_trial(st, zeros(B.nbf, B.nbf))
    assert ei.value.code == mess.MESS_E_ARG
    lda = mess.mess_scf_create(B, xc=mess.MESS_XC_LDA_X)
    with pytest.raises(mess.MessError) as ei:
        mess.mess_dmin_step(lda, lr=0.1)
    assert ei.value.code == mess.MESS_E_UNSUPPORTED
