"""GPU parity of the analytic Hartree-Fock nuclear gradient (mess_hf_gradient)
against the oracle's central differences of its converged energy, given the
oracle's converged density and Fock matrix:

* minimal-basis H2: the force along the bond against the derivative of the
  textbook closed-form energy (within 1e-9 Ha/bohr);
* an s/p molecule (6 atoms) and a water molecule with d functions: every
  component within 1e-6 Ha/bohr of the differences (their own accuracy is
  about 1e-8);
* invariants of the analytic forces: they sum to zero and exert no torque
  (to rounding, far tighter than the differences);
* the SCF handle's gradient (its own converged D and F) agrees with the one
  at the oracle's D and F.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from closed_forms import h2_minimal_energy  # noqa: E402
from gpu_common import announce, dev, need_gpu  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import grad as ograd  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "hco6_sp/1": lambda: G.random_small_molecule(1),
    "water1_spd/0": lambda: G.water_cluster(0, n_waters=1),
}


def test_h2_force_closed_form():
    mess = need_gpu()
    alpha, R = 0.42, 1.3
    mol = G.single_gaussian_system("H2", alpha, bond=R)
    D, F, E = ograd.converged(mol)
    B = mess.basis_from_molecule(mol)
    g = mess.mess_hf_gradient(B, dev(D), dev(F))
    h = 1e-3
    dE = (8 * (h2_minimal_energy(alpha, R + h) - h2_minimal_energy(alpha, R - h))
          - (h2_minimal_energy(alpha, R + 2 * h) - h2_minimal_energy(alpha, R - 2 * h))) / (12 * h)
    announce(f"H2 force {g[1, 2]!r} vs closed-form dE/dR {dE!r}")
    assert abs(g[1, 2] - dE) < 1e-9 and abs(g[0, 2] + dE) < 1e-9
    assert np.abs(g[:, :2]).max() < 1e-12


@pytest.mark.parametrize("case", list(CASES))
def test_gradient_matches_oracle_differences(case):
    mess = need_gpu()
    mol = CASES[case]()
    D, F, E = ograd.converged(mol)
    B = mess.basis_from_molecule(mol)
    g = mess.mess_hf_gradient(B, dev(D), dev(F))
    fd = ograd.fd_gradient(mol)
    err = np.abs(g - fd).max()
    xyz = np.asarray(mol.xyz).reshape(-1, 3)
    announce(f"gradient {case}: max |g - fd| {err:.2e} (max |g| {np.abs(g).max():.3f}); "
             f"sum {np.abs(g.sum(0)).max():.1e}, torque {np.abs(np.cross(xyz, g).sum(0)).max():.1e}")
    assert err < 1e-6
    assert np.abs(g.sum(axis=0)).max() < 1e-10 * max(1.0, np.abs(g).max())
    assert np.abs(np.cross(xyz, g).sum(axis=0)).max() < 1e-8
    # the SCF handle's own converged state
    st = mess.mess_scf_create(B, schwarz_tol=0.0, conv_tol=1e-12, diis_size=8)
    for _ in range(200):
        e, de, r, c = mess.mess_scf_step(st)
        if c:
            break
    assert c
    g2 = mess.mess_scf_gradient(st)
    assert np.abs(g2 - g).max() < 1e-7
    st.close()
    B.close()
