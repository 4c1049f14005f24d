"""Batched conformer scans (the paper's batched-conformation example):
many geometries of one molecule as one batch, one launch per angular class
and step for all of them.

* Minimal-basis H2 at 64 bond lengths in [0.6, 10] bohr: every energy equals
  the closed form within 1e-10 Ha.
* A bond of a 3-atom molecule (fixed per-element s/p/d basis) stretched over
  16 displacements: every conformer's batched energy equals its own
  single-molecule SCF within 1e-9 Ha, and two of them the oracle's SCF."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import closed_forms as CF  # noqa: E402
from gpu_common import announce, need_gpu  # noqa: E402

from mess_inputs import generators as G  # noqa: E402
from oracle import scf as oscf  # noqa: E402

pytestmark = pytest.mark.gpu


def _run_batch(mess, mols, tol=1e-11, steps=60):
    B = mess.mess_batch_create(mols)
    bs = mess.mess_batch_scf_create(B, schwarz_tol=0.0, conv_tol=tol, diis_size=8, use_graph=True)
    for _ in range(steps):
        mess.mess_batch_scf_step(bs)
        st = mess.mess_batch_scf_status(bs)
        if st["n_converged"] == len(mols):
            break
    bs.close()
    return st


def test_h2_dissociation_scan_closed_form():
    mess = need_gpu()
    alpha = 0.5
    mols = G.h2_scan(alpha, 64, 0.6, 10.0)
    st = _run_batch(mess, mols)
    assert st["n_converged"] == 64
    rs = np.linspace(0.6, 10.0, 64)
    ref = np.array([CF.h2_minimal_energy(alpha, r) for r in rs])
    err = np.abs(st["energy"] - ref)
    announce(f"H2 scan: max |E - closed form| {err.max():.2e}; minimum at R = {rs[np.argmin(ref)]:.3f}")
    assert err.max() < 1e-10


def test_bond_stretch_scan_batch_equals_single():
    mess = need_gpu()
    base = G.batched_molecule(1007)
    a, b = 0, 1
    d = base.xyz[b] - base.xyz[a]
    mols = G.conformer_scan(base, b, d, np.linspace(-0.3, 1.2, 16))
    st = _run_batch(mess, mols)
    assert st["n_converged"] == len(mols)
    for k, m in enumerate(mols):
        Bm = mess.basis_from_molecule(m)
        sc = mess.mess_scf_create(Bm, schwarz_tol=0.0, conv_tol=1e-11, diis_size=8)
        for _ in range(60):
            e, de, r, c = mess.mess_scf_step(sc)
            if c:
                break
        assert abs(st["energy"][k] - e) < 1e-9, k
    for k in (0, 9):
        ref = oscf.RHF(mols[k], conv_tol=1e-11, max_iter=200).run()
        assert abs(st["energy"][k] - ref["energy"]) < 1e-8, k
    announce(f"bond scan energies {np.round(st['energy'], 6)}")
