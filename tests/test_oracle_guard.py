"""The oracle's SCF divergence guard (reset DIIS, then damp 0.5, then restart
from the core-Hamiltonian guess), checked on the CPU:

* it leaves a run whose energy never rises untouched (same energies, bit for
  bit, as with the guard off);
* a non-finite energy restarts the run from the core guess: the energy after
  the restart is the run's first energy, bit for bit, and the run then
  converges to the ordinary result;
* on a molecule whose DIIS path climbs repeatedly (batched-molecule seed 1013)
  every stage is reached in order and the run converges to the energy of the
  unguarded run within the convergence tolerance.
"""
import numpy as np
import pytest

from mess_inputs import generators as G
from oracle import scf


def _stage_starts(stages):
    st = np.array(stages)
    return [int(np.argmax(st == s)) for s in range(st.max() + 1)]


def test_guard_leaves_monotone_run_alone():
    mol = G.random_small_molecule(1)
    a = scf.RHF(mol, jk="dense", conv_tol=1e-10, guard=True).run()
    b = scf.RHF(mol, jk="dense", conv_tol=1e-10, guard=False).run()
    assert np.all(np.diff(a["energies"]) <= 1e-6)
    assert a["energies"] == b["energies"] and max(a["stages"]) == 0


def test_non_finite_energy_restarts_from_core_guess():
    mol = G.random_small_molecule(1)
    ref = scf.RHF(mol, jk="dense", conv_tol=1e-10).run()
    rhf = scf.RHF(mol, jk="dense", conv_tol=1e-10)
    fock = rhf.fock
    calls = {"n": 0}

    def poisoned(D):
        calls["n"] += 1
        F, E = fock(D)
        return (F, float("nan")) if calls["n"] == 3 else (F, E)

    rhf.fock = poisoned
    r = rhf.run()
    assert np.isnan(r["energies"][2])
    assert r["stages"][:3] == [0, 0, 0] and set(r["stages"][3:]) == {3}
    assert r["energies"][3] == ref["energies"][0]  # the core guess again
    assert r["converged"] and abs(r["energy"] - ref["energy"]) < 1e-9


def test_non_finite_energy_after_restart_raises():
    mol = G.random_small_molecule(1)
    rhf = scf.RHF(mol, jk="dense", conv_tol=1e-10)
    fock = rhf.fock
    rhf.fock = lambda D: (fock(D)[0], float("nan"))
    with pytest.raises(FloatingPointError):
        rhf.run()


def test_guard_walks_every_stage_and_converges():
    mol = G.batched_molecule(1013)
    assert mol.n_bf == 34
    rhf = scf.RHF(mol, jk="dense", conv_tol=1e-8, max_iter=150, guard=False)
    off = rhf.run()
    rhf.guard = True
    on = rhf.run()
    assert off["converged"] and on["converged"]
    starts = _stage_starts(on["stages"])
    assert len(starts) == 4 and starts == sorted(starts) and starts[0] == 0
    E = np.array(on["energies"])
    # each stage change follows the second energy rise of the stage before
    for s in range(1, 4):
        seg = E[starts[s - 1]:starts[s]]
        assert int(np.sum(np.diff(seg) > scf.RHF.RISE_TOL)) >= 1
    # the restart is the core guess again
    assert E[starts[3]] == E[0]
    assert abs(on["energy"] - off["energy"]) < 2e-8
