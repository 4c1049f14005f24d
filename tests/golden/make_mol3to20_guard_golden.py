"""Write the divergence-guard golden of the batched-molecule seed 1002
(18 atoms, 114 functions), a molecule whose plain DIIS iteration oscillates
by several Hartree without settling.

Runs only the CPU oracle: restricted Hartree-Fock from the core-Hamiltonian
guess, Pulay DIIS over 8 Fock matrices, |dE| < 1e-8 Ha, J/K from the dense
tensor, with the divergence guard on (stages: DIIS, DIIS afresh, damped
DIIS, restart from the core guess) and, for contrast, off.
Usage: python tests/golden/make_mol3to20_guard_golden.py   (about 15 min of CPU)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from mess_inputs import generators as G  # noqa: E402
from oracle import scf  # noqa: E402

SEED = 1002
OUT = os.path.join(HERE, "mol3to20_seed1002_guard.json")


def main():
    mol = G.batched_molecule(SEED)
    t0 = time.time()
    rhf = scf.RHF(mol, jk="dense", diis=True, diis_size=8, conv_tol=1e-8, max_iter=200)
    print(f"ERI tensor after {time.time() - t0:.0f} s", flush=True)
    r = rhf.run()
    stages = np.array(r["stages"])
    rhf.guard = False
    r0 = rhf.run()
    out = {
        "workload": f"mol3to20/{SEED}", "n_bf": mol.n_bf, "conv_tol": 1e-8, "diis": 8,
        "guess": "core Hamiltonian",
        "guard": {"energies": r["energies"], "energy": r["energy"], "converged": r["converged"],
                  "iterations": r["iterations"],
                  "stage_starts": [int(np.argmax(stages == s)) for s in range(4)]},
        "no_guard": {"converged": r0["converged"], "iterations": r0["iterations"],
                     "energy_min": float(min(r0["energies"])), "energy_max_after_10": float(max(r0["energies"][10:]))},
        "generator": "tests/golden/make_mol3to20_guard_golden.py (CPU oracle only)",
        "cpu_seconds": time.time() - t0,
    }
    json.dump(out, open(OUT, "w"), indent=1)
    print("wrote", OUT, r["energy"], r["iterations"], flush=True)


if __name__ == "__main__":
    main()
