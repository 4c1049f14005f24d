"""Write the converged-energy golden for the 60-atom water cluster.

Runs only the CPU oracle: restricted Hartree-Fock (core-Hamiltonian guess,
Pulay DIIS over 8 Fock matrices, |dE| < 1e-10 Ha) with J/K from unique
shell quartets under Schwarz screening (skip iff Q_ab Q_cd < 1e-10).
Usage: python tests/golden/make_water60_golden.py [seed]   (hours of CPU)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from mess_inputs import generators as G  # noqa: E402
from oracle import scf  # noqa: E402


def main():
    seed = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    mol = G.water_cluster(seed)
    t0 = time.time()
    rhf = scf.RHF(mol, jk="unique", tau=1e-10, diis=True, conv_tol=1e-10, max_iter=60)
    energies = []
    orig_jk = rhf.jk

    def jk_logged(D):
        out = orig_jk(D)
        print(f"J/K build {len(energies) + 1} done after {time.time() - t0:.0f} s", flush=True)
        energies.append(None)
        return out

    rhf.jk = jk_logged
    r = rhf.run()
    out = {
        "workload": mol.name, "n_bf": mol.n_bf, "schwarz_tol": 1e-10, "conv_tol": 1e-10, "diis": 8,
        "guess": "core Hamiltonian", "energies": r["energies"], "energy": r["energy"],
        "converged": r["converged"], "iterations": r["iterations"], "e_nuc": r["e_nuc"],
        "generator": "tests/golden/make_water60_golden.py (CPU oracle only)",
        "cpu_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, f"water60_spd_seed{seed}_rhf.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["energy"], flush=True)


if __name__ == "__main__":
    main()
