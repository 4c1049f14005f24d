"""Write full-size J/K goldens for the 60-atom water cluster (300 functions).

Runs only the CPU oracle (unique shell quartets, 8-permutation update rule,
Schwarz screening: skip iff Q_ab Q_cd < 1e-10):

1. J, K of the seeded test density ``symmetric_density(300, 21)``.
2. The restricted Hartree-Fock run of ``make_water60_golden.py`` (core
   guess, Pulay DIIS over 8 Fock matrices, |dE| < 1e-10 Ha), keeping the
   density of its last iteration, D*, and J(D*), K(D*) from that iteration's
   Fock build.

Output: ``water60_spd_seed0_jk.npz`` with the upper triangles (row-major,
``numpy.triu_indices``) of every symmetric matrix:
  d21_J, d21_K            J, K of the seed-21 density
  dstar_D, dstar_J, dstar_K  D*, J(D*), K(D*)
  energies                the SCF energies (must equal the energy golden's)
Usage: python tests/golden/make_water60_jk_golden.py   (hours of CPU)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from mess_inputs import generators as G  # noqa: E402
from oracle import core  # noqa: E402
from oracle import scf  # noqa: E402

TAU = 1e-10
OUT = os.path.join(HERE, "water60_spd_seed0_jk.npz")


def upper(M):
    return M[np.triu_indices(M.shape[0])]


def main():
    mol = G.water_cluster(0)
    N = mol.n_bf
    t0 = time.time()
    part = {}
    D21 = G.symmetric_density(N, 21)
    J, K, nq = core.jk_unique(mol, D21, TAU)
    part["d21_J"], part["d21_K"] = upper(J), upper(K)
    print(f"seed-21 J/K done after {time.time() - t0:.0f} s ({nq} quartets)", flush=True)
    np.savez_compressed(OUT + ".part.npz", **part)

    rhf = scf.RHF(mol, jk="unique", tau=TAU, diis=True, conv_tol=1e-10, max_iter=60)
    last = {}
    orig_jk = rhf.jk

    def jk_logged(D):
        J, K = orig_jk(D)
        last["D"], last["J"], last["K"] = D.copy(), J, K
        print(f"SCF J/K build done after {time.time() - t0:.0f} s", flush=True)
        return J, K

    rhf.jk = jk_logged
    r = rhf.run()
    assert r["converged"]
    assert np.array_equal(last["D"], r["D"])
    part["dstar_D"], part["dstar_J"], part["dstar_K"] = upper(last["D"]), upper(last["J"]), upper(last["K"])
    part["energies"] = np.array(r["energies"])
    part["cpu_seconds"] = np.array(time.time() - t0)
    np.savez_compressed(OUT, **part)
    os.remove(OUT + ".part.npz")
    print("wrote", OUT, r["energy"], flush=True)


if __name__ == "__main__":
    main()
