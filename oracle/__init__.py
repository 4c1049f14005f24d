"""CPU FP64 oracle — test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import or execute anything in this package.  It shares no
code with the HIP library and does not import it.

* ``mess_oracle.c`` — closed-form Gaussian integrals (McMurchie-Davidson),
  Boys function, J/K (paper section 3, eqs. 1-3).
* ``core.py`` — ctypes binding of the C oracle plus dense-tensor J/K by the
  plain sums that define them.
* ``scf.py`` — restricted Hartree-Fock self-consistent field (eq. 2, the
  Roothaan equation, solved by fixed-point iteration), with core-Hamiltonian
  guess and Pulay DIIS.
* ``lda.py`` — Dirac-Slater exchange on a Becke molecular grid.
"""
