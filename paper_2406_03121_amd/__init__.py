"""MI355X (gfx950) HIP implementation of the Gaussian-basis Hartree-Fock hot
path of MESS (arXiv 2406.03121): ERIs, J/K and the SCF step behind the C ABI
in include/mess.h.  ``mess`` is the ctypes binding; ``build`` compiles
libmess_hip.so with hipcc."""
