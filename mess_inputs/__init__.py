"""Seeded synthetic molecule + basis generators.

This package is the only code shared by the CPU oracle and the HIP path.  It
draws geometries, element choices, shell layouts, exponents and contraction
coefficients from ``numpy.random.Generator(PCG64(seed))`` and returns plain
arrays.  It holds none of the method's arithmetic (no normalisation, no
integrals, no energies).
"""
from .generators import (  # noqa: F401
    Molecule,
    ELEMENT_Z,
    random_small_molecule,
    water_cluster,
    batched_molecule,
    batch_of_molecules,
    fixed_element_basis,
    single_gaussian_system,
    workload,
)
