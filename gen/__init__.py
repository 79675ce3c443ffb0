"""Seeded synthetic inputs: diamond-lattice carbon cells with voids, vacancies and noise.

This package produces atomic structures (positions in an orthorhombic periodic
box) and the run settings that go with them.  It holds none of the electronic
structure arithmetic: no Hamiltonian, no clusters, no Krylov steps.  Seeded
initial velocities for MD runs come from here too.  Both the
GPU library's tests and the CPU oracle draw their inputs from here.
"""
from .structures import (  # noqa: F401
    Structure,
    diamond_sites,
    make_structure,
    make,
    CONFIGS,
    config_seed,
    random_velocities,
)
