"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package generates inputs only: crystal geometry, plane-wave basis
spheres, a model local-potential Hamiltonian, its eigenpairs (the stand-in for
the DFT wavefunctions the method consumes), k/q sets, the chi0 G-set and the
imaginary-frequency list. It holds none of the method's arithmetic (no
oscillator strengths, no response function, no Dyson equation).
"""

from .crystal import (  # noqa: F401
    Lattice, Crystal, fcc_lattice, sc_lattice, make_crystal, gset_sorted,
    kgrid_gamma, frequencies,
)
from .configs import CONFIGS, crystal_for  # noqa: F401
from .rand import rng, random_complex  # noqa: F401
