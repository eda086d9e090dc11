"""MI355X-native vectorial lattice Boltzmann (VLBM) hot path (arXiv 2609.10639).

The compute path is the HIP library libvlbm.so (include/vlbm.h); this package
is its thin Python binding plus the seeded input generators.
"""
from .solver import Solver  # noqa: F401
