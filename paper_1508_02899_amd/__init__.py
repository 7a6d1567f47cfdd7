"""MI355X-native phase-space lattice method for diffusive heavy particles.

Implements the lattice update of Laenen, Krstulovic & Bec,
arXiv:1508.02899 (Sec. 2) as hand-written HIP kernels for gfx950 behind the
C ABI in ``include/lattice.h``; ``lattice`` is the Python binding and
``inputs`` the seeded synthetic flows and initial conditions.
"""
from .lattice import (Batch, Lattice, LatticeError,  # noqa: F401
                      LatticeLibraryMissing, LatticeSpec, Member, Mlp,
                      load_library, restrict, strerror, velocity)
