"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds no arithmetic of the Fock-exchange method itself: it only
draws orbitals (random planewave coefficients inside a kinetic-energy sphere,
Loewdin-orthonormalised) and Poisson request streams.  Both the CPU oracle and
the HIP library receive exactly the arrays produced here.
"""
from .orbitals import (  # noqa: F401
    WORKLOADS,
    cell_of,
    make_orbitals,
    planewave_orbitals,
    random_grid_vectors,
    random_unitary,
    workload,
)
