"""FP64 CPU oracle for the Fock exchange operator and the ACE operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
package; only the tests, the smoke check and the benchmark's CPU-baseline leg
may use it.  It shares no code with the HIP path (no kernels, headers, tables
or helpers): it is a direct, slow transcription of the definitions.

Every function cites the passage of Jia, Wang & Lin, "Parallel Transport
Time-Dependent Density Functional Theory Calculations with Hybrid Functional on
Summit" (arXiv:1905.01348) that it follows.  Pinning status of each function is
listed in ``oracle.fock.PINS``; no function is "parity unpinned".
"""
from .fock import (  # noqa: F401
    PINS,
    apply_ace,
    apply_kinetic,
    apply_vx,
    build_ace,
    density,
    exchange_energy,
    g2_grid,
    kernel_table,
    orthonormalize,
    pair_potential,
    pt_residual,
    vx_dense_matrix,
    volume,
)
