"""The FP64 oracle against closed forms, brute force and invariants (CPU only)."""
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("name", sorted(pins.ALL))
def test_pin(name):
    fn, bound = pins.ALL[name]
    err = fn(oracle)
    assert err <= bound, f"{name}: {err:.3e} > {bound:.1e}"


def test_coulomb_single_constant_orbital_is_not_definite():
    """-M = 0 for one constant orbital with the Coulomb kernel (K(0) = 0): Cholesky must fail."""
    import numpy as np

    n3, L3 = (4, 4, 4), (3.0, 3.0, 3.0)
    psi = np.full((1, 4, 4, 4), 1.0 / 8.0, dtype=complex)
    w = oracle.apply_vx(psi, psi, n3, L3, "coulomb")
    assert np.abs(w).max() < 1e-14
    with pytest.raises(np.linalg.LinAlgError):
        oracle.build_ace(psi, w)
