"""CPU checks of the C ABI: the library loads, exports every declared symbol,
rejects bad arguments, and its pass code (run on the host) matches the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1905_01348_amd import fock as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:fx_status|const char\*)\s+(fx_\w+)\s*\(", txt, re.M))
    return sorted(names)


def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(F.LIB_PATH)
    names = declared_symbols()
    assert "fx_apply_vx" in names and "fx_build_ace" in names and "fx_serve" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows every declared symbol
    assert set(names) <= set(F._SIGS)


def test_version_and_error_strings():
    lib = F.load()
    assert b"libfock" in lib.fx_version()
    assert lib.fx_apply_vx(None, None, None, None, 1, 1, None, 1, 1, None, 1, 0, 0, 0, None, None) == F.FX_ERR_INVALID
    assert b"ctx" in lib.fx_last_error()


@pytest.mark.parametrize("n3", [(4, 4, 4), (6, 4, 8), (24, 24, 24), (12, 18, 16), (96, 9, 2), (27, 32, 81),
                                (2, 3, 96), (48, 72, 36), (54, 64, 9)])
@pytest.mark.parametrize("kind", ["hse", "coulomb"])
def test_host_pass_code_matches_oracle(n3, kind):
    L3 = (3.0, 4.0, 5.0)
    a = synth.random_grid_vectors(1, n3, 1)[0]
    b = synth.random_grid_vectors(2, n3, 1)[0]
    K = oracle.kernel_table(n3, L3, kind, 0.3)
    ref = -oracle.pair_potential(a, b, K) / np.prod(L3)
    got = F.debug_host_pair(a, b, n=n3, L=L3, kernel=kind, omega=0.3)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n", [1, 5, 25, 97, 100, 192, 0, -4])
def test_unsupported_grid_edges_rejected(n):
    a = np.zeros(8, dtype=complex)
    with pytest.raises(F.FockError) as ei:
        F.debug_host_pair(a, a, n=(n, 2, 2), L=1.0)
    assert ei.value.status == F.FX_ERR_UNSUPPORTED


def test_bad_kernel_rejected():
    a = np.zeros(8, dtype=complex)
    with pytest.raises(F.FockError) as ei:
        F.debug_host_pair(a, a, n=2, L=1.0, kernel="hse", omega=-1.0)
    assert ei.value.status == F.FX_ERR_INVALID
    with pytest.raises(F.FockError) as ei:
        F.debug_host_pair(a, a, n=2, L=1.0, kernel=7)
    assert ei.value.status == F.FX_ERR_UNSUPPORTED
    with pytest.raises(F.FockError) as ei:
        F.debug_host_pair(a, a, n=2, L=(1.0, 0.0, 1.0))
    assert ei.value.status == F.FX_ERR_INVALID


def test_axis_plan_enumeration():
    """Every schedule the autotuner may pick multiplies to its edge, uses the radix set,
    has at most three stages, and the default (balanced two-stage where possible) comes first."""
    rad = {2, 3, 4, 6, 8, 9, 12}
    for n in [2, 3, 4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 54, 64, 72, 81, 96]:
        plans = F.debug_axis_plans(n)
        assert plans, n
        for p in plans:
            assert int(np.prod(p)) == n and set(p) <= rad and 1 <= len(p) <= 3, (n, p)
        assert len({tuple(p) for p in plans}) == len(plans)
    assert F.debug_axis_plans(96)[0] == [12, 8] and F.debug_axis_plans(24)[0] == [6, 4]


@pytest.mark.parametrize("n3", [(8, 12, 16), (24, 36, 9), (96, 4, 2), (2, 72, 3)])
def test_every_radix_schedule_matches_oracle(n3):
    """The pass code with each enumerated radix schedule (one axis varied at a time) equals the oracle."""
    L3 = (3.0, 4.5, 5.0)
    a = synth.random_grid_vectors(3, n3, 1)[0]
    b = synth.random_grid_vectors(4, n3, 1)[0]
    K = oracle.kernel_table(n3, L3, "hse", 0.3)
    ref = -oracle.pair_potential(a, b, K) / np.prod(L3)
    for ax in range(3):
        for p in F.debug_axis_plans(n3[ax]):
            radix = [[], [], []]
            radix[ax] = p
            got = F.debug_host_pair(a, b, n=n3, L=L3, kernel="hse", omega=0.3, radix=radix)
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (ax, p)


def test_invalid_radix_schedules_rejected():
    a = np.zeros(8 * 6 * 4, dtype=complex)
    for bad in ([[5], [], []], [[2, 2], [], []], [[], [6, 2], []], [[8, 1], [], []], [[16], [], []]):
        with pytest.raises(F.FockError) as ei:
            F.debug_host_pair(a, a, n=(8, 6, 4), L=1.0, radix=bad)
        assert ei.value.status == F.FX_ERR_INVALID, bad
