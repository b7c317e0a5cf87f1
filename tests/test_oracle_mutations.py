"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each one.

The mistake is planted by a text substitution in the oracle's source, loaded
as a separate module; the real oracle is never modified.
"""
import os
import types

import pytest

from tests import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "fock.py")

MUTATIONS = {
    "conjugate_target_not_orbital": ("rho = np.conj(psi_j) * phi_k", "rho = psi_j * np.conj(phi_k)"),
    "dropped_minus": ("out[t] = -acc / omega_vol", "out[t] = acc / omega_vol"),
    "prefactor_1_over_Nr": ("out[t] = -acc / omega_vol", "out[t] = -acc / acc.size"),
    "missing_Nr_in_inverse": ("return _ifftn(f, workers) * rho.size", "return _ifftn(f, workers)"),
    "hse_k0_zero": ("k[~nz0] = np.pi / (omega * omega)", "k[~nz0] = 0.0"),
    "hse_wrong_screening": ("np.exp(-g2[nz0] / (4.0 * omega * omega))", "np.exp(-g2[nz0] / (omega * omega))"),
    "coulomb_k0_nonzero": ("k[~nz0] = 0.0\n    elif", "k[~nz0] = 1.0\n    elif"),
    "kernel_axes_swapped": ("return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2",
                            "return gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2"),
    "kernel_shifted": ("    return k * scale", "    return np.fft.fftshift(k) * scale"),
    "wrong_length_per_axis": ("gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / ly",
                              "gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / lx"),
    "dropped_diagonal_pair": ("        for j in range(psi.shape[0]):\n            acc",
                              "        for j in range(psi.shape[0]):\n            if j == k:\n                continue\n            acc"),
    "psi_not_multiplied_back": ("acc += psi[j] * pair_potential", "acc += phi[k] * pair_potential"),
    "energy_without_half": ("return 0.5 * float(np.real(np.sum(np.conj(p) * v)))", "return float(np.real(np.sum(np.conj(p) * v)))"),
    "ace_missing_conj_transpose": ("xi = xiH.conj().T  # N_r x N", "xi = xiH.T  # N_r x N"),
    "ace_apply_sign": ("Y = -(X @ (X.conj().T @ F))", "Y = X @ (X.conj().T @ F)"),
    "ace_apply_transpose": ("Y = -(X @ (X.conj().T @ F))", "Y = -(X @ (X.T @ F))"),
    "ace_unsymmetrised_upper": ("L = np.linalg.cholesky(-M)", "L = np.linalg.cholesky(-M).conj().T"),
    "residual_sign_of_i": ("R = X + 0.5j * dt * (HX - T) - Xh", "R = X - 0.5j * dt * (HX - T) - Xh"),
    "residual_full_dt": ("R = X + 0.5j * dt * (HX - T) - Xh", "R = X + 1j * dt * (HX - T) - Xh"),
    "residual_overlap_without_conj": ("S = X.conj().T @ HX\n    T = X @ S", "S = X.T @ HX\n    T = X @ S"),
    "residual_rotation_transposed": ("T = X @ S\n", "T = X @ S.T\n"),
    "residual_half_added": ("R = X + 0.5j * dt * (HX - T) - Xh", "R = X + 0.5j * dt * (HX - T) + Xh"),
    "cholqr_upper_factor": ("Z = _sla.solve_triangular(L, X.conj().T, lower=True)",
                            "Z = _sla.solve_triangular(L.conj().T, X.conj().T, lower=False)"),
    "cholqr_missing_conj": ("return Z.conj().reshape(np.shape(psi))", "return Z.reshape(np.shape(psi))"),
    "density_square_not_modulus": ("rho += f[i] * (X[i].real ** 2 + X[i].imag ** 2)",
                                   "rho += f[i] * (X[i].real ** 2 - X[i].imag ** 2)"),
    "kinetic_without_half": ("half_g2 = 0.5 * g2_grid(n, L)", "half_g2 = g2_grid(n, L)"),
    "kinetic_sign": ("half_g2 = 0.5 * g2_grid(n, L)", "half_g2 = -0.5 * g2_grid(n, L)"),
    "kinetic_inverse_missing": ("out[k] = np.fft.ifftn(half_g2 * np.fft.fftn(phi[k]))",
                                "out[k] = half_g2 * np.fft.fftn(phi[k]) / phi[k].size"),
    "kinetic_lengths_reversed": ("half_g2 = 0.5 * g2_grid(n, L)", "half_g2 = 0.5 * g2_grid(n, _as_l3(L)[::-1])"),
    "density_ignores_occupation": ("rho += f[i] * (X[i].real ** 2 + X[i].imag ** 2)",
                                   "rho += (X[i].real ** 2 + X[i].imag ** 2)"),
}


def _load_mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/absent: {old!r}"
    mod = types.ModuleType("oracle_mutant")
    mod.__dict__["__name__"] = "oracle_mutant"
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    mutant = _load_mutant(*MUTATIONS[name])
    caught = []
    for pin, (fn, bound) in pins.ALL.items():
        try:
            err = fn(mutant)
        except Exception:
            caught.append(pin)
            continue
        if not (err <= bound):
            caught.append(pin)
        if caught:
            break
    assert caught, f"no pin caught the planted mistake {name}"
