"""Seeded orbital generators for the Fock-exchange workloads.

Orbitals are stored orbital-major: an array of shape (N, nz, ny, nx), so that
orbital j is one contiguous grid vector with x fastest, r = ix + nx*(iy + ny*iz).
They are Euclidean-orthonormal grid vectors (sum_r conj(psi_i) psi_j = delta_ij).

Recipe (stated once, used by every workload):
  * reciprocal grid G_a = 2*pi*m_a/L_a with m_a in numpy's fftfreq order;
  * planewaves kept where |G|^2/2 < ecut (strict), ecut = 10 Ha, the cutoff of
    the paper's silicon runs (Sec. "Setup of the test physical system");
  * coefficients (re, im) iid N(0,1) scaled by exp(-|G|^2/4), drawn from
    numpy's PCG64 as standard_normal((N, n_pw, 2)) over the in-sphere G taken
    in C order of (iz, iy, ix);
  * Loewdin orthonormalisation of the coefficient block, then the inverse
    DFT scaled by sqrt(N_r), which is unitary, so orthonormality carries over
    to the grid.

Cell edges are multiples of the silicon lattice constant 5.43 A = 10.26 bohr
and each cell holds 2 orbitals per Si atom, 16 per 8-atom cubic cell.
"""
from __future__ import annotations

import os

import numpy as np

try:  # scipy's pocketfft takes a worker count; numpy's does not
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None

ECUT_HA = 10.0
A_SI_BOHR = 10.26
HSE_OMEGA = 0.106

# Workloads: name -> parameters.  Only shapes, seeds and kernels live here.
WORKLOADS = {
    # 8-Si-atom cubic cell, 24^3, 16 orbitals, Coulomb, phi = psi
    "24cube_16": dict(n=24, L=A_SI_BOHR, N=16, n_targets=16, kernel="coulomb", seed=0),
    # 64-Si-atom cell, 48^3, 128 orbitals, screened HSE, phi = psi
    "48cube_128": dict(n=48, L=2 * A_SI_BOHR, N=128, n_targets=128, kernel="hse", seed=1),
    # one GPU's band-index share of a 512-atom cell: 96^3, 1024 psi, 32 targets
    "96cube_1024x32": dict(n=96, L=4 * A_SI_BOHR, N=1024, n_targets=32, kernel="hse", seed=2),
    # serving classes
    "serveA": dict(n=24, L=A_SI_BOHR, N=16, n_targets=8, kernel="hse", seed=4000),
    "serveB": dict(n=48, L=2 * A_SI_BOHR, N=128, n_targets=8, kernel="hse", seed=4100),
    "serveC": dict(n=72, L=3 * A_SI_BOHR, N=432, n_targets=8, kernel="hse", seed=4200),
}


def workload(name: str) -> dict:
    w = dict(WORKLOADS[name])
    w["name"] = name
    return w


def cell_of(n, L):
    """(n3, len3) for a cubic cell, or pass through 3-tuples."""
    n3 = tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))
    l3 = tuple(float(v) for v in (L if np.ndim(L) else (L, L, L)))
    return n3, l3


def _g2_grid(n3, l3):
    """|G|^2 on the (nz, ny, nx) grid, fftfreq order."""
    nx, ny, nz = n3
    lx, ly, lz = l3
    gx = 2 * np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / lx
    gy = 2 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / ly
    gz = 2 * np.pi * np.fft.fftfreq(nz, d=1.0 / nz) / lz
    return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2


def make_orbitals(seed, n, L, N, ecut=ECUT_HA, dtype=np.complex128, workers=None):
    """N orthonormal orbitals on an n^3 (or n3) grid of a cell with edge(s) L.

    Returns an array of shape (N, nz, ny, nx) and the given dtype.  complex64
    output is the complex128 result rounded once.
    """
    n3, l3 = cell_of(n, L)
    nx, ny, nz = n3
    nr = nx * ny * nz
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    g2 = _g2_grid(n3, l3)
    mask = 0.5 * g2 < ecut
    idx = np.flatnonzero(mask.ravel())  # C order of (iz, iy, ix)
    npw = idx.size
    if npw < N:
        raise ValueError(f"only {npw} planewaves below the cutoff for {N} orbitals")
    rng = np.random.default_rng(seed)
    draw = rng.standard_normal((N, npw, 2))
    amp = np.exp(-g2.ravel()[idx] / 4.0)
    coef = (draw[..., 0] + 1j * draw[..., 1]) * amp[None, :]  # (N, npw)
    del draw
    # Loewdin: rows are orbitals, S_ij = <c_i, c_j>
    s = coef.conj() @ coef.T
    s = 0.5 * (s + s.conj().T)
    w, v = np.linalg.eigh(s)
    s_inv_half = (v * (1.0 / np.sqrt(w))[None, :]) @ v.conj().T
    # new row i = sum_j (S^{-1/2})_{ji} c_j  ->  C' = (S^{-1/2})^T C
    coef = s_inv_half.T @ coef
    out = np.empty((N, nz, ny, nx), dtype=dtype)
    scale = np.sqrt(nr)
    chunk = max(1, min(N, int(2e8 // (nr * 16))))
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        full = np.zeros((c1 - c0, nr), dtype=np.complex128)
        full[:, idx] = coef[c0:c1]
        full = full.reshape(c1 - c0, nz, ny, nx)
        grid = _ifftn_batch(full, workers)
        out[c0:c1] = grid * scale
    return out


def _ifftn_batch(a, workers):
    if _sfft is not None:
        return _sfft.ifftn(a, axes=(1, 2, 3), workers=workers)
    return np.fft.ifftn(a, axes=(1, 2, 3))


def planewave_orbitals(n, L, mvecs, dtype=np.complex128):
    """Planewaves e_G(r) = exp(i G.r)/sqrt(N_r) for integer index triples (mx, my, mz).

    G.r on the grid is 2*pi*(mx*ix/nx + my*iy/ny + mz*iz/nz); the result is
    orthonormal for distinct index triples modulo the grid.
    """
    n3, _ = cell_of(n, L)
    nx, ny, nz = n3
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.empty((len(mvecs), nz, ny, nx), dtype=dtype)
    for i, (mx, my, mz) in enumerate(mvecs):
        ph = 2 * np.pi * (mx * ix / nx + my * iy / ny + mz * iz / nz)
        out[i] = np.exp(1j * ph) / np.sqrt(nx * ny * nz)
    return out


def random_unitary(seed, N):
    """Haar-ish random unitary (QR of a complex Gaussian), for gauge tests."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def random_grid_vectors(seed, n, count, dtype=np.complex128):
    """Unstructured complex grid vectors (not band limited), for operator tests."""
    n3, _ = cell_of(n, 1.0)
    nx, ny, nz = n3
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((count, nz, ny, nx, 2))
    return (a[..., 0] + 1j * a[..., 1]).astype(dtype)
