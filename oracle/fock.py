"""Plain FP64 definitions of V_X, the exchange energy, ACE, the kinetic operator, and the
end-of-step operations (PT residual, Cholesky-QR re-orthonormalisation, density) (test
infrastructure).

Conventions (readings of the paper, each listed in the design notes):
  * An orbital is a Euclidean-normalised grid vector on an nx*ny*nz grid of a
    box with edges (lx, ly, lz), stored as an array (nz, ny, nx), x fastest.
  * FFT_u / IFFT_u are the unnormalised DFT pair (exp(-i..) forward).  numpy's
    ifftn carries 1/N_r, so IFFT_u = N_r * ifftn.
  * With Euclidean orbitals the continuum operator of the paper's equation for
    applying V_X (Sec. 2, Eq. "applyVX") reads
        (V_X phi_k) = -(1/Omega) sum_j psi_j * IFFT_u[ K * FFT_u( conj(psi_j) phi_k ) ],
    the sum running over all orbitals j, for every target k (the double loop
    of the Fock-application algorithm in Sec. 3.2).  The mixing fraction alpha
    of the kernel definition in Sec. 2 enters as ``scale``.
  * K(G): Coulomb 4 pi/|G|^2 with K(0) = 0; screened (HSE-type)
    4 pi/|G|^2 (1 - exp(-|G|^2/(4 w^2))) with K(0) = pi/w^2, its G -> 0 limit.
    The paper only names the screened kernel it uses (Sec. 2, Sec. 4).
  * ACE (cited in Sec. 1, not defined in the paper): W = V_X Psi, M = Psi^H W,
    Hermitised; -M = L L^H with L lower triangular, real positive diagonal;
    xi = W L^{-H}; K_ACE phi = -xi (xi^H phi).  E_X = 1/2 Re tr(Psi^H V_X Psi).

Arrays of orbitals have shape (N, nz, ny, nx) or (N, N_r).
"""
from __future__ import annotations

import numpy as np

try:
    import scipy.fft as _fft
    import scipy.linalg as _sla
except Exception:  # pragma: no cover
    _fft = None
    _sla = None

# What pins each function (tests/test_oracle_*.py).  None is unpinned.
PINS = {
    "g2_grid": "naive DFT eigen-relation and closed-form planewave test",
    "kernel_table": "series limits (HSE->Coulomb as w->0, continuity at G=0) and planewave closed form",
    "pair_potential": "brute-force circular convolution with the real-space kernel; naive O(N_r^2) DFT",
    "apply_vx": "planewave closed form; brute-force real-space double sum; Hermiticity; sign; gauge invariance",
    "exchange_energy": "planewave closed form of the trace",
    "build_ace": "planewave closed form of M and L; K_ACE psi_i = W_i; tr M = -||L||_F^2",
    "apply_ace": "exactness on span(Psi); annihilation of the orthogonal complement; Hermitian NSD rank <= N",
    "apply_kinetic": "planewave closed form |G|^2/2 (Nyquist rows, orthorhombic cell); second differences of a "
                     "band-limited function against the exact Laplacian; Hermitian and positive semidefinite",
    "pt_residual": "planewave eigenbasis (H Psi = Psi Lambda gives R = Psi - Psi_half); projections onto span(Psi) "
                   "(zero) and onto its complement from a complete Householder QR ((i dt/2) Q_perp^H H Psi); gauge "
                   "covariance",
    "orthonormalize": "equals the Householder QR factor with a positive real diagonal; Q^H Q = I; span preserved",
    "density": "planewave orbitals give the constant N/N_r; gauge invariance under unitary mixing; sum rule",
}


def _as_n3(n):
    return tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))


def _as_l3(L):
    return tuple(float(v) for v in (L if np.ndim(L) else (L, L, L)))


def volume(L):
    lx, ly, lz = _as_l3(L)
    return lx * ly * lz


def g2_grid(n, L):
    """|G|^2 on the (nz, ny, nx) grid; G_a = 2 pi m_a / L_a with m_a in fftfreq order.

    This is the reciprocal grid of the planewave discretisation (Sec. 2, the
    FFT solution of the Poisson-like equations).
    """
    nx, ny, nz = _as_n3(n)
    lx, ly, lz = _as_l3(L)
    gx = 2.0 * np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / lx
    gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / ly
    gz = 2.0 * np.pi * np.fft.fftfreq(nz, d=1.0 / nz) / lz
    return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2


def kernel_table(n, L, kind="coulomb", omega=0.106, scale=1.0):
    """K(G) on the FFT grid (kernel of V_X, Sec. 2; screened form used in Sec. 4).

    kind: "coulomb" (or 0) -> 4 pi/|G|^2, K(0) = 0;
          "hse" (or 1)     -> 4 pi/|G|^2 (1 - exp(-|G|^2/(4 omega^2))), K(0) = pi/omega^2.
    ``scale`` multiplies the table (the mixing fraction alpha).
    """
    g2 = g2_grid(n, L)
    k = np.zeros_like(g2)
    nz0 = g2 > 0
    if kind in ("coulomb", 0):
        k[nz0] = 4.0 * np.pi / g2[nz0]
        k[~nz0] = 0.0
    elif kind in ("hse", 1):
        k[nz0] = 4.0 * np.pi / g2[nz0] * (1.0 - np.exp(-g2[nz0] / (4.0 * omega * omega)))
        k[~nz0] = np.pi / (omega * omega)
    else:
        raise ValueError(f"unknown kernel kind {kind!r}")
    return k * scale


def _fftn(a, workers):
    if _fft is not None:
        return _fft.fftn(a, workers=workers)
    return np.fft.fftn(a)


def _ifftn(a, workers):
    if _fft is not None:
        return _fft.ifftn(a, workers=workers)
    return np.fft.ifftn(a)


def pair_potential(psi_j, phi_k, K, workers=1):
    """IFFT_u[ K * FFT_u( conj(psi_j) * phi_k ) ]: one Poisson-like solve (Sec. 2, after Eq. applyVX).

    psi_j, phi_k: (nz, ny, nx) complex; K: (nz, ny, nx) real.  Returns (nz, ny, nx).
    """
    rho = np.conj(psi_j) * phi_k
    f = _fftn(rho, workers) * K
    return _ifftn(f, workers) * rho.size


def _grid(a, n):
    nx, ny, nz = _as_n3(n)
    a = np.asarray(a)
    return a.reshape(a.shape[0], nz, ny, nx)


def apply_vx(psi, phi, n, L, kind="coulomb", omega=0.106, scale=1.0, targets=None, workers=1):
    """V_X[Psi] applied to the targets phi_k (Eq. applyVX; loop structure of the Fock algorithm, Sec. 3.2).

    For each target k and each orbital j in ascending order: form the pair
    density conj(psi_j) phi_k, solve the Poisson-like equation through the FFT,
    multiply by psi_j and add; finally scale by -1/Omega.

    psi: (N, ...) orbitals; phi: (N_t, ...) targets; ``targets`` selects a
    subset of target indices (default: all).  Returns complex128 (len(targets), nz, ny, nx).
    """
    psi = _grid(psi, n).astype(np.complex128)
    phi = _grid(phi, n).astype(np.complex128)
    K = kernel_table(n, L, kind, omega, scale)
    omega_vol = volume(L)
    ks = range(phi.shape[0]) if targets is None else list(targets)
    out = np.zeros((len(ks),) + psi.shape[1:], dtype=np.complex128)
    for t, k in enumerate(ks):
        acc = np.zeros(psi.shape[1:], dtype=np.complex128)
        for j in range(psi.shape[0]):
            acc += psi[j] * pair_potential(psi[j], phi[k], K, workers)
        out[t] = -acc / omega_vol
    return out


def exchange_energy(psi, w):
    """E_X = 1/2 Re sum_k <psi_k, (V_X psi)_k> (one Fock application per energy evaluation, Sec. 7)."""
    p = np.asarray(psi).reshape(np.shape(psi)[0], -1).astype(np.complex128)
    v = np.asarray(w).reshape(np.shape(w)[0], -1).astype(np.complex128)
    return 0.5 * float(np.real(np.sum(np.conj(p) * v)))


def build_ace(psi, w):
    """ACE factors from Psi and W = V_X Psi (ACE is cited in Sec. 1; definitions as stated in the module doc).

    Returns dict(M, L, xi, ex): M (N, N) Hermitised Psi^H W; L the lower
    Cholesky factor of -M; xi (N, N_r) rows = columns of W L^{-H}; ex = 1/2 Re tr M.
    Raises numpy.linalg.LinAlgError when -M is not positive definite.
    """
    P = np.asarray(psi).reshape(np.shape(psi)[0], -1).astype(np.complex128).T  # N_r x N
    Wm = np.asarray(w).reshape(np.shape(w)[0], -1).astype(np.complex128).T  # N_r x N
    M = P.conj().T @ Wm
    M = 0.5 * (M + M.conj().T)
    L = np.linalg.cholesky(-M)
    # xi L^H = W  <=>  L xi^H = W^H
    if _sla is not None:
        xiH = _sla.solve_triangular(L, Wm.conj().T, lower=True)
    else:  # pragma: no cover
        xiH = np.linalg.solve(L, Wm.conj().T)
    xi = xiH.conj().T  # N_r x N
    return dict(M=M, L=L, xi=xi.T.copy(), ex=0.5 * float(np.real(np.trace(M))))


def apply_ace(xi, phi):
    """K_ACE phi = -xi (xi^H phi) for xi given as rows (N, N_r) and phi as (R, ...)."""
    X = np.asarray(xi).reshape(np.shape(xi)[0], -1).astype(np.complex128).T  # N_r x N
    shp = np.shape(phi)
    F = np.asarray(phi).reshape(shp[0], -1).astype(np.complex128).T  # N_r x R
    Y = -(X @ (X.conj().T @ F))
    return Y.T.reshape(shp)


def vx_dense_matrix(psi, n, L, kind="coulomb", omega=0.106, scale=1.0):
    """The N_r x N_r matrix of V_X[Psi], column c = V_X applied to the unit vector e_c (tiny grids only)."""
    nx, ny, nz = _as_n3(n)
    nr = nx * ny * nz
    eye = np.eye(nr, dtype=np.complex128).reshape(nr, nz, ny, nx)
    cols = apply_vx(psi, eye, n, L, kind, omega, scale)
    return cols.reshape(nr, nr).T


def apply_kinetic(phi, n, L):
    """Kinetic operator -(1/2) Laplacian of the Hamiltonian (Sec. 2) applied to each orbital of phi.

    On the periodic grid it is diagonal in the planewave basis: each planewave
    coefficient of phi is multiplied by |G|^2/2 (G as in g2_grid, so the
    Nyquist row of an even edge has |G_a| = pi n_a / L_a).  Returns complex128
    with the shape (N, nz, ny, nx).
    """
    phi = _grid(phi, n).astype(np.complex128)
    half_g2 = 0.5 * g2_grid(n, L)
    out = np.empty_like(phi)
    for k in range(phi.shape[0]):
        out[k] = np.fft.ifftn(half_g2 * np.fft.fftn(phi[k]))
    return out


def _cols(a):
    """Orbitals (N, ...) as the columns of an N_r x N matrix."""
    a = np.asarray(a)
    return a.reshape(a.shape[0], -1).T


def pt_residual(psi_f, hpsi_f, psi_half, dt):
    """Residual R_f of the PT-CN fixed point (the residual algorithm of Sec. 3.3, for the PT equation of Sec. 2).

    S = Psi_f^H (H_f Psi_f); Psi_temp = Psi_f S; R_f = Psi_f + (i dt/2)(H_f Psi_f - Psi_temp) - Psi_{n+1/2}.
    All three inputs are orbital blocks of the same shape (N, ...); so is the result.
    """
    X = _cols(psi_f).astype(np.complex128)
    HX = _cols(hpsi_f).astype(np.complex128)
    Xh = _cols(psi_half).astype(np.complex128)
    S = X.conj().T @ HX
    T = X @ S
    R = X + 0.5j * dt * (HX - T) - Xh
    return R.T.reshape(np.shape(psi_f))


def orthonormalize(psi):
    """Re-orthonormalisation at the end of a time step (Sec. 3.4): overlap S = Psi^H Psi, Cholesky
    S = L L^H (L lower, real positive diagonal), then Psi L^{-H}."""
    X = _cols(psi).astype(np.complex128)
    S = X.conj().T @ X
    S = 0.5 * (S + S.conj().T)
    L = np.linalg.cholesky(S)
    Z = _sla.solve_triangular(L, X.conj().T, lower=True)  # L^{-1} X^H = (X L^{-H})^H
    return Z.conj().reshape(np.shape(psi))


def density(psi, occ=None):
    """Electron density rho(r) = sum_i f_i |psi_i(r)|^2 (Sec. 3.4, where every f_i = 1)."""
    a = np.asarray(psi)
    X = a.reshape(a.shape[0], -1).astype(np.complex128)
    f = np.ones(a.shape[0]) if occ is None else np.asarray(occ, dtype=np.float64)
    rho = np.zeros(X.shape[1])
    for i in range(X.shape[0]):
        rho += f[i] * (X[i].real ** 2 + X[i].imag ** 2)
    return rho.reshape(a.shape[1:])

