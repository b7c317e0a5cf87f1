"""Pins for the FP64 oracle: checks against things other than the oracle itself.

Each check returns the observed error (a float); the tests compare it with a
bound.  The same checks run against deliberately broken copies of the oracle
(tests/test_oracle_mutations.py) to show that a plausible mistake is caught.

What each check rests on:
  naive_dft        - an explicit O(N^2) DFT matrix, the textbook definition.
  brute_convolution- a direct real-space circular convolution with the kernel
                     synthesised by an explicit Fourier sum.
  planewave        - the closed form for planewave orbitals: V_X e_Gk =
                     -(1/Omega) sum_j K(Gk - Gj) e_Gk (exact on the grid).
  continuum        - the continuum operator with continuum-normalised orbitals
                     and a convolution integral, related to the grid operator
                     by the quadrature weight Omega/N_r.
  erf_potential    - the screened potential of a Gaussian charge in closed form
                     (erf(sqrt(a) r)/r - erf(mu r)/r, 1/mu^2 = 1/a + 1/w^2).
  fd_poisson       - a fourth-order finite-difference Laplacian of the Coulomb
                     potential reproduces 4 pi (rho - mean rho).
  hermitian / nsd  - properties of any operator -sum_j P K P with real even K.
  gauge / pair symmetry / linearity / translation - exact invariants.
  ace_*            - algebraic identities of the ACE factorisation.
"""
from __future__ import annotations

import numpy as np

import synth


def _mgrid(n3):
    nx, ny, nz = n3
    mx = np.fft.fftfreq(nx, d=1.0 / nx)
    my = np.fft.fftfreq(ny, d=1.0 / ny)
    mz = np.fft.fftfreq(nz, d=1.0 / nz)
    return mx, my, mz


def naive_dft3(a, sign=-1):
    """Unnormalised 3D DFT of a (nz, ny, nx) array by explicit per-axis DFT matrices."""
    nz, ny, nx = a.shape

    def mat(n):
        idx = np.arange(n)
        return np.exp(sign * 2j * np.pi * np.outer(idx, idx) / n)

    out = np.einsum("kx,zyx->zyk", mat(nx), a)
    out = np.einsum("ky,zyx->zkx", mat(ny), out)
    out = np.einsum("kz,zyx->kyx", mat(nz), out)
    return out


def check_naive_dft(orc, n3=(4, 9, 6), L3=(3.0, 5.0, 4.0), seed=0):
    """pair_potential equals IFFT_u(K . FFT_u(conj(a) b)) with explicit DFT matrices."""
    nx, ny, nz = n3
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    b = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    K = orc.kernel_table(n3, L3, "hse", 0.3)
    ref = naive_dft3(K * naive_dft3(np.conj(a) * b, -1), +1)
    got = orc.pair_potential(a, b, K)
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def _kernel_formula(kind, g2, omega):
    """K(|G|^2) written out from the workload definitions, evaluated pointwise."""
    out = np.empty_like(g2)
    for i, v in np.ndenumerate(g2):
        if v == 0.0:
            out[i] = 0.0 if kind == "coulomb" else np.pi / omega**2
        elif kind == "coulomb":
            out[i] = 4 * np.pi / v
        else:
            out[i] = 4 * np.pi / v * (1 - np.exp(-v / (4 * omega**2)))
    return out


def check_brute_convolution(orc, kind="hse", n3=(4, 3, 6), L3=(2.5, 3.5, 4.0), omega=0.4, seed=1):
    """pair_potential = N_r * sum_r' Kt(r - r') rho(r') with Kt(d) = (1/N_r) sum_G K(G) e^{i G.d}."""
    nx, ny, nz = n3
    lx, ly, lz = L3
    nr = nx * ny * nz
    mx, my, mz = _mgrid(n3)
    # all (m, G) in a flat list, independent of the oracle's table layout
    M = np.array([(a, b, c) for c in mz for b in my for a in mx])
    G = 2 * np.pi * M / np.array([lx, ly, lz])
    Kg = _kernel_formula(kind, np.sum(G**2, axis=1), omega)
    R = np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)])
    # Kt(d) for every grid offset d
    frac = R / np.array([nx, ny, nz])  # d / n per axis
    Kt = (np.exp(2j * np.pi * (frac @ M.T)) @ Kg) / nr  # indexed like R
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
    b = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
    rho = np.conj(a) * b
    v = np.zeros(nr, dtype=complex)
    for i in range(nr):
        d = (R[i][None, :] - R) % np.array([nx, ny, nz])
        di = d[:, 0] + nx * (d[:, 1] + ny * d[:, 2])
        v[i] = nr * np.sum(Kt[di] * rho)
    K = orc.kernel_table(n3, L3, kind, omega)
    got = orc.pair_potential(a.reshape(nz, ny, nx), b.reshape(nz, ny, nx), K).ravel()
    return float(np.abs(got - v).max() / np.abs(v).max())


def _wrap(m, n):
    """Integer index m folded into numpy's fftfreq range for a grid of n."""
    m = m % n
    return m - n if m >= (n + 1) // 2 else m


def check_planewave(orc, kind="hse", n3=(6, 6, 6), L3=(5.0, 5.0, 5.0), omega=0.3, mvecs=None):
    """V_X[e_Gj] e_Gk = -(1/Omega) sum_j K(wrap(Gk - Gj)) e_Gk, including a Nyquist-wrapped G."""
    nx, ny, nz = n3
    if mvecs is None:
        mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (3, 1, -1), (-2, 2, 1)]
    psi = synth.planewave_orbitals(n3, L3, mvecs)
    out = orc.apply_vx(psi, psi, n3, L3, kind, omega)
    omega_vol = L3[0] * L3[1] * L3[2]
    err = 0.0
    for k, mk in enumerate(mvecs):
        lam = 0.0
        for mj in mvecs:
            d = [_wrap(mk[a] - mj[a], n3[a]) for a in range(3)]
            g2 = sum((2 * np.pi * d[a] / L3[a]) ** 2 for a in range(3))
            lam += _kernel_formula(kind, np.array([g2]), omega)[0]
        ref = -lam / omega_vol * psi[k]
        err = max(err, float(np.abs(out[k] - ref).max() / np.abs(ref).max()))
    return err


def check_continuum(orc, kind="hse", n3=(8, 6, 10), L3=(6.0, 4.5, 7.0), omega=0.5, N=3, seed=2):
    """Grid operator on Euclidean orbitals = sqrt(dV) x continuum operator on psi/sqrt(dV).

    The continuum operator is built from a convolution integral evaluated by
    the rectangle rule (spectrally exact for band-limited data) with the
    real-space kernel synthesised from K(G) by a Fourier series; no -1/Omega
    factor appears in it.
    """
    nx, ny, nz = n3
    nr = nx * ny * nz
    dV = L3[0] * L3[1] * L3[2] / nr
    psi = synth.make_orbitals(seed, n3, L3, N, ecut=30.0)
    phi = synth.make_orbitals(seed + 1, n3, L3, 2, ecut=30.0)
    mx, my, mz = _mgrid(n3)
    M = np.array([(a, b, c) for c in mz for b in my for a in mx])
    Gs = 2 * np.pi * M / np.array(L3)
    Kg = _kernel_formula(kind, np.sum(Gs**2, axis=1), omega)
    R = np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)])
    # continuum kernel Kt(d) = (1/Omega) sum_G K(G) e^{iG.d}
    Kt = (np.exp(2j * np.pi * ((R / np.array([nx, ny, nz])) @ M.T)) @ Kg) / (L3[0] * L3[1] * L3[2])
    pc = psi.reshape(N, nr) / np.sqrt(dV)
    fc = phi.reshape(2, nr) / np.sqrt(dV)
    D = (R[:, None, :] - R[None, :, :]) % np.array([nx, ny, nz])
    Dflat = D[..., 0] + nx * (D[..., 1] + ny * D[..., 2])
    Kmat = Kt[Dflat]  # Kt(r - r')
    out_c = np.zeros((2, nr), dtype=complex)
    for k in range(2):
        for j in range(N):
            out_c[k] -= pc[j] * (Kmat @ (np.conj(pc[j]) * fc[k]) * dV)
    ref = np.sqrt(dV) * out_c
    got = orc.apply_vx(psi, phi, n3, L3, kind, omega).reshape(2, nr)
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def check_erf_potential(orc, n=64, L=30.0, alpha=0.5, omega=0.5):
    """Screened potential of a unit Gaussian charge: erf(sqrt(a) r)/r - erf(mu r)/r.

    The periodic images are negligible here (erfc(omega*L/2) ~ 1e-25).  The
    potential is v = ifftn(K fftn(rho)), i.e. pair_potential(1, rho)/N_r.
    """
    from scipy.special import erf

    n3 = (n, n, n)
    h = L / n
    x = (np.arange(n) - n // 2) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt(X**2 + Y**2 + Z**2)
    rho = (alpha / np.pi) ** 1.5 * np.exp(-alpha * r**2)
    K = orc.kernel_table(n3, (L, L, L), "hse", omega)
    v = orc.pair_potential(np.ones_like(rho, dtype=complex), rho.astype(complex), K) / rho.size
    mu = 1.0 / np.sqrt(1.0 / alpha + 1.0 / omega**2)
    sel = (r > 0.5) & (r < 8.0)
    ref = erf(np.sqrt(alpha) * r[sel]) / r[sel] - erf(mu * r[sel]) / r[sel]
    # value at the centre: limit 2 (sqrt(a) - mu)/sqrt(pi)
    c = (n // 2, n // 2, n // 2)
    ref0 = 2 * (np.sqrt(alpha) - mu) / np.sqrt(np.pi)
    e1 = np.abs(v.real[sel] - ref).max() / np.abs(ref).max()
    e2 = abs(v.real[c] - ref0) / abs(ref0)
    return float(max(e1, e2))


def check_fd_poisson(orc, n=48, L=12.0, alpha=1.2):
    """-Laplacian_h v = 4 pi (rho - mean rho) + O(h^4) for the Coulomb kernel (K(0) = 0)."""
    n3 = (n, n, n)
    h = L / n
    x = (np.arange(n) - n // 2) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho = np.exp(-alpha * ((X - 0.3) ** 2 + Y**2 + (Z + 0.2) ** 2))
    K = orc.kernel_table(n3, (L, L, L), "coulomb")
    v = (orc.pair_potential(np.ones_like(rho, dtype=complex), rho.astype(complex), K) / rho.size).real
    # fourth-order central difference stencil
    lap = sum(-np.roll(v, 2, a) + 16 * np.roll(v, 1, a) - 30 * v + 16 * np.roll(v, -1, a) - np.roll(v, -2, a)
              for a in range(3)) / (12 * h**2)
    rhs = 4 * np.pi * (rho - rho.mean())
    return float(np.abs(-lap - rhs).max() / np.abs(rhs).max())


def check_kernel_limits(orc):
    """HSE -> Coulomb for G != 0 as omega -> 0; HSE continuous at G -> 0 (limit pi/omega^2)."""
    n3, L3 = (6, 6, 6), (4.0, 4.0, 4.0)
    kc = orc.kernel_table(n3, L3, "coulomb")
    kh = orc.kernel_table(n3, L3, "hse", 1e-3)
    m = kc > 0
    e1 = np.abs(kh[m] - kc[m]).max() / kc[m].max()
    # continuity: a huge cell makes the smallest nonzero G tiny
    om = 0.3
    Lb = 1e4
    kb = orc.kernel_table((4, 4, 4), (Lb, Lb, Lb), "hse", om)
    e2 = abs(kb[0, 0, 1] - kb[0, 0, 0]) / kb[0, 0, 0]
    e3 = abs(kb[0, 0, 0] - np.pi / om**2) / (np.pi / om**2)
    return float(max(e1, e2, e3))


def _random_case(seed=3, n3=(6, 4, 5), L3=(4.0, 3.0, 3.5), N=4):
    psi = synth.make_orbitals(seed, n3, L3, N, ecut=40.0)
    return psi, n3, L3


def check_hermitian(orc, kind="hse"):
    psi, n3, L3 = _random_case()
    A = orc.vx_dense_matrix(psi, n3, L3, kind, 0.4)
    return float(np.abs(A - A.conj().T).max() / np.abs(A).max())


def check_nsd(orc, kind="hse"):
    """Largest eigenvalue of V_X: <= 0 (Coulomb), < 0 (HSE, K > 0).  Returns max eigenvalue / norm."""
    psi, n3, L3 = _random_case()
    A = orc.vx_dense_matrix(psi, n3, L3, kind, 0.4)
    A = 0.5 * (A + A.conj().T)
    ev = np.linalg.eigvalsh(A)
    return float(ev.max() / np.abs(ev).max())


def check_gauge(orc, kind="hse", seed=4):
    psi, n3, L3 = _random_case()
    N = psi.shape[0]
    U = synth.random_unitary(seed, N)
    psiU = np.einsum("jzyx,jk->kzyx", psi, U)
    phi = synth.random_grid_vectors(seed, n3, 2)
    a = orc.apply_vx(psi, phi, n3, L3, kind, 0.4)
    b = orc.apply_vx(psiU, phi, n3, L3, kind, 0.4)
    return float(np.abs(a - b).max() / np.abs(a).max())


def check_pair_symmetry(orc, kind="hse"):
    psi, n3, L3 = _random_case()
    K = orc.kernel_table(n3, L3, kind, 0.4)
    v01 = orc.pair_potential(psi[0], psi[1], K)
    v10 = orc.pair_potential(psi[1], psi[0], K)
    return float(np.abs(v10 - np.conj(v01)).max() / np.abs(v01).max())


def check_linearity_scaling(orc, kind="hse", seed=5):
    psi, n3, L3 = _random_case()
    phi = synth.random_grid_vectors(seed, n3, 2)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    lhs = orc.apply_vx(psi, (a * phi[0] + b * phi[1])[None], n3, L3, kind, 0.4)[0]
    o = orc.apply_vx(psi, phi, n3, L3, kind, 0.4)
    rhs = a * o[0] + b * o[1]
    e1 = np.abs(lhs - rhs).max() / np.abs(rhs).max()
    c = 1.7 - 0.6j
    oc = orc.apply_vx(c * psi, phi, n3, L3, kind, 0.4)
    e2 = np.abs(oc - abs(c) ** 2 * o).max() / np.abs(o).max()
    return float(max(e1, e2))


def check_translation(orc, kind="hse", seed=6):
    psi, n3, L3 = _random_case()
    phi = synth.random_grid_vectors(seed, n3, 1)
    sh = (1, 2, 3)  # (z, y, x) shift
    o = orc.apply_vx(psi, phi, n3, L3, kind, 0.4)
    os_ = orc.apply_vx(np.roll(psi, sh, (1, 2, 3)), np.roll(phi, sh, (1, 2, 3)), n3, L3, kind, 0.4)
    return float(np.abs(os_ - np.roll(o, sh, (1, 2, 3))).max() / np.abs(o).max())


def check_exchange_energy(orc, kind="hse", n3=(6, 6, 6), L3=(5.0, 5.0, 5.0), omega=0.3):
    """E_X for planewaves: -(1/(2 Omega)) sum_{j,k} K(Gk - Gj)."""
    mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (3, 1, -1)]
    psi = synth.planewave_orbitals(n3, L3, mvecs)
    w = orc.apply_vx(psi, psi, n3, L3, kind, omega)
    ex = orc.exchange_energy(psi, w)
    ref = 0.0
    for mk in mvecs:
        for mj in mvecs:
            d = [_wrap(mk[a] - mj[a], n3[a]) for a in range(3)]
            g2 = sum((2 * np.pi * d[a] / L3[a]) ** 2 for a in range(3))
            ref += _kernel_formula(kind, np.array([g2]), omega)[0]
    ref *= -0.5 / (L3[0] * L3[1] * L3[2])
    return float(abs(ex - ref) / abs(ref))


def check_ace_planewave(orc, n3=(6, 6, 6), L3=(5.0, 5.0, 5.0), omega=0.3):
    """For planewave Psi, M is diagonal with M_kk = -(1/Omega) sum_j K(Gk - Gj) and L = diag(sqrt(-M_kk))."""
    mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (3, 1, -1)]
    psi = synth.planewave_orbitals(n3, L3, mvecs)
    w = orc.apply_vx(psi, psi, n3, L3, "hse", omega)
    ace = orc.build_ace(psi, w)
    ref = np.zeros(len(mvecs))
    for k, mk in enumerate(mvecs):
        for mj in mvecs:
            d = [_wrap(mk[a] - mj[a], n3[a]) for a in range(3)]
            g2 = sum((2 * np.pi * d[a] / L3[a]) ** 2 for a in range(3))
            ref[k] -= _kernel_formula("hse", np.array([g2]), omega)[0] / (L3[0] * L3[1] * L3[2])
    e1 = np.abs(ace["M"] - np.diag(ref)).max() / np.abs(ref).max()
    e2 = np.abs(ace["L"] - np.diag(np.sqrt(-ref))).max() / np.sqrt(np.abs(ref).max())
    return float(max(e1, e2))


def check_ace_identities(orc, kind="hse", seed=7):
    """K_ACE psi_i = W_i; tr M = -||L||_F^2; K_ACE kills span(W)^perp; Hermitian NSD, rank <= N; gauge-free."""
    psi, n3, L3 = _random_case(seed=seed, N=4)
    N = psi.shape[0]
    nr = int(np.prod(n3))
    w = orc.apply_vx(psi, psi, n3, L3, kind, 0.4)
    ace = orc.build_ace(psi, w)
    errs = []
    kp = orc.apply_ace(ace["xi"], psi)
    errs.append(np.abs(kp - w).max() / np.abs(w).max())
    errs.append(abs(np.trace(ace["M"]).real + np.linalg.norm(ace["L"]) ** 2) / abs(np.trace(ace["M"]).real))
    # a vector orthogonal to span(W) is annihilated
    Wm = w.reshape(N, nr).T
    q, _ = np.linalg.qr(Wm)
    z = synth.random_grid_vectors(seed, n3, 1).reshape(nr)
    z = z - q @ (q.conj().T @ z)
    kz = orc.apply_ace(ace["xi"], z.reshape((1,) + psi.shape[1:]))
    errs.append(np.abs(kz).max() / np.abs(orc.apply_ace(ace["xi"], psi)).max())
    # dense K_ACE: Hermitian, NSD, rank <= N
    eye = np.eye(nr, dtype=complex).reshape((nr,) + psi.shape[1:])
    A = orc.apply_ace(ace["xi"], eye).reshape(nr, nr).T
    errs.append(np.abs(A - A.conj().T).max() / np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
    errs.append(max(0.0, ev.max()) / np.abs(ev).max())
    errs.append(np.sort(np.abs(ev))[::-1][N] / np.abs(ev).max())
    # gauge: K_ACE built from Psi U equals K_ACE built from Psi
    U = synth.random_unitary(seed, N)
    psiU = np.einsum("jzyx,jk->kzyx", psi, U)
    wU = orc.apply_vx(psiU, psiU, n3, L3, kind, 0.4)
    aceU = orc.build_ace(psiU, wU)
    AU = orc.apply_ace(aceU["xi"], eye).reshape(nr, nr).T
    errs.append(np.abs(AU - A).max() / np.abs(A).max())
    # K_ACE = V_X on span(Psi): <psi_i, K_ACE psi_j> = M_ij
    errs.append(np.abs(psi.reshape(N, nr).conj() @ kp.reshape(N, nr).T - ace["M"]).max() / np.abs(ace["M"]).max())
    return float(max(errs))


def _planewave_block(n3, L3, mvecs):
    """Orthonormal planewave orbitals e^{i G.r}/sqrt(N_r), rows (N, nz, ny, nx); written here, not in synth."""
    nx, ny, nz = n3
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    nr = nx * ny * nz
    return np.array([np.exp(2j * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)) / np.sqrt(nr)
                     for m in mvecs])


def _random_hermitian(rng, n):
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (a + a.conj().T)


def check_residual_eigenbasis(orc, n3=(6, 4, 5), L3=(4.0, 3.0, 3.5), omega=0.3, dt=0.37, seed=8):
    """Planewaves are eigenvectors of V_X (eigenvalue from the closed form of Eq. applyVX): then
    H Psi - Psi (Psi^H H Psi) = 0 and the residual reduces to Psi - Psi_half for any dt."""
    mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (2, 1, -1)]
    psi = _planewave_block(n3, L3, mvecs)
    lam = []
    for mk in mvecs:
        acc = 0.0
        for mj in mvecs:
            d = [_wrap(mk[a] - mj[a], n3[a]) for a in range(3)]
            g2 = sum((2 * np.pi * d[a] / L3[a]) ** 2 for a in range(3))
            acc += _kernel_formula("hse", np.array([g2]), omega)[0]
        lam.append(-acc / np.prod(L3))
    hpsi = np.array(lam)[:, None, None, None] * psi
    rng = np.random.default_rng(seed)
    half = rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape)
    r = orc.pt_residual(psi, hpsi, half, dt)
    return float(np.abs(r - (psi - half)).max())


def _residual_case(seed, nr=40, n=5):
    rng = np.random.default_rng(seed)
    x, _ = np.linalg.qr(rng.standard_normal((nr, n)) + 1j * rng.standard_normal((nr, n)))
    h = _random_hermitian(rng, nr)
    half = rng.standard_normal((nr, n)) + 1j * rng.standard_normal((nr, n))
    return x, h, half


def check_residual_projections(orc, dt=0.29, seed=9):
    """R - Psi + Psi_half is fixed by its two projections: onto span(Psi) it vanishes (S is the
    overlap Psi^H H Psi), onto the orthogonal complement (a basis from a complete Householder QR)
    it equals (i dt/2) Q_perp^H (H Psi).  Sensitive to the sign and size of the i dt/2 factor."""
    x, h, half = _residual_case(seed)
    hx = h @ x
    r = orc.pt_residual(x.T, hx.T, half.T, dt).T
    d = r - x + half
    q, _ = np.linalg.qr(x, mode="complete")
    qp = q[:, x.shape[1]:]
    e1 = np.abs(x.conj().T @ d).max()
    e2 = np.abs(qp.conj().T @ d - 0.5j * dt * (qp.conj().T @ hx)).max()
    return float(max(e1, e2) / max(1.0, np.abs(hx).max()))


def check_residual_gauge(orc, dt=0.41, seed=10):
    """Gauge covariance: Psi -> Psi U (U unitary, H Psi and Psi_half transformed alike) gives R U."""
    x, h, half = _residual_case(seed)
    rng = np.random.default_rng(seed + 1)
    u, _ = np.linalg.qr(rng.standard_normal((x.shape[1],) * 2) + 1j * rng.standard_normal((x.shape[1],) * 2))
    r = orc.pt_residual(x.T, (h @ x).T, half.T, dt).T
    ru = orc.pt_residual((x @ u).T, (h @ x @ u).T, (half @ u).T, dt).T
    return float(np.abs(ru - r @ u).max())


def check_cholqr_vs_householder(orc, seed=11, nr=60, n=7):
    """Cholesky-QR of a full-rank block equals its Householder QR factor Q with the phases that make
    diag(R) real positive (both are the unique such factorisation)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nr, n)) + 1j * rng.standard_normal((nr, n))
    a[:, 1] += 0.5 * a[:, 0]  # not orthogonal, still well conditioned
    q, rr = np.linalg.qr(a)
    ph = np.diag(rr) / np.abs(np.diag(rr))
    q = q * ph[None, :]
    got = orc.orthonormalize(a.T).T
    return float(np.abs(got - q).max())


def check_cholqr_properties(orc, seed=12, n3=(4, 5, 3), n=6):
    """Q^H Q = I and span preserved: the projector Q Q^H reproduces the input block."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n,) + n3[::-1]) + 1j * rng.standard_normal((n,) + n3[::-1])
    q = orc.orthonormalize(a)
    Q = q.reshape(n, -1).T
    A = a.reshape(n, -1).T
    e1 = np.abs(Q.conj().T @ Q - np.eye(n)).max()
    e2 = np.abs(Q @ (Q.conj().T @ A) - A).max() / np.abs(A).max()
    return float(max(e1, e2))


def check_density_planewave(orc, n3=(6, 4, 5), L3=(4.0, 3.0, 3.5)):
    """|e^{iG.r}|^2 / N_r is the same at every point: the density of N planewaves is N / N_r."""
    mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (2, 1, -1), (-3, 2, 2)]
    psi = _planewave_block(n3, L3, mvecs)
    rho = orc.density(psi)
    nr = int(np.prod(n3))
    return float(np.abs(rho - len(mvecs) / nr).max() * nr)


def check_density_gauge_and_sum(orc, seed=13, n3=(5, 4, 6), n=4):
    """Unit occupations: rho is invariant under unitary mixing of the orbitals and sums to N for an
    orthonormal block; weights: each orbital counts with its occupation."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((int(np.prod(n3)), n)) + 1j * rng.standard_normal((int(np.prod(n3)), n))
    x, _ = np.linalg.qr(a)
    u, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    psi = x.T.reshape((n,) + n3[::-1])
    psiu = (x @ u).T.reshape((n,) + n3[::-1])
    r1, r2 = orc.density(psi), orc.density(psiu)
    e1 = np.abs(r1 - r2).max() / np.abs(r1).max()
    e2 = abs(r1.sum() - n) / n
    occ = np.array([2.0, 0.5, 0.0, 1.0])
    rw = orc.density(psi, occ)
    e3 = abs(rw.sum() - occ.sum()) / occ.sum()
    e4 = np.abs(rw - sum(occ[i] * np.abs(psi[i]) ** 2 for i in range(n))).max() / np.abs(rw).max()
    return float(max(e1, e2, e3, e4))


def check_kinetic_planewave(orc, n3=(6, 4, 8), L3=(4.0, 3.0, 5.5)):
    """-(1/2) Laplacian of e^{i G.r} is (|G|^2/2) e^{i G.r}; m = n/2 on an even edge is the Nyquist row,
    whose |G_a| is pi n_a / L_a whichever sign it is given."""
    mvecs = [(0, 0, 0), (1, 0, 0), (0, -1, 2), (3, 2, 4), (-2, 1, -3), (2, -2, 1)]
    psi = _planewave_block(n3, L3, mvecs)
    out = orc.apply_kinetic(psi, n3, L3)
    err = 0.0
    for k, m in enumerate(mvecs):
        g2 = sum((2 * np.pi * _wrap(m[a], n3[a]) / L3[a]) ** 2 for a in range(3))
        ref = 0.5 * g2 * psi[k]
        err = max(err, float(np.abs(out[k] - ref).max() / np.abs(psi[k]).max() / max(g2, 1.0)))
    return err


def check_kinetic_smooth(orc, n3=(40, 32, 48), L3=(6.0, 4.5, 7.5), amp=(0.4, 0.3, 0.5)):
    """f = exp(sum_a c_a cos(2 pi x_a / L_a)) is smooth and periodic; -(1/2) Laplacian f, written out
    from the chain rule, is f * sum_a -(1/2) (c_a^2 k_a^2 sin^2 - c_a k_a^2 cos) with k_a = 2 pi / L_a.
    The spectral operator reaches it to rounding once the coefficients have decayed."""
    nx, ny, nz = n3
    ax = [np.arange(n3[a]) * L3[a] / n3[a] for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    coords = (X, Y, Z)
    e = sum(amp[a] * np.cos(2 * np.pi * coords[a] / L3[a]) for a in range(3))
    f = np.exp(e)
    lap = np.zeros_like(f)
    for a in range(3):
        k = 2 * np.pi / L3[a]
        c = amp[a]
        lap += (c * c * k * k * np.sin(k * coords[a]) ** 2 - c * k * k * np.cos(k * coords[a])) * f
    ref = -0.5 * lap
    got = orc.apply_kinetic(f[None].astype(complex), n3, L3)[0]
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def check_kinetic_hermitian_psd(orc, n3=(5, 6, 4), L3=(3.0, 4.0, 2.5), seed=14):
    """<x, T y> = <T x, y> and <x, T x> >= 0 (T = -(1/2) Laplacian).  Returns the worse of the
    asymmetry and any negative part, relative to ||x|| ||T y||."""
    rng = np.random.default_rng(seed)
    nr = n3[0] * n3[1] * n3[2]
    x = (rng.standard_normal(nr) + 1j * rng.standard_normal(nr)).reshape(1, n3[2], n3[1], n3[0])
    y = (rng.standard_normal(nr) + 1j * rng.standard_normal(nr)).reshape(1, n3[2], n3[1], n3[0])
    tx = orc.apply_kinetic(x, n3, L3)
    ty = orc.apply_kinetic(y, n3, L3)
    scale = np.linalg.norm(x) * np.linalg.norm(ty)
    asym = abs(np.vdot(x, ty) - np.vdot(tx, y)) / scale
    q = np.vdot(x, tx)
    neg = max(0.0, -q.real) / scale + abs(q.imag) / scale
    return float(max(asym, neg))


# name -> (callable, bound)
ALL = {
    "naive_dft": (check_naive_dft, 1e-12),
    "brute_convolution_hse": (lambda o: check_brute_convolution(o, "hse"), 1e-12),
    "brute_convolution_coulomb": (lambda o: check_brute_convolution(o, "coulomb"), 1e-12),
    "planewave_hse": (lambda o: check_planewave(o, "hse"), 1e-12),
    "planewave_coulomb": (lambda o: check_planewave(o, "coulomb"), 1e-12),
    "planewave_ortho": (lambda o: check_planewave(o, "hse", (4, 6, 8), (3.0, 4.0, 5.5), 0.2,
                                                  [(0, 0, 0), (2, 1, -3), (-1, 3, 4), (1, -2, 2)]), 1e-12),
    "continuum": (check_continuum, 1e-10),
    "erf_potential": (check_erf_potential, 1e-6),
    "fd_poisson": (check_fd_poisson, 3e-3),
    "kernel_limits": (check_kernel_limits, 1e-4),
    "hermitian": (check_hermitian, 1e-13),
    "nsd_hse": (lambda o: check_nsd(o, "hse"), -1e-6),  # strictly negative
    "nsd_coulomb": (lambda o: check_nsd(o, "coulomb"), 1e-13),
    "gauge": (check_gauge, 1e-12),
    "pair_symmetry": (check_pair_symmetry, 1e-13),
    "linearity_scaling": (check_linearity_scaling, 1e-12),
    "translation": (check_translation, 1e-12),
    "exchange_energy": (check_exchange_energy, 1e-12),
    "ace_planewave": (check_ace_planewave, 1e-12),
    "ace_identities": (check_ace_identities, 1e-10),
    "residual_eigenbasis": (check_residual_eigenbasis, 1e-13),
    "residual_projections": (check_residual_projections, 1e-12),
    "residual_gauge": (check_residual_gauge, 1e-12),
    "cholqr_vs_householder": (check_cholqr_vs_householder, 1e-12),
    "cholqr_properties": (check_cholqr_properties, 1e-12),
    "density_planewave": (check_density_planewave, 1e-12),
    "density_gauge_and_sum": (check_density_gauge_and_sum, 1e-12),
    "kinetic_planewave": (check_kinetic_planewave, 1e-13),
    "kinetic_smooth": (check_kinetic_smooth, 1e-10),
    "kinetic_hermitian_psd": (check_kinetic_hermitian_psd, 1e-13),
}
