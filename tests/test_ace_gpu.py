"""ACE build and apply on the GPU through the C ABI against the FP64 oracle.

Tolerances (relative, per column, element-wise and L2): FP64 forms 1e-10
(including K_ACE psi_i = W_i); FP32 + residual step 1e-5 (the stated bar for
the FP32 forms); BF16 + residual step 3e-5 (two 8-bit pieces per operand and
the dropped r_A r_B leave about 3 * 2^-18 per product; it must beat the
unrefined BF16 form by a wide margin); unrefined FP32 1e-5; unrefined BF16
2e-2.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_err, dev, host, say

pytestmark = pytest.mark.gpu

TOL = {"ace_fp64": 1e-10, "ace_fp32r": 1e-5, "ace_bf16r": 3e-5, "ace_fp16r": 1e-5, "ace_fp32": 1e-5,
       "ace_bf16": 2e-2, "ace_fp16": 3e-3}


@pytest.fixture(scope="module")
def ctx():
    from paper_1905_01348_amd import Context

    c = Context(0)
    yield c
    c.close()


def _case(n3, L3, N, kind, seed, R):
    psi = synth.make_orbitals(seed, n3, L3, N, ecut=1e4)
    w = oracle.apply_vx(psi, psi, n3, L3, kind, 0.4)
    ace = oracle.build_ace(psi, w)
    phi = synth.random_grid_vectors(seed + 100, n3, R)
    y = oracle.apply_ace(ace["xi"], phi)
    return psi, w, ace, phi, y


CASES = [
    ((6, 4, 3), (4.0, 3.0, 3.5), 5, "hse", 3),
    ((8, 8, 8), (5.0, 5.0, 5.0), 37, "coulomb", 65),
    ((12, 9, 8), (6.0, 4.5, 4.0), 70, "hse", 1),
    ((16, 16, 16), (7.0, 7.0, 7.0), 130, "hse", 131),
    # a workload edge: W = V_X Psi runs the halved pair path
    ((24, 24, 24), (10.26, 10.26, 10.26), 40, "hse", 9),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-N{c[2]}-{c[3]}-R{c[4]}" for c in CASES])
def test_ace_build_and_apply_all_precisions(ctx, case):
    import torch

    n3, L3, N, kind, R = case
    say("ace case", case)
    psi, w, ace_ref, phi, y_ref = _case(n3, L3, N, kind, 21, R)
    P = dev(psi)
    ace = ctx.build_ace(P, n=n3, L=L3, kernel=kind, omega=0.4, vx_prec="fp64", ace_prec="ace_fp64")
    xi, L, M = ace.export()
    torch.cuda.synchronize()
    nr = int(np.prod(n3))
    assert np.abs(host(M) - ace_ref["M"]).max() <= 1e-10 * np.abs(ace_ref["M"]).max()
    assert np.abs(host(L) - ace_ref["L"]).max() <= 1e-10 * np.abs(ace_ref["L"]).max()
    assert rel_err(host(xi), ace_ref["xi"]) <= 1e-10
    assert abs(ace.ex - ace_ref["ex"]) <= 1e-12 * abs(ace_ref["ex"])
    F = dev(phi)
    errs = {}
    for prec in ("ace_fp64", "ace_fp32r", "ace_bf16r", "ace_fp16r", "ace_fp32", "ace_bf16", "ace_fp16"):
        y = ace.apply(F, prec=prec, out_dtype=torch.complex128)
        torch.cuda.synchronize()
        errs[prec] = rel_err(host(y), y_ref)
        # K_ACE psi_i = W_i
        yw = ace.apply(P, prec=prec, out_dtype=torch.complex128)
        torch.cuda.synchronize()
        ew = rel_err(host(yw), w.reshape(N, nr))
        say("  ", prec, "K_ACE phi err", errs[prec], "K_ACE psi = W err", ew)
        assert errs[prec] <= TOL[prec], (prec, errs[prec])
        assert ew <= TOL[prec], (prec, ew)
    # the residual step must help where the rounding error dominates
    assert errs["ace_bf16r"] < 0.05 * errs["ace_bf16"]
    assert errs["ace_fp16r"] < 0.05 * errs["ace_fp16"]
    ace.free()


def test_ace_complex64_io(ctx):
    import torch

    n3, L3, N, R = (8, 6, 9), (4.0, 3.0, 4.5), 11, 7
    psi, w, ace_ref, phi, y_ref = _case(n3, L3, N, "hse", 5, R)
    ace = ctx.build_ace(dev(psi, torch.complex64), n=n3, L=L3, kernel="hse", omega=0.4, vx_prec="fp32acc64",
                        ace_prec="ace_fp32r")
    # the oracle consumes the complex64-rounded orbitals it was given
    psi32 = psi.astype(np.complex64).astype(np.complex128)
    w32 = oracle.apply_vx(psi32, psi32, n3, L3, "hse", 0.4)
    ref32 = oracle.build_ace(psi32, w32)
    phi32 = phi.astype(np.complex64)
    y32 = oracle.apply_ace(ref32["xi"], phi32.astype(np.complex128))
    for prec in ("ace_fp32r", "ace_bf16r", "ace_fp16r", "ace_fp64"):
        y = ace.apply(dev(phi32), prec=prec, out_dtype=torch.complex64)
        torch.cuda.synchronize()
        assert y.dtype == torch.complex64
        err = rel_err(host(y), y32)
        say("c64 io", prec, err)
        assert err <= max(TOL[prec], 1e-5)
    ace.free()


def test_fp16_scaling_per_right_hand_side(ctx):
    """FP16 operands are scaled by powers of two per right-hand side (and per column of xi^H phi):
    right-hand sides 12 orders of magnitude apart still each meet 1e-5 against the FP64 form."""
    import torch

    n3, L3, N = (12, 12, 12), (6.0, 6.0, 6.0), 24
    psi = synth.make_orbitals(8, n3, L3, N, ecut=1e4)
    ace = ctx.build_ace(dev(psi), n=n3, L=L3, kernel="hse", omega=0.4, vx_prec="fp64", ace_prec="ace_fp16r")
    phi = synth.random_grid_vectors(9, n3, 4)
    phi *= np.array([1e-8, 1e4, 1.0, 1e-3])[:, None, None, None]
    F = dev(phi)
    y64 = host(ace.apply(F, prec="ace_fp64", out_dtype=torch.complex128))
    for prec in ("ace_fp16r", "ace_bf16r", "ace_fp32r"):
        y = host(ace.apply(F, prec=prec, out_dtype=torch.complex128))
        err = rel_err(y, y64)
        say("scaled right-hand sides", prec, err)
        assert err <= TOL[prec], prec
    ace.free()


def test_not_positive_definite(ctx):
    from paper_1905_01348_amd import FockError

    n3 = (4, 4, 4)
    psi = np.full((1, 4, 4, 4), 1.0 / 8.0, dtype=complex)
    with pytest.raises(FockError) as ei:
        ctx.build_ace(dev(psi), n=n3, L=3.0, kernel="coulomb", vx_prec="fp64")
    assert ei.value.status == -4


def test_ace_errors(ctx):
    import torch
    from paper_1905_01348_amd import FockError

    n3, L3 = (6, 6, 6), (4.0, 4.0, 4.0)
    psi = synth.make_orbitals(2, n3, L3, 4, ecut=1e4)
    P = dev(psi)
    ace = ctx.build_ace(P, n=n3, L=L3, kernel="hse", vx_prec="fp64")
    with pytest.raises(FockError) as ei:
        ace.apply(P, prec="fp64")  # not an ACE precision
    assert ei.value.status == -2
    with pytest.raises(FockError) as ei:
        ace.apply(P, prec="ace_fp64", out=P)  # aliasing
    assert ei.value.status == -1
    with pytest.raises(FockError) as ei:
        ctx.build_ace(P, n=n3, L=L3, vx_prec="ace_fp64")
    assert ei.value.status == -2
    ace.free()
    torch.cuda.synchronize()


def test_handles_outlive_their_context():
    """An ACE handle and a server (with a registered trajectory) still alive when
    their context is finalized: the context takes their device memory back, a
    later free only deletes the handle, and any other use is refused."""
    import torch
    from paper_1905_01348_amd import Context, FockError, Server

    c = Context(0)
    n3, L3 = (6, 6, 6), (4.0, 4.0, 4.0)
    P = dev(synth.make_orbitals(3, n3, L3, 4, ecut=1e4))
    ace = c.build_ace(P, n=n3, L=L3, kernel="hse", vx_prec="fp64")
    srv = Server(c, max_slots=2, n_streams=1)
    srv.register(0, P.to(torch.complex64), n=n3, L=L3)
    c.close()
    with pytest.raises(FockError) as ei:
        ace.export()
    assert ei.value.status == -1
    with pytest.raises(FockError) as ei:
        srv.register(1, P.to(torch.complex64), n=n3, L=L3)
    assert ei.value.status == -1
    ace.free()
    srv.close()
    torch.cuda.synchronize()
    # a fresh context on the same device works as usual
    c2 = Context(0)
    ace2 = c2.build_ace(P, n=n3, L=L3, kernel="hse", vx_prec="fp64")
    y = ace2.apply(P, prec="ace_fp64")
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(y)).all()
    ace2.free()
    c2.close()
