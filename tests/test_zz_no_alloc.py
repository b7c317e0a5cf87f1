"""The allocation-free V_X entry point (fx_apply_vx_noalloc) through the C ABI.

Calls in a row, each on a smaller input than the one before (96^3, then 48^3,
then 24^3), each checked against fx_apply_vx on the same inputs (1e-5 for the
FP32 forms, 1e-10 and the exchange energy for FP64), the middle one also
against the FP64 oracle; the context that makes them allocates nothing
(its byte count stays 0) and calls that do not fit the fixed scratch region,
or would need a conversion, are refused before any launch.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_1905_01348_amd import Context, FockError

    na = Context(0)    # makes only allocation-free calls
    ref_ctx = Context(0)
    assert na.memory() == (0, 0)
    cases = [
        # grid, L, orbitals, targets, prec, input dtype, out dtype, kernel
        (96, 41.04, 40, 4, "fp32acc64", np.complex64, torch.complex128, "hse"),
        (48, 20.52, 24, 8, "fp32acc64", np.complex64, torch.complex128, "hse"),
        (24, 10.26, 10, 10, "fp64", np.complex128, torch.complex128, "coulomb"),
    ]
    for n, L, N, Nt, prec, idt, odt, kern in cases:
        say("no-alloc case", n, N, Nt, prec)
        psi = synth.make_orbitals(100 + n, n, L, N, dtype=idt)
        P = dev(psi)
        phi = P if Nt == N else P[:Nt]
        energy = Nt == N
        out = torch.full((Nt, n, n, n), complex(7.0, -7.0), dtype=odt, device="cuda")
        ex = torch.full((), 3.0, dtype=torch.float64, device="cuda") if energy else None
        na.apply_vx_noalloc(P, phi, out=out, n=n, L=L, kernel=kern, omega=0.106, prec=prec, energy_out=ex)
        torch.cuda.synchronize()
        assert na.memory() == (0, 0), "the allocation-free call allocated"
        if energy:
            ref, ex_ref = ref_ctx.apply_vx(P, phi, n=n, L=L, kernel=kern, omega=0.106, prec=prec, out_dtype=odt,
                                           energy=True)
        else:
            ref = ref_ctx.apply_vx(P, phi, n=n, L=L, kernel=kern, omega=0.106, prec=prec, out_dtype=odt)
        torch.cuda.synchronize()
        tol = 1e-10 if prec == "fp64" else 1e-5
        err = rel_err(host(out), host(ref))
        say("  vs fx_apply_vx", err)
        assert err <= tol
        if energy:
            say("  E_X", ex.item(), ex_ref.item())
            assert abs(ex.item() - ex_ref.item()) <= 1e-12 * abs(ex_ref.item())
        if n == 48:
            r = oracle.apply_vx(psi, psi[:Nt], n, L, kern, 0.106)
            e_or = rel_err(host(out), r)
            say("  vs oracle", e_or)
            assert e_or <= tol
    # refused before any launch: partial sums of 32 targets at 96^3 cannot live in a complex64
    # out and do not fit the scratch region; complex128 input on an FP32 path needs a conversion
    psi = dev(synth.random_grid_vectors(5, (96, 96, 96), 33, dtype=np.complex64))
    o32 = torch.zeros((32, 96, 96, 96), dtype=torch.complex64, device="cuda")
    with pytest.raises(FockError) as ei:
        na.apply_vx_noalloc(psi, psi[:32], out=o32, n=96, L=41.04, prec="fp32acc64")
    assert ei.value.status == -1
    assert torch.count_nonzero(o32).item() == 0
    p128 = dev(synth.random_grid_vectors(6, (12, 12, 12), 3))
    o128 = torch.zeros((3, 12, 12, 12), dtype=torch.complex128, device="cuda")
    with pytest.raises(FockError) as ei:
        na.apply_vx_noalloc(p128, out=o128, n=12, L=6.0, prec="fp32acc64")
    assert ei.value.status == -2
    assert na.memory() == (0, 0)
    na.close()
    ref_ctx.close()
