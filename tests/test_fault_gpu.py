"""Device allocation failures forced from the host, one allocation at a time.

fx_debug_fail_alloc(k) makes the k-th device allocation of the library after
the call fail once with FX_ERR_OOM.  For each operation below, on a fresh
context, every k from 1 up to the number of allocations the operation makes is
tried in turn: the call must either fail with FX_ERR_OOM (and nothing else) or
succeed, and the same call on the same context afterwards must succeed and
match the FP64 oracle to its usual tolerance.  The serving loop must absorb a
failed workspace allocation (it hands back idle workspaces and retries).
"""
import numpy as np
import pytest

import oracle
import synth
from paper_1905_01348_amd import fock as F
from tests.gpu_util import rel_err, dev, host, say

pytestmark = pytest.mark.gpu

N24, L24 = (24, 24, 24), (10.26,) * 3
G3, L3 = (18, 16, 12), (7.0, 8.0, 6.0)


def _cases():
    import torch

    psi_g = synth.make_orbitals(300, G3, L3, 4, ecut=1e4)
    phi_g = synth.random_grid_vectors(301, G3, 3)
    psi24 = synth.make_orbitals(302, N24, L24, 6)
    half = synth.random_grid_vectors(303, (12, 12, 12), 5)
    psi12 = synth.make_orbitals(304, (12, 12, 12), (6.0,) * 3, 5, ecut=1e4)
    blk = synth.random_grid_vectors(305, (12, 12, 12), 5)
    blk[1] += 0.5 * blk[0]
    ace_phi = synth.random_grid_vectors(306, N24, 3)
    w24 = oracle.apply_vx(psi24, psi24, N24, L24, "hse", 0.106)
    xi = oracle.build_ace(psi24, w24)["xi"]

    def vx_generic(ctx):
        return host(ctx.apply_vx(dev(psi_g), dev(phi_g), n=G3, L=L3, prec="fp64"))

    def vx_square(ctx):
        return host(ctx.apply_vx(dev(psi24), n=N24, L=L24, prec="fp32acc64"))

    def kinetic(ctx):
        return host(ctx.apply_kinetic(dev(phi_g), n=G3, L=L3))

    def ace(ctx):
        a = ctx.build_ace(dev(psi24), n=N24, L=L24, vx_prec="fp64")
        try:
            return host(a.apply(dev(ace_phi), prec="ace_fp32r"))
        finally:
            a.free()

    def residual(ctx):
        return host(ctx.pt_residual(dev(psi12), dev(half), n=(12, 12, 12), L=(6.0,) * 3, dt=0.3, vx_prec="fp64",
                                    kinetic=True))

    def orthonormalize(ctx):
        t = dev(blk)
        ctx.orthonormalize(t)
        torch.cuda.synchronize()
        return host(t)

    t12 = oracle.apply_vx(psi12, psi12, (12, 12, 12), (6.0,) * 3, "hse", 0.106) + \
        oracle.apply_kinetic(psi12, (12, 12, 12), (6.0,) * 3)
    return {
        "apply_vx_generic": (vx_generic, oracle.apply_vx(psi_g, phi_g, G3, L3, "hse", 0.106), 1e-10),
        "apply_vx_square_24": (vx_square, w24, 1e-5),
        "apply_kinetic": (kinetic, oracle.apply_kinetic(phi_g, G3, L3), 1e-10),
        "build_and_apply_ace": (ace, oracle.apply_ace(xi, ace_phi), 1e-5),
        "pt_residual_kinetic": (residual, oracle.pt_residual(psi12, t12, half, 0.3), 1e-10),
        "orthonormalize": (orthonormalize, oracle.orthonormalize(blk), 1e-11),
    }


CASES = None


@pytest.mark.parametrize("name", ["apply_vx_generic", "apply_vx_square_24", "apply_kinetic", "build_and_apply_ace",
                                  "pt_residual_kinetic", "orthonormalize"])
def test_each_allocation_failure_leaves_a_usable_context(name):
    from paper_1905_01348_amd import Context

    global CASES
    if CASES is None:
        CASES = _cases()
    op, ref, tol = CASES[name]
    failed = 0
    for k in range(1, 200):
        ctx = Context(0)
        try:
            F.debug_fail_alloc(k)
            try:
                op(ctx)
                ok = True
            except F.FockError as e:
                assert e.status == F.FX_ERR_OOM, (name, k, e.status, str(e))
                ok = False
                failed += 1
            F.debug_fail_alloc(0)
            err = rel_err(op(ctx), ref)
            assert err <= tol, (name, k, err)
        finally:
            F.debug_fail_alloc(0)
            ctx.close()
        if ok:
            break
    else:
        pytest.fail(f"{name}: more than 199 allocations")
    say(name, "allocations that failed in turn:", failed)
    assert failed >= 1


def test_serving_absorbs_a_failed_workspace_allocation():
    import torch

    from paper_1905_01348_amd import Context, Server

    psi = synth.make_orbitals(310, N24, L24, 8).astype(np.complex64)
    ref = oracle.apply_vx(psi.astype(np.complex128), psi[:4].astype(np.complex128), N24, L24, "hse", 0.106)
    ctx = Context(0)
    try:
        srv = Server(ctx, max_slots=2, n_streams=2, max_batch_pairs=4096)
        srv.register(0, dev(psi), n=N24, L=L24, vx_prec="fp32acc64", ace_prec="ace_fp32r")
        for k in (1, 2, 3):
            outs = [torch.zeros((4,) + N24, dtype=torch.complex64, device="cuda") for _ in range(2)]
            reqs = [dict(traj=0, op=0, first=0, count=4, t=0.0, out=outs[0]),
                    dict(traj=0, op=1, first=0, count=4, t=0.0, out=outs[1])]
            F.debug_fail_alloc(k)
            st, _, rep = srv.serve(reqs)
            F.debug_fail_alloc(0)
            torch.cuda.synchronize()
            assert st == [0, 0], (k, st)
            for o in outs:
                assert rel_err(host(o).astype(np.complex128), ref) <= 1e-5, k
        srv.close()
    finally:
        F.debug_fail_alloc(0)
        ctx.close()
