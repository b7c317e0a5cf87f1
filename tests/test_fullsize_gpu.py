"""Full-size parity: one GPU's share of the 512-atom cell (96^3, 1024 orbitals).

The FP64 oracle cannot redo the whole workload in test time (a full V_X
column is 1024 pair FFTs of 96^3), so the checks are: sampled output columns
recomputed by the oracle one by one, graded element-wise as well as by norm
(rel_err), properties that hold at any size (Hermiticity and sign of the
projected operator), and the FP32 forms against the GPU FP64 form on every
column.  The sampled targets 0, 5, 17 and 31 fall in four different
eighths of the 32 targets (the plane-inverse pass gives each of the eight
XCDs a contiguous eighth of a batch's targets) and at both ends of the
target range; launch configuration as in bench.py.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import host, l2_err, rel_err, say, workers

pytestmark = pytest.mark.gpu

VX_COLS = (0, 5, 17, 31)      # targets of the 32-target share checked against the oracle
ACE_COLS = (5, 700)           # K_ACE psi_k = V_X psi_k checked against the oracle
# BF16 with one residual step keeps 2 x 8 significant bits of each operand and
# drops r_A r_B: about 3 * 2^-18 = 1.1e-5 per product, so it does not reach
# 1e-5 reliably (measured 1.5e-5 element-wise at this size); held to 3e-5
TOL_BF16R = 3e-5


@pytest.fixture(scope="module")
def share():
    import torch

    w = synth.workload("96cube_1024x32")
    say("generating the 96^3 share (1024 orbitals)")
    psi = synth.make_orbitals(w["seed"], w["n"], w["L"], w["N"], dtype=np.complex64)
    P = torch.from_numpy(psi).to("cuda:0")
    return w, psi, P


_ORACLE = {}


def oracle_col(share, k):
    """V_X psi_k over all 1024 orbitals, by the FP64 oracle (cached per module)."""
    w, psi, _ = share
    if k not in _ORACLE:
        say("oracle column", k)
        _ORACLE[k] = oracle.apply_vx(psi, psi[k:k + 1], w["n"], w["L"], "hse", 0.106, workers=workers())
    return _ORACLE[k]


@pytest.mark.timeout(900)
def test_vx_share_fullsize(share):
    import torch
    from paper_1905_01348_amd import Context

    w, psi, P = share
    n, L, Nt = w["n"], w["L"], w["n_targets"]
    ctx = Context(0)
    out = ctx.apply_vx(P, P[:Nt], n=n, L=L, kernel="hse", omega=0.106, prec="fp32acc64")
    torch.cuda.synchronize()
    o = host(out)
    # FP64 form on every column
    P64 = P.to(torch.complex128)
    out64 = ctx.apply_vx(P64, P64[:Nt], n=n, L=L, kernel="hse", omega=0.106, prec="fp64")
    torch.cuda.synchronize()
    o64 = host(out64)
    del P64, out64
    ctx.close()
    for k in VX_COLS:
        ref = oracle_col(share, k)
        err = rel_err(o[k:k + 1], ref)
        err64 = rel_err(o64[k:k + 1], ref)
        say("column", k, "fp32acc64 err", err, "(l2", l2_err(o[k:k + 1], ref), ") fp64 err", err64)
        assert err <= 1e-5, k
        assert err64 <= 1e-10, k
    # projected operator on the 32 targets: Hermitian, negative diagonal
    T = psi[:Nt].reshape(Nt, -1).astype(np.complex128)
    Mb = T.conj() @ o.reshape(Nt, -1).T
    assert np.abs(Mb - Mb.conj().T).max() <= 1e-6 * np.abs(Mb).max()
    assert np.all(np.diag(Mb).real < 0)
    e64 = rel_err(o, o64)
    say("fp32acc64 vs fp64 (all columns)", e64)
    assert e64 <= 1e-5


@pytest.mark.timeout(1200)
def test_ace_fullsize(share):
    """ACE at N = R = 1024 on 96^3: K_ACE psi_k = V_X psi_k (oracle columns), precision forms vs FP64."""
    import torch
    from paper_1905_01348_amd import Context

    w, psi, P = share
    n, L, N = w["n"], w["L"], w["N"]
    ctx = Context(0)
    say("building ACE (1024^2 pairs)")
    ace = ctx.build_ace(P, n=n, L=L, kernel="hse", omega=0.106, vx_prec="fp32acc64", ace_prec="ace_fp64")
    ks = list(ACE_COLS)
    ys = {}
    for prec in ("ace_fp64", "ace_fp32r", "ace_bf16r", "ace_fp16r"):
        ys[prec] = host(ace.apply(P[ks], prec=prec, out_dtype=torch.complex128))
    torch.cuda.synchronize()
    for i, k in enumerate(ks):
        ref = oracle_col(share, k)
        for prec in ("ace_fp64", "ace_fp32r", "ace_bf16r", "ace_fp16r"):
            err = rel_err(ys[prec][i:i + 1], ref)
            say("K_ACE psi_k vs oracle V_X psi_k", k, prec, err)
            # the W columns come from the FP32-FFT pair path (fp32acc64), so the forms are held to 1e-5,
            # except BF16 with one residual step (its floor: see TOL_BF16R)
            assert err <= (TOL_BF16R if prec == "ace_bf16r" else 1e-5), (k, prec)
    say("right-hand sides (seed 3)")
    phi = torch.from_numpy(synth.make_orbitals(3, n, L, N, dtype=np.complex64)).to("cuda:0")
    y64 = ace.apply(phi, prec="ace_fp64", out_dtype=torch.complex128)
    r64 = host(y64)
    del y64
    for prec in ("ace_fp32r", "ace_bf16r", "ace_fp16r"):
        y = ace.apply(phi, prec=prec, out_dtype=torch.complex64)
        torch.cuda.synchronize()
        err = rel_err(host(y), r64)
        say(prec, "vs fp64 on 1024 columns", err)
        assert err <= (TOL_BF16R if prec == "ace_bf16r" else 1e-5), prec
        del y
    # K_ACE Hermitian on a sample of the right-hand sides
    S = phi[:16].reshape(16, -1).to(torch.complex128)
    KS = torch.from_numpy(r64[:16].reshape(16, -1)).to("cuda:0")
    G = (S.conj() @ KS.T).cpu().numpy()
    assert np.abs(G - G.conj().T).max() <= 1e-8 * np.abs(G).max()
    assert np.all(np.diag(G).real <= 0)
    ace.free()
    ctx.close()
