"""Argument checks of the Python binding that stop before any launch: an output
with too few columns or the wrong dtype would be written past its end by the
library, which writes n columns of the stated dtype at the stated stride."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def test_outputs_are_checked_before_launch():
    import torch
    from paper_1905_01348_amd import Context, Server

    ctx = Context(0)
    n3, L3 = (8, 8, 8), (5.0, 5.0, 5.0)
    psi = synth.make_orbitals(3, n3, L3, 6, ecut=1e4)
    P = dev(psi)
    ace = ctx.build_ace(P, n=n3, L=L3, kernel="hse", vx_prec="fp64")
    short = torch.zeros((5, 8, 8, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        ace.apply(P, prec="ace_fp64", out=short)
    with pytest.raises(ValueError):
        ctx.pt_residual(P, P.clone(), n=n3, L=L3, dt=0.1, out=short)
    with pytest.raises(ValueError):
        ctx.pt_residual(P, P.clone(), n=n3, L=L3, dt=0.1,
                        out=torch.zeros((6, 8, 8, 8), dtype=torch.complex64, device="cuda"))
    assert torch.count_nonzero(short).item() == 0
    srv = Server(ctx, max_slots=2, n_streams=1)
    srv.register(0, P.to(torch.complex64), n=n3, L=L3)
    few = torch.zeros((3, 8, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        srv.serve([dict(traj=0, op=0, first=0, count=4, t=0.0, out=few)])
    wrong = torch.zeros((4, 8, 8, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        srv.serve([dict(traj=0, op=1, first=0, count=4, t=0.0, out=wrong)])
    ok = torch.zeros((4, 8, 8, 8), dtype=torch.complex64, device="cuda")
    st, _, _ = srv.serve([dict(traj=0, op=0, first=0, count=4, t=0.0, out=ok)])
    torch.cuda.synchronize()
    assert st == [0] and torch.count_nonzero(few).item() == 0 and torch.count_nonzero(wrong).item() == 0
    srv.close()
    ace.free()
    ctx.close()
