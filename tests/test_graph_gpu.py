"""HIP graph capture of fx_apply_vx, fx_apply_kinetic and fx_apply_ace.

After one uncaptured call of the same shape (workspace and grid tables in
place), the call is captured into a graph on a side stream; every replay
must reproduce the eager result bitwise, with eager calls and host waits of
the program's own in between.  A captured call that would have to allocate
fails with FX_ERR_INVALID instead of allocating.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _bits(a):
    return a.view(np.float64 if a.dtype == np.complex128 else np.float32)


@pytest.fixture(scope="module")
def ctx():
    from paper_1905_01348_amd import Context

    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32acc64", "fp32"])
def test_apply_vx_graph_replays_match_eager(ctx, prec):
    import torch

    n, L, N = 24, 10.26, 16
    psi = dev(synth.make_orbitals(0, n, L, N))
    phi = psi[:5].clone()
    s = torch.cuda.Stream()
    out_e = torch.empty_like(phi)
    out_g = torch.empty_like(phi)
    with torch.cuda.stream(s):
        ctx.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out_e)
    torch.cuda.synchronize()
    ref = host(out_e)
    g = torch.cuda.CUDAGraph()
    say("capture apply_vx", prec)
    with torch.cuda.graph(g, stream=s):
        ctx.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out_g)
    torch.cuda.synchronize()
    for rep in range(3):
        out_g.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = host(out_g)
        say("  replay", rep)
        assert np.array_equal(_bits(got), _bits(ref)), f"replay {rep}"
        # eager work of the same shape between replays
        ctx.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out_e)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(out_e)), _bits(ref))
    del g


def test_apply_kinetic_graph_replays_match_eager(ctx):
    """The kinetic operator (the pair path with the constant orbital, filled by a kernel on every
    call) captured once and replayed: each replay equals the eager result bitwise."""
    import torch

    n3, L3 = (24, 18, 16), (10.0, 8.0, 7.0)
    phi = dev(synth.random_grid_vectors(5, n3, 4))
    s = torch.cuda.Stream()
    out_e = torch.empty_like(phi)
    out_g = torch.empty_like(phi)
    with torch.cuda.stream(s):
        ctx.apply_kinetic(phi, n=n3, L=L3, out=out_e)
    torch.cuda.synchronize()
    ref = host(out_e)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.apply_kinetic(phi, n=n3, L=L3, out=out_g)
    torch.cuda.synchronize()
    for rep in range(3):
        out_g.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(out_g)), _bits(ref)), f"replay {rep}"
        ctx.apply_kinetic(phi, n=n3, L=L3, out=out_e)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(out_e)), _bits(ref))
    del g


def test_capture_refuses_to_allocate(ctx):
    """A shape never run before needs a larger workspace: the captured call fails cleanly."""
    import torch
    from paper_1905_01348_amd import FockError

    # an orthorhombic grid not used anywhere else on this context
    psi = dev(synth.make_orbitals(3, (18, 16, 12), (8.0, 7.5, 6.0), 40))
    s = torch.cuda.Stream()
    out = torch.empty_like(psi)
    g = torch.cuda.CUDAGraph()
    with pytest.raises(FockError) as ei:
        with torch.cuda.graph(g, stream=s):
            ctx.apply_vx(psi, n=(18, 16, 12), L=(8.0, 7.5, 6.0), prec="fp64", out=out)
    assert ei.value.status == -1
    del g
    torch.cuda.synchronize()
    # the context still works uncaptured afterwards
    ctx.apply_vx(psi, n=(18, 16, 12), L=(8.0, 7.5, 6.0), prec="fp64", out=out)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(out)).all()


@pytest.mark.parametrize("prec", ["ace_fp64", "ace_fp32r", "ace_bf16r"])
def test_apply_ace_graph_replays_match_eager(ctx, prec):
    import torch

    n, L, N, R = 12, 6.0, 10, 7
    psi = dev(synth.make_orbitals(5, n, L, N))
    ace = ctx.build_ace(psi, n=n, L=L, kernel="hse", omega=0.3)
    phi = dev(synth.random_grid_vectors(6, n, R))
    s = torch.cuda.Stream()
    out_e = torch.empty_like(phi)
    out_g = torch.empty_like(phi)
    with torch.cuda.stream(s):
        ace.apply(phi, prec=prec, out=out_e)
    torch.cuda.synchronize()
    ref = host(out_e)
    g = torch.cuda.CUDAGraph()
    say("capture apply_ace", prec)
    with torch.cuda.graph(g, stream=s):
        ace.apply(phi, prec=prec, out=out_g)
    torch.cuda.synchronize()
    for rep in range(3):
        out_g.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(out_g)), _bits(ref)), f"replay {rep}"
        ace.apply(phi, prec=prec, out=out_e)
        torch.cuda.synchronize()
    del g
    ace.free()


@pytest.mark.parametrize("prec", ["fp32acc64", "fp64"])
def test_library_replay_cache(prec):
    """fx_graph_cache: the first call of a set of arguments runs eagerly and is captured; later
    calls with the same arguments replay the graph. Every replay equals the eager result bitwise
    (with eager work and host waits of the program's own in between); new values in the same input
    buffer give the new result; another output buffer or a new launch configuration is a miss."""
    import torch
    from paper_1905_01348_amd import Context

    n, L, N = 24, 10.26, 16
    p_np = synth.make_orbitals(0, n, L, N, dtype=np.complex64 if prec == "fp32acc64" else np.complex128)
    ref_ctx = Context(0)
    psi = dev(p_np)
    phi = psi[:5].clone()
    ref = host(ref_ctx.apply_vx(psi, phi, n=n, L=L, prec=prec))
    c = Context(0)
    c.graph_cache(8)
    out = torch.full((5, n, n, n), complex(3.0, 3.0), dtype=torch.complex128, device="cuda")
    for rep in range(4):
        out.fill_(complex(3.0, 3.0))
        c.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(out)), _bits(ref)), f"call {rep}"
        ref_ctx.apply_vx(psi, phi, n=n, L=L, prec=prec)  # other work between replays
        torch.cuda.synchronize()
    hits, misses, entries = c.graph_cache_stats()
    say("replay cache", prec, hits, misses, entries)
    assert (hits, misses, entries) == (3, 1, 1)
    # new values in the same buffers: the replay reads them
    phi.copy_(psi[5:10])
    c.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out)
    torch.cuda.synchronize()
    ref2 = host(ref_ctx.apply_vx(psi, psi[5:10].clone(), n=n, L=L, prec=prec))
    assert np.array_equal(_bits(host(out)), _bits(ref2))
    assert c.graph_cache_stats()[:2] == (4, 1)
    # another output buffer: a new entry
    out2 = torch.empty_like(out)
    c.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out2)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(host(out2)), _bits(ref2))
    assert c.graph_cache_stats() == (4, 2, 2)
    # a changed launch configuration makes the stored graphs stale
    cfg, _ = c.get_vx_config(n=n, prec=prec, phi_is_psi=False)
    cfg["work_mb"] = 64
    c.set_vx_config(cfg, n=n, prec=prec, phi_is_psi=False)
    c.apply_vx(psi, phi, n=n, L=L, prec=prec, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(host(out)), _bits(ref2))
    assert c.graph_cache_stats()[:2] == (4, 3)
    # ACE through the cache
    ace = c.build_ace(psi, n=n, L=L, kernel="hse", omega=0.106)
    y_e = host(ace.apply(phi, prec="ace_fp32r"))
    y = torch.empty_like(phi)
    for rep in range(3):
        ace.apply(phi, prec="ace_fp32r", out=y)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(host(y)), _bits(y_e)), f"ace call {rep}"
    c.graph_cache(0)
    assert c.graph_cache_stats() == (0, 0, 0)
    ace.free()
    c.close()
    ref_ctx.close()
