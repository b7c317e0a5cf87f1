"""Serving loop on the GPU: continuous batching over resident trajectories.

Checks: every request completes; each result is bitwise the same alone and in
the mix; sampled results match the FP64 oracle (1e-5, the FP32 forms' bar);
admission under a small HBM budget queues or refuses instead of failing.
"""
import numpy as np
import pytest

import oracle
import synth
from synth.requests import poisson_requests
from tests.gpu_util import dev, host, rel_err, say, workers

pytestmark = pytest.mark.gpu

TRAJ = {  # traj id -> (grid, L, N, seed)
    0: ((12, 12, 12), 6.0, 8, 40),
    1: ((12, 12, 12), 6.0, 8, 41),
    2: ((16, 16, 16), 8.0, 16, 42),
    3: ((24, 24, 24), 10.26, 16, 43),
}


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1905_01348_amd import Context, Server

    ctx = Context(0)
    srv = Server(ctx, max_slots=6, n_streams=3, max_batch_pairs=4096)
    psis = {}
    for t, (n3, L, N, seed) in TRAJ.items():
        psi = synth.make_orbitals(seed, n3, L, N, dtype=np.complex64)
        psis[t] = psi
        srv.register(t, dev(psi), n=n3, L=L, kernel="hse", omega=0.106, vx_prec="fp32acc64", ace_prec="ace_fp32r")
    torch.cuda.synchronize()
    yield ctx, srv, psis
    srv.close()
    ctx.close()


def _reqs(seed, n, rate):
    by_class = {0: [(0, 8), (1, 8)], 1: [(2, 16)], 2: [(3, 16)]}
    return poisson_requests(seed, n, rate, by_class, {0: 0.5, 1: 0.35, 2: 0.15}, block=4)


def _outs(reqs):
    import torch

    outs = []
    for r in reqs:
        n3 = TRAJ[r["traj"]][0]
        outs.append(torch.full((r["count"],) + tuple(n3[::-1]), complex(9.0, 9.0), dtype=torch.complex64,
                               device="cuda"))
    return outs


def test_mix_equals_alone_and_oracle(setup):
    import torch

    ctx, srv, psis = setup
    reqs = _reqs(7, 48, 5000.0)  # arrivals far faster than service: batches and overlap
    outs = _outs(reqs)
    for r, o in zip(reqs, outs):
        r["out"] = o
    st, lat, rep = srv.serve(reqs)
    torch.cuda.synchronize()
    say("mix report", rep)
    assert all(s == 0 for s in st), st
    assert rep["n_done"] == len(reqs) and rep["n_rejected"] == 0
    assert 0 <= rep["p50_ms"] <= rep["p99_ms"] <= rep["max_ms"]
    assert rep["n_batches"] < len(reqs), "same-trajectory requests should have been merged"
    assert all(v >= 0 for v in lat)
    mix = [host(o) for o in outs]
    # each request alone
    for i, r in enumerate(reqs):
        alone = dict(r, t=0.0, out=_outs([r])[0])
        st1, _, _ = srv.serve([alone])
        assert st1 == [0]
        a = host(alone["out"])
        assert np.array_equal(a.view(np.float32), mix[i].view(np.float32)), f"request {i} differs alone vs mix"
    # oracle on a sample: V_X and K_ACE of the block (K_ACE = V_X on span(Psi))
    checked = set()
    for i, r in enumerate(reqs):
        key = (r["traj"], r["first"])
        if key in checked or len(checked) >= 4:
            continue
        checked.add(key)
        n3, L, N, _ = TRAJ[r["traj"]]
        psi = psis[r["traj"]].astype(np.complex128)
        ref = oracle.apply_vx(psi, psi[r["first"]:r["first"] + r["count"]], n3, L, "hse", 0.106)
        err = rel_err(mix[i], ref)
        say("req", i, "op", r["op"], "err", err)
        assert err <= 1e-5


def test_admission_under_small_budget(setup):
    import torch
    from paper_1905_01348_amd import Server

    ctx, srv, psis = setup
    used, _ = ctx.memory()
    # a budget just above what is resident: no batch workspace fits -> refused, not failed
    tiny = Server(ctx, max_slots=2, n_streams=1, max_batch_pairs=4096, hbm_budget_bytes=used + (1 << 20))
    psi = psis[0]
    with pytest.raises(Exception):
        # registering needs memory for psi and the ACE factors beyond the budget
        tiny.register(0, dev(psi), n=(12, 12, 12), L=6.0)
    tiny.close()
    reqs = _reqs(9, 12, 2000.0)
    outs = _outs(reqs)
    for r, o in zip(reqs, outs):
        r["out"] = o
    # the big server with only one slot: everything queues and completes
    one = Server(ctx, max_slots=1, n_streams=1, max_batch_pairs=64)
    for t, (n3, L, N, seed) in TRAJ.items():
        one.register(t, dev(psis[t]), n=n3, L=L, kernel="hse", omega=0.106)
    st, lat, rep = one.serve(reqs)
    torch.cuda.synchronize()
    assert all(s == 0 for s in st)
    assert rep["n_batches"] >= 1
    one.close()


def test_invalid_requests_reported(setup):
    import torch

    ctx, srv, psis = setup
    o = torch.zeros((4, 12, 12, 12), dtype=torch.complex64, device="cuda")
    reqs = [dict(traj=99, op=0, first=0, count=4, t=0.0, out=o),
            dict(traj=0, op=0, first=6, count=4, t=0.0, out=o),
            dict(traj=0, op=5, first=0, count=4, t=0.0, out=o),
            dict(traj=0, op=1, first=0, count=4, t=0.0, out=o)]
    st, lat, rep = srv.serve(reqs)
    assert st[:3] == [-1, -1, -1] and st[3] == 0


def test_autotuned_registration(setup):
    """With autotune on, registration stores tuned configurations for the trajectory's grid
    (request form and ACE-build form), and served results still match the oracle."""
    import torch
    from paper_1905_01348_amd import Context, Server

    _, _, psis = setup
    ctx = Context(0)
    srv = Server(ctx, max_slots=4, n_streams=2, max_batch_pairs=4096, autotune=True, autotune_targets=4)
    for t in (2, 3):
        n3, L, N, seed = TRAJ[t]
        srv.register(t, dev(psis[t]), n=n3, L=L, kernel="hse", omega=0.106, vx_prec="fp32acc64", ace_prec="ace_fp32r")
        for square in (False, True):
            cfg, is_set = ctx.get_vx_config(n=n3, prec="fp32acc64", phi_is_psi=square)
            say("traj", t, "square" if square else "requests", cfg)
            assert is_set and cfg["kernels"] in (1, 2)
    reqs = [dict(traj=t, op=op, first=4, count=4, t=0.001 * i) for i, (t, op) in
            enumerate([(2, 0), (3, 0), (2, 1), (3, 1)])]
    outs = _outs(reqs)
    for r, o in zip(reqs, outs):
        r["out"] = o
    st, lat, rep = srv.serve(reqs)
    torch.cuda.synchronize()
    assert all(s == 0 for s in st)
    for r, o in zip(reqs, outs):
        n3, L, N, seed = TRAJ[r["traj"]]
        psi = psis[r["traj"]].astype(np.complex128)
        phi = psi[r["first"]:r["first"] + r["count"]]
        if r["op"] == 0:
            ref = oracle.apply_vx(psi, phi, n3, L, "hse", 0.106)
        else:
            w = oracle.apply_vx(psi, psi, n3, L, "hse", 0.106)
            ref = oracle.apply_ace(oracle.build_ace(psi, w)["xi"], phi)
        assert rel_err(host(o), ref) <= 1e-5, r
    srv.close()
    ctx.close()


@pytest.mark.timeout(600)
def test_workload_classes_oracle_sample():
    """The serving workload's three cell classes (24^3 / N = 16, 48^3 / N = 128, 72^3 / N = 432,
    complex64, screened kernel) in one mix: every request completes; for each class one V_X and one
    ACE request are checked against the FP64 oracle (V_X on the block's first and last target;
    K_ACE psi_i = V_X psi_i for psi_i of the block, since K_ACE equals V_X on span(Psi)) and
    bitwise against the same request served alone."""
    import torch
    from paper_1905_01348_amd import Context, Server

    classes = {10: ((24, 24, 24), 10.26, 16, 4010), 11: ((48, 48, 48), 20.52, 128, 4110),
               12: ((72, 72, 72), 30.78, 432, 4210)}
    ctx = Context(0)
    srv = Server(ctx, max_slots=6, n_streams=3, max_batch_pairs=1 << 16)
    psis = {}
    for t, (n3, L, N, seed) in classes.items():
        say("registering class", n3[0], "N", N)
        psis[t] = synth.make_orbitals(seed, n3, L, N, dtype=np.complex64)
        srv.register(t, dev(psis[t]), n=n3, L=L, kernel="hse", omega=0.106, vx_prec="fp32acc64",
                     ace_prec="ace_fp32r")
    torch.cuda.synchronize()
    by_class = {0: [(10, 16)], 1: [(11, 128)], 2: [(12, 432)]}
    reqs = poisson_requests(44, 30, 400.0, by_class, {0: 0.5, 1: 0.35, 2: 0.15}, block=8)
    # make sure every (class, op) appears at least once
    t_last = reqs[-1]["t"]
    for i, (t, op) in enumerate([(10, 0), (10, 1), (11, 0), (11, 1), (12, 0), (12, 1)]):
        reqs.append(dict(traj=t, op=op, first=8 * (i % 2), count=8, t=t_last + 0.001 * (i + 1)))

    def outs_for(rs):
        return [torch.full((r["count"],) + tuple(classes[r["traj"]][0][::-1]), complex(9.0, 9.0),
                           dtype=torch.complex64, device="cuda") for r in rs]

    outs = outs_for(reqs)
    for r, o in zip(reqs, outs):
        r["out"] = o
    st, lat, rep = srv.serve(reqs)
    torch.cuda.synchronize()
    say("classes report", rep)
    assert all(s == 0 for s in st), st
    mix = [host(o) for o in outs]
    done = set()
    for i, r in enumerate(reqs):
        key = (r["traj"], r["op"])
        if key in done:
            continue
        done.add(key)
        n3, L, N, _ = classes[r["traj"]]
        psi = psis[r["traj"]].astype(np.complex128)
        ks = [r["first"], r["first"] + r["count"] - 1]
        ref = oracle.apply_vx(psi, psi[ks], n3, L, "hse", 0.106, workers=workers())
        err = rel_err(mix[i][[0, r["count"] - 1]], ref)
        say("class", n3[0], "op", r["op"], "oracle err", err)
        assert err <= 1e-5, (n3, r["op"], err)
        alone = dict(r, t=0.0, out=outs_for([r])[0])
        st1, _, _ = srv.serve([alone])
        assert st1 == [0]
        assert np.array_equal(host(alone["out"]).view(np.float32), mix[i].view(np.float32)), \
            f"request {i} differs alone vs mix"
    assert len(done) == 6
    srv.close()
    ctx.close()


@pytest.mark.parametrize("c_split", [None, 4])
def test_same_grid_trajectories_share_a_launch(c_split):
    """V_X requests of two trajectories on one grid (same cell, kernel, orbital count and precision)
    run as one launch, each target paired with its own trajectory's orbitals: one batch, results
    bitwise equal to each request served alone and within 1e-5 of the oracle, also with the
    plane-inverse sums split into groups. ACE requests of the two trajectories stay in separate
    launches."""
    import torch
    from paper_1905_01348_amd import Context, Server

    n3, L, N = (24, 24, 24), 10.26, 16
    ctx = Context(0)
    if c_split:
        ctx.set_vx_config({"kernels": 1, "c_split": c_split}, n=24, L=L, prec="fp32acc64")
    srv = Server(ctx, max_slots=1, n_streams=1, max_batch_pairs=1 << 16)
    psis = {}
    for t, seed in ((5, 501), (6, 502)):
        psis[t] = synth.make_orbitals(seed, n3, L, N, dtype=np.complex64)
        srv.register(t, dev(psis[t]), n=n3, L=L, kernel="hse", omega=0.106, vx_prec="fp32acc64",
                     ace_prec="ace_fp32r")

    def outs(rs):
        return [torch.full((r["count"], 24, 24, 24), complex(9.0, 9.0), dtype=torch.complex64, device="cuda")
                for r in rs]

    reqs = [dict(traj=5, op=0, first=0, count=4, t=0.0), dict(traj=6, op=0, first=8, count=4, t=0.0),
            dict(traj=5, op=0, first=12, count=4, t=0.0), dict(traj=6, op=0, first=2, count=3, t=0.0)]
    for r, o in zip(reqs, outs(reqs)):
        r["out"] = o
    st, lat, rep = srv.serve(reqs)
    torch.cuda.synchronize()
    say("two trajectories, V_X:", rep)
    assert st == [0, 0, 0, 0]
    assert rep["n_batches"] == 1, "same-grid V_X requests of two trajectories should share one launch"
    for i, r in enumerate(reqs):
        psi = psis[r["traj"]].astype(np.complex128)
        ref = oracle.apply_vx(psi, psi[r["first"]:r["first"] + r["count"]], n3, L, "hse", 0.106)
        mixed = host(r["out"])
        err = rel_err(mixed, ref)
        say("  request", i, "traj", r["traj"], "oracle err", err)
        assert err <= 1e-5
        alone = dict(r, out=outs([r])[0])
        st1, _, rep1 = srv.serve([alone])
        assert st1 == [0] and rep1["n_batches"] == 1
        assert np.array_equal(host(alone["out"]).view(np.float32), mixed.view(np.float32)), i
    ace_reqs = [dict(traj=5, op=1, first=0, count=4, t=0.0), dict(traj=6, op=1, first=0, count=4, t=0.0)]
    for r, o in zip(ace_reqs, outs(ace_reqs)):
        r["out"] = o
    st, lat, rep = srv.serve(ace_reqs)
    assert st == [0, 0] and rep["n_batches"] == 2
    srv.close()
    ctx.close()


def test_admission_busy_and_cancel():
    """A queue cap refuses arrivals with FX_ERR_BUSY; cancelled requests report FX_ERR_CANCELLED and
    the others complete; a cancellation from another thread while serving leaves every request
    either done or cancelled."""
    import threading

    import torch
    from paper_1905_01348_amd import Context, Server

    ctx = Context(0)
    n3, L, N = (24, 24, 24), 10.26, 16
    psi = synth.make_orbitals(77, n3, L, N, dtype=np.complex64)

    def mk(n):
        rs = [dict(traj=0, op=i % 2, first=(4 * i) % 16, count=4, t=0.0) for i in range(n)]
        for r in rs:
            r["out"] = torch.zeros((4, 24, 24, 24), dtype=torch.complex64, device="cuda")
        return rs

    srv = Server(ctx, max_slots=1, n_streams=1, max_batch_pairs=64, max_queue=3)
    srv.register(0, dev(psi), n=n3, L=L)
    st, lat, rep = srv.serve(mk(12))
    say("queue cap 3:", st, rep)
    assert st.count(-6) > 0 and all(s in (0, -6) for s in st)
    assert rep["n_rejected"] == st.count(-6) and rep["n_done"] == st.count(0)
    srv.close()

    srv = Server(ctx, max_slots=1, n_streams=1, max_batch_pairs=64)
    srv.register(0, dev(psi), n=n3, L=L)
    reqs = mk(10)
    for i in (1, 4, 7):
        srv.cancel(i)
    st, lat, rep = srv.serve(reqs)
    say("cancelled 1, 4, 7:", st, rep)
    assert [i for i, s in enumerate(st) if s == -7] == [1, 4, 7] and rep["n_cancelled"] == 3
    assert all(s == 0 for i, s in enumerate(st) if i not in (1, 4, 7))
    for i in (1, 4, 7):
        assert torch.count_nonzero(reqs[i]["out"]).item() == 0
    # cancellations were forgotten when serve returned
    st, lat, rep = srv.serve(mk(4))
    assert st == [0, 0, 0, 0]
    # from another thread while serving (arrivals spread over 0.2 s)
    reqs = mk(40)
    for i, r in enumerate(reqs):
        r["t"] = 0.005 * i
    th = threading.Thread(target=lambda: [srv.cancel(i) for i in range(20, 40)])
    th.start()
    st, lat, rep = srv.serve(reqs)
    th.join()
    say("threaded cancel:", rep)
    assert all(s in (0, -7) for s in st) and all(s == 0 for s in st[:10])
    assert rep["n_done"] + rep["n_cancelled"] == 40
    srv.close()
    ctx.close()
