"""Launch configurations of the V_X path and the autotuner, on the GPU.

* Every specialised-kernel variant (prefetch form, z-pass tile, plane-inverse
  threads) agrees with the default to rounding and with the oracle to the
  tolerance; another batch volume gives bitwise the same result.
* Every generic radix schedule, z-pass tile and thread count matches the
  FP64 oracle within the precision's tolerance (1e-10 FP64, 1e-5 FP32).
* The autotuner stores a configuration that later applies use, and the
  result still matches the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_1905_01348_amd import fock as F
from tests.gpu_util import rel_err, dev, host, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32acc64": 1e-5, "fp32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    from paper_1905_01348_amd import Context

    c = Context(0)
    yield c
    c.close()


def _bits(a):
    return a.view(np.float64 if a.dtype == np.complex128 else np.float32)


def test_config_store_roundtrip_and_validation(ctx):
    n = (24, 24, 24)
    cfg, is_set = ctx.get_vx_config(n=n, prec="fp64")
    assert not is_set and cfg["a_prefetch"] == -1
    want = {"kernels": 1, "work_mb": 2048, "a_prefetch": 1, "b_variant": 2}
    ctx.set_vx_config(want, n=n, prec="fp64")
    got, is_set = ctx.get_vx_config(n=n, prec="fp64")
    assert is_set and all(got[k] == v for k, v in want.items())
    # other precision / form untouched
    assert not ctx.get_vx_config(n=n, prec="fp32")[1]
    assert not ctx.get_vx_config(n=n, prec="fp64", phi_is_psi=True)[1]
    ctx.set_vx_config(None, n=n, prec="fp64")
    assert not ctx.get_vx_config(n=n, prec="fp64")[1]
    bad = [
        ({"kernels": 3}, n), ({"a_prefetch": 2}, n), ({"b_variant": 5}, n), ({"c_variant": 6}, n), ({"c_split": 3}, n), ({"a_variant": -1}, n), ({"nt_hint": 2}, n), ({"b_xtile": 25}, n),
        ({"b_threads": 100}, n), ({"b_threads": 512}, n), ({"radix": [[5, 5]]}, n), ({"radix": [[6, 2]]}, n),
        ({"kernels": 1}, (18, 16, 12)),  # no specialised kernels off the workload edges
        ({"kernels": 1, "radix": [[4, 6]]}, n),  # specialised kernels run the default schedule only
    ]
    for c, grid in bad:
        with pytest.raises(F.FockError) as ei:
            ctx.set_vx_config(c, n=grid, prec="fp64")
        assert ei.value.status == F.FX_ERR_INVALID, c


@pytest.mark.parametrize("n", [24, 48, 72, 96])
def test_specialised_variants_match(ctx, n):
    """Kernel-shape variants (other instantiations: the compiler may fuse multiply-adds
    differently) agree with the default to rounding and with the oracle to the tolerance;
    the batch volume (same kernels) gives bitwise the same result."""
    L = n * 10.26 / 24
    N, Nt = 5, 3
    psi = synth.make_orbitals(50 + n, n, L, N)
    phi = synth.random_grid_vectors(51 + n, n, Nt)
    P, Q = dev(psi), dev(phi)
    refs = {False: oracle.apply_vx(psi, phi, n, L, "hse", 0.106), True: oracle.apply_vx(psi, psi, n, L, "hse", 0.106)}
    shapes = [{"a_prefetch": 1}, {"b_variant": 2}, {"b_variant": 3}, {"b_variant": 4}, {"c_variant": 1}, {"c_variant": 2}, {"c_variant": 3}, {"c_variant": 4},
              {"c_variant": 5}, {"a_variant": 2}, {"a_variant": 3},
              {"c_split": 2}, {"c_split": 4}, {"c_split": 8, "c_variant": 1},
              {"nt_hint": 1},
              {"a_prefetch": 1, "a_variant": 2, "b_variant": 2, "c_variant": 2}]
    close = {"fp64": 1e-13, "fp32acc64": 1e-6, "fp32": 1e-6}
    for prec in ("fp64", "fp32acc64", "fp32"):
        for square in (False, True):
            ctx.set_vx_config(None, n=n, prec=prec, phi_is_psi=square)
            call = (lambda: ctx.apply_vx(P, n=n, L=L, prec=prec)) if square else \
                (lambda: ctx.apply_vx(P, Q, n=n, L=L, prec=prec))
            ref = host(call())
            worst = 0.0
            for v in shapes:
                ctx.set_vx_config(dict(v, kernels=1), n=n, prec=prec, phi_is_psi=square)
                got = host(call())
                d = rel_err(got, ref)
                worst = max(worst, d)
                assert d <= close[prec], (prec, square, v, d)
                assert rel_err(got, refs[square]) <= TOL[prec], (prec, square, v)
            ctx.set_vx_config({"kernels": 1, "work_mb": 64}, n=n, prec=prec, phi_is_psi=square)
            assert np.array_equal(_bits(host(call())), _bits(ref)), (prec, square, "work_mb")
            ctx.set_vx_config(None, n=n, prec=prec, phi_is_psi=square)
            say("edge", n, prec, "square" if square else "rect", "largest variant difference", worst)


@pytest.mark.parametrize("n3", [(24, 36, 16), (48, 12, 18)])
def test_generic_schedules_tiles_threads_match_oracle(ctx, n3):
    L3 = (7.0, 9.0, 5.5)
    N, Nt = 4, 3
    psi = synth.make_orbitals(60, n3, L3, N, ecut=1e4)
    phi = synth.random_grid_vectors(61, n3, Nt)
    ref = oracle.apply_vx(psi, phi, n3, L3, "hse", 0.106)
    P, Q = dev(psi), dev(phi)
    cfgs = []
    for ax in range(3):
        for p in F.debug_axis_plans(n3[ax]):
            r = [[], [], []]
            r[ax] = p
            cfgs.append({"kernels": 2, "radix": r})
    for xt in (4, 8, 16, n3[0]):
        cfgs.append({"kernels": 2, "b_xtile": xt})
    for nt in (64, 128, 256):
        cfgs.append({"kernels": 2, "b_threads": nt})
    for prec in ("fp64", "fp32acc64"):
        worst = 0.0
        for c in cfgs:
            ctx.set_vx_config(c, n=n3, L=L3, prec=prec)
            got = host(ctx.apply_vx(P, Q, n=n3, L=L3, kernel="hse", prec=prec))
            e = rel_err(got, ref)
            worst = max(worst, e)
            assert e <= TOL[prec], (prec, c, e)
        ctx.set_vx_config(None, n=n3, L=L3, prec=prec)
        say("generic", n3, prec, len(cfgs), "configurations, worst err", worst)


@pytest.mark.parametrize("case", [((24, 24, 24), 16, 16, True, "fp64"), ((24, 24, 24), 16, 6, False, "fp32acc64"),
                                  ((18, 16, 12), 9, 5, False, "fp64"), ((48, 48, 48), 40, 40, True, "fp32acc64")],
                         ids=["24-square-fp64", "24-fp32acc64", "generic-fp64", "48-square-fp32acc64"])
def test_autotune_stores_a_config_that_applies_use(ctx, case):
    n3, N, Nt, square, prec = case
    L3 = tuple(0.43 * x for x in n3)
    cfg, ms = ctx.vx_autotune(n=n3, L=L3, n_psi=N, n_phi=Nt, phi_is_psi=square, prec=prec)
    say("autotune", case, cfg, f"{ms:.4f} ms per 1000 pairs")
    assert ms > 0
    stored, is_set = ctx.get_vx_config(n=n3, prec=prec, phi_is_psi=square)
    assert is_set and stored == cfg
    assert cfg["kernels"] in (1, 2)
    psi = synth.make_orbitals(70, n3, L3, N, ecut=1e4)
    ref_phi = psi[:Nt] if square else synth.random_grid_vectors(71, n3, Nt)
    ref = oracle.apply_vx(psi, ref_phi, n3, L3, "hse", 0.106)
    P = dev(psi)
    got = host(ctx.apply_vx(P, None if square else dev(ref_phi), n=n3, L=L3, kernel="hse", prec=prec))
    assert rel_err(got, ref) <= TOL[prec]
    ctx.set_vx_config(None, n=n3, prec=prec, phi_is_psi=square)


def test_configurations_saved_and_loaded(tmp_path, monkeypatch):
    """Tuned configurations survive the context: saved to a file and loaded by a new context
    (explicitly, or at fx_init through FX_TUNE_CACHE, which fx_vx_autotune also writes)."""
    from paper_1905_01348_amd import Context

    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("FX_TUNE_CACHE", path)
    c = Context(0)
    cfg, ms = c.vx_autotune(n=24, L=10.26, n_psi=16, n_phi=4, prec="fp32acc64")
    c.close()
    text = open(path).read()
    say("tune cache file:", text)
    assert "fxcfg gfx950/" in text
    c2 = Context(0)  # loads FX_TUNE_CACHE at init
    got, is_set = c2.get_vx_config(n=24, prec="fp32acc64", phi_is_psi=False)
    assert is_set and got == cfg
    c2.close()
    monkeypatch.delenv("FX_TUNE_CACHE")
    c3 = Context(0)
    assert not c3.get_vx_config(n=24, prec="fp32acc64", phi_is_psi=False)[1]
    assert c3.load_configs(path) >= 1
    assert c3.get_vx_config(n=24, prec="fp32acc64", phi_is_psi=False) == (cfg, True)
    # saving keeps lines of other devices
    with open(path, "a") as f:
        f.write("fxcfg gfx000/1 24 24 24 2 0 1 0 0 1 1 1 1 0 0 0 0 0 0 0 0 0 0 0 0 0 0\n")
    c3.save_configs(path)
    assert "gfx000/1" in open(path).read()
    with open(path, "a") as f:
        f.write("not a configuration\n")
    from paper_1905_01348_amd import FockError
    with pytest.raises(FockError):
        c3.load_configs(path)
    c3.close()
