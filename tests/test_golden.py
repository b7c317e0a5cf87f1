"""Frozen oracle outputs (tests/golden, written by tests/golden/make_golden.py from oracle/ only)."""
import json
import os

import numpy as np

import oracle
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_24cube_oracle_frozen():
    g = json.load(open(os.path.join(HERE, "24cube_16_oracle.json")))
    w = synth.workload("24cube_16")
    psi = synth.make_orbitals(w["seed"], w["n"], w["L"], w["N"])
    out = oracle.apply_vx(psi, psi, w["n"], w["L"], "coulomb")
    assert abs(oracle.exchange_energy(psi, out) - g["ex"]) <= 1e-11 * abs(g["ex"])
    norms = [np.linalg.norm(out[k]) for k in range(out.shape[0])]
    np.testing.assert_allclose(norms, g["col_norms"], rtol=1e-11)
    for k, z, y, x, re, im in g["probes"]:
        assert abs(out[k, z, y, x] - complex(re, im)) <= 1e-11 * max(norms)
    ace = oracle.build_ace(psi, out)
    np.testing.assert_allclose(np.diag(ace["L"]).real, g["L_diag"], rtol=1e-11)
    # E_X = 1/2 tr M
    assert abs(0.5 * g["trace_M"] - g["ex"]) <= 1e-12 * abs(g["ex"])
