"""Write tests/golden/*.json from the FP64 oracle alone.

The paper prints no worked example (its figures are not reproduced in the
text), so stored values here are oracle outputs on seeded inputs, frozen so
that any later change to the oracle's arithmetic shows up as a diff.  Run:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def small_case():
    """24^3 cell of 10.26 bohr, 16 orbitals, Coulomb: the 8-Si-atom workload."""
    w = synth.workload("24cube_16")
    psi = synth.make_orbitals(w["seed"], w["n"], w["L"], w["N"])
    out = oracle.apply_vx(psi, psi, w["n"], w["L"], "coulomb")
    ace = oracle.build_ace(psi, out)
    probes = [(0, 0, 0, 0), (3, 5, 7, 11), (15, 23, 1, 9), (8, 12, 12, 12)]
    return {
        "workload": "24cube_16",
        "ex": oracle.exchange_energy(psi, out),
        "trace_M": float(np.trace(ace["M"]).real),
        "col_norms": [float(np.linalg.norm(out[k])) for k in range(out.shape[0])],
        "probes": [[k, z, y, x, float(out[k, z, y, x].real), float(out[k, z, y, x].imag)]
                   for (k, z, y, x) in probes],
        "L_diag": [float(v.real) for v in np.diag(ace["L"])],
    }


if __name__ == "__main__":
    data = small_case()
    with open(os.path.join(HERE, "24cube_16_oracle.json"), "w") as f:
        json.dump(data, f, indent=1)
    print("wrote 24cube_16_oracle.json")
