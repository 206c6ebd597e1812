"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Calls only oracle/ and the seeded input generator.  Run from the repo root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import floquet_inputs as fin  # noqa: E402
import oracle as O  # noqa: E402


def c1_energy_series():
    L, n, seed = 12, 1000, fin.DEFAULT_SEED
    w = fin.xyz_workload(L, seed=seed)
    hs = O.xyz_bond_hamiltonians(L, w["J"], w["fields"])
    _, rows = O.run_energy_series(L, hs, w["T"], w["spinors"], n, every=1)
    keep = [0, 1, 2, 3, 5, 10, 20, 50, 100, 200, 500, 999, 1000]
    out = {
        "_about": "Energy density e = <H0>/(L <psi|psi>) of the L=12 XYZ-plus-fields chain "
                  "(T = 0.25, seed 2111) from the FP64 oracle, gate by gate.",
        "L": L, "n": n, "seed": seed, "T": w["T"],
        "energy_density": {str(t): rows[t][1] for t in keep},
        "norm": {str(t): rows[t][3] for t in keep},
    }
    with open(os.path.join(HERE, "c1_energy_L12.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    c1_energy_series()
