"""Writes oracle_energies.json.  Calls only the oracle (and the input generators)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2107_01664_amd import meshgen as mg  # noqa: E402


def main():
    out = {"icosphere_unperturbed": {}, "small_sphere": {}}
    for L in range(4):
        m = mg.icosphere(L)
        out["icosphere_unperturbed"][str(L)] = O.energy(m.V, m.F)
    m = mg.workload("small_sphere")
    E, g = O.gradient(m.V, m.F)
    out["small_sphere"] = {"E": E, "dE_norm": float(np.linalg.norm(g))}
    out["_source"] = ("oracle FP64, alpha=6 beta=12; icosphere levels 0-3 by midpoint "
                      "subdivision; small_sphere = icosphere 3 + N(0, 0.01^2) noise, seed 0")
    with open(os.path.join(HERE, "oracle_energies.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
