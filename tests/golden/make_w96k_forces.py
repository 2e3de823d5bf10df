"""Writes w96k_forces.json: FP64 oracle energies (all components) and the total
force on 600 sampled atoms of the 96,000-atom water box's initial state.
Calls only synth/ (inputs) and oracle/.

    python tests/golden/make_w96k_forces.py

Terms: LJ and real-space Ewald over the float32-decided interaction set
(Eqs. 4-5, 10), exclusion correction and self term (Eq. 12), bonds and
angles (Eqs. 1-2), and the reciprocal sum by smooth PME on the 100^3 grid.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import forcefield  # noqa: E402

N_SAMPLE = 600


def main():
    t0 = time.perf_counter()
    s = synth.config_system("water96k")
    nb = forcefield.nonbonded_terms(s)
    rec = forcefield.pme_terms(s)
    F = nb["F"] + rec["F"]
    sample = np.sort(np.random.default_rng(96).choice(s.n_atoms, N_SAMPLE, replace=False))
    out = {
        "citation": "oracle FP64 energies and forces of the seeded 96,000-atom water box "
                    "(Eqs. 1-2, 4-5, 10, 12 and smooth PME); written by this script",
        "energy_names": list(forcefield.ENERGY_NAMES) + ["coul_rec"],
        "energies": [float(v) for v in nb["E"]] + [float(rec["E"])],
        "n_interacting": int(nb["n_interacting"]),
        "sample": [int(i) for i in sample],
        "forces": [[float(F[d, i]) for d in range(3)] for i in sample],
        "force_rms_all": float(np.sqrt((F * F).mean())),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "w96k_forces.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} in {time.perf_counter() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
