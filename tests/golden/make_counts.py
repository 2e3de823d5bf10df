"""Writes pair_counts.json: unique non-excluded pairs within r_c (interacting)
and within r_c + r_g (listed) of each workload's initial state, counted by the
oracle's float32 predicate, and the sha256 of the whole sorted list (int32
(i, j) rows, i < j, little-endian, row-major), so that a GPU test can compare
the complete list of the largest workload without recomputing it. Calls only
synth/ (inputs) and oracle/.

    python tests/golden/make_counts.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import neighbors  # noqa: E402


def main():
    out = {"citation": "pair counts of the seeded synthetic workloads; Verlet list of Sec. II.A.2 "
                       "with the float32 inclusion predicate (oracle/neighbors.py)"}
    for name in ("lj1k", "water9k", "water96k"):
        s = synth.config_system(name)
        pairs = neighbors.tree_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
        inter = int(neighbors.interacting(s.pos, s.box, s.r_cut, s.r_ghost, pairs).sum())
        rows = np.ascontiguousarray(pairs, dtype="<i4")
        out[name] = {"n_atoms": s.n_atoms, "listed_pairs": int(len(pairs)),
                     "interacting_pairs": inter, "excluded_pairs": int(len(s.exclusions)),
                     "list_sha256": hashlib.sha256(rows.tobytes()).hexdigest()}
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_counts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
