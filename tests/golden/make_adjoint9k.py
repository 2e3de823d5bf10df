"""Writes adjoint_water9k.json: the FP64 adjoint oracle's loss and gradients
for the 9,000-atom water box (3,000 flexible waters, L = 44.8 A, PME 48^3),
100 velocity-Verlet steps of 1 fs from the seeded initial state, loss
U(x_T)/N + (1/N) sum |x_T - x_0|^2, charge direction 1 on O and -1/2 on H.
Stored: the loss, dL/d(eps_O, sigma_O, q_O, dt), the x0 and v0 gradients
projected on three seeded random directions, and 64 seeded sampled
coordinates of each; and the same quantities of a second oracle run whose
start positions carry float32-sized relative perturbations (6e-8, seeded):
how far rounding of the size a float32 run makes carries through 100 steps
of this chaotic system, the scale of the comparison with a float32 run.
Calls only synth/ (inputs) and oracle/; about half an hour of CPU.

    python tests/golden/make_adjoint9k.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import adjoint  # noqa: E402

N_STEPS, DT, SEED = 100, 1.0, 20541


def probes(n):
    """Seeded directions [3, 3, n] and sampled (axis, atom) coordinates [64, 2]."""
    rng = np.random.Generator(np.random.PCG64(SEED))
    dirs = rng.standard_normal((3, 3, n))
    flat = rng.choice(3 * n, 64, replace=False)
    return dirs, np.stack([flat // n, flat % n], axis=1)


def summary(g, dirs, coords):
    th = g["theta"]
    return {"loss": g["loss"], "eps_O": th[0], "sig_O": th[2], "q_O": th[4], "dt": g["dt"],
            "x0_dirs": [float((g["x0"] * d).sum()) for d in dirs],
            "v0_dirs": [float((g["v0"] * d).sum()) for d in dirs],
            "x0_coords": [float(g["x0"][a, i]) for a, i in coords],
            "v0_coords": [float(g["v0"][a, i]) for a, i in coords]}


def main():
    s = synth.config_system("water9k")
    ff = adjoint.ForceField(s)
    dq = np.where(s.atom_type == 0, 1.0, -0.5)
    t0 = time.time()
    x0 = s.pos.astype(np.float64)
    g = adjoint.gradients(ff, ff.params0(), x0, s.vel.astype(np.float64), DT, N_STEPS, dq)
    dirs, coords = probes(s.n_atoms)
    rng = np.random.Generator(np.random.PCG64(SEED + 1))
    xp = x0 * (1.0 + 6e-8 * rng.standard_normal(x0.shape))
    gp = adjoint.gradients(ff, ff.params0(), xp, s.vel.astype(np.float64), DT, N_STEPS, dq)
    th = g["theta"]
    out = {
        "citation": "gradients of a velocity-Verlet trajectory loss (Sec. I and IV: the "
                    "simulation is differentiated end to end); oracle/adjoint.py, frozen "
                    "interaction sets",
        "system": "water9k", "n_steps": N_STEPS, "dt_fs": DT, "seed": SEED,
        "loss": g["loss"], "eps_O": th[0], "sig_O": th[2], "q_O": th[4], "dt": g["dt"],
        "x0_dirs": [float((g["x0"] * d).sum()) for d in dirs],
        "v0_dirs": [float((g["v0"] * d).sum()) for d in dirs],
        "coords": coords.tolist(),
        "x0_coords": [float(g["x0"][a, i]) for a, i in coords],
        "v0_coords": [float(g["v0"][a, i]) for a, i in coords],
        "x0_norm": float(np.linalg.norm(g["x0"])), "v0_norm": float(np.linalg.norm(g["v0"])),
        "perturbed_start": summary(gp, dirs, coords),
        "cpu_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_water9k.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("loss", "eps_O", "sig_O", "q_O", "dt",
                                          "cpu_seconds")}))


if __name__ == "__main__":
    main()
