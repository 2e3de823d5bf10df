"""Rigid water by holonomic constraints (test infrastructure; the paper's
SETTLE option for water, Sec. III, which allows the 4x longer time step).

SETTLE solves analytically what SHAKE solves iteratively: the three distance
constraints of a rigid water molecule (O-H1, O-H2, H1-H2). The oracle uses the
plain definitions, in float64:

* shake: given the constrained positions x (the reference directions) and
  unconstrained new positions y, find y' = y + sum_c g_c s_c,i r_c(x) / m_i
  (r_c = x_a - x_b, minimum image; s = +1 on a, -1 on b) with every
  |y'_a - y'_b| = d_c, by SHAKE iterations to a relative tolerance of 1e-12
  (coordinates of tens of units round |y_a - y_b|^2 at about 1e-14).
* rattle_velocities: v' = v + sum_c mu_c s_c,i r_c / m_i with
  r_c . (v'_a - v'_b) = 0 for every constraint, an exact 3 x 3 solve per
  molecule.
* velocity_verlet_rattle: the velocity-Verlet step with both (RATTLE).
"""
from __future__ import annotations

import numpy as np


def _mi(d, L):
    return d - L * np.round(d / L)


def _pairs(mols):
    """Constraint atom pairs per molecule: (O,H1), (O,H2), (H1,H2)."""
    m = np.asarray(mols, np.int64)
    return [(m[:, 0], m[:, 1]), (m[:, 0], m[:, 2]), (m[:, 1], m[:, 2])]


def shake(x_ref, y, mass, box, mols, d_oh, d_hh, tol=1e-12, max_iter=1000):
    x_ref = np.asarray(x_ref, np.float64)
    y = np.asarray(y, np.float64).copy()
    L = np.asarray(box, np.float64)[:, None]
    inv_m = 1.0 / np.asarray(mass, np.float64)
    pairs = _pairs(mols)
    dist = [d_oh, d_oh, d_hh]
    refs = [_mi(x_ref[:, a] - x_ref[:, b], L) for a, b in pairs]
    for it in range(max_iter):
        worst = 0.0
        for (a, b), d, r in zip(pairs, dist, refs):
            s = _mi(y[:, a] - y[:, b], L)
            diff = (s * s).sum(axis=0) - d * d
            worst = max(worst, float(np.abs(diff).max()) / (d * d))
            g = diff / (2.0 * (inv_m[a] + inv_m[b]) * (s * r).sum(axis=0))
            y[:, a] -= g * r * inv_m[a]
            y[:, b] += g * r * inv_m[b]
        if worst < tol:
            return y, it
    raise RuntimeError("SHAKE did not converge")


def rattle_velocities(x, v, mass, box, mols):
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64).copy()
    L = np.asarray(box, np.float64)[:, None]
    inv_m = 1.0 / np.asarray(mass, np.float64)
    pairs = _pairs(mols)
    r = [_mi(x[:, a] - x[:, b], L) for a, b in pairs]           # [3, M] each
    nm = len(pairs[0][0])
    A = np.zeros((nm, 3, 3))
    rhs = np.zeros((nm, 3))
    for c, (a, b) in enumerate(pairs):
        rhs[:, c] = -(r[c] * (v[:, a] - v[:, b])).sum(axis=0)
        for c2, (a2, b2) in enumerate(pairs):
            # d(v_a - v_b) / d mu_c2 = r_c2 (s_c2,a / m_a - s_c2,b / m_b)
            coef = ((a2 == a) * inv_m[a] - (b2 == a) * inv_m[a]
                    - (a2 == b) * inv_m[b] + (b2 == b) * inv_m[b])
            A[:, c, c2] = (r[c] * r[c2]).sum(axis=0) * coef
    mu = np.linalg.solve(A, rhs[:, :, None])[:, :, 0]
    for c2, (a2, b2) in enumerate(pairs):
        v[:, a2] += mu[:, c2] * r[c2] * inv_m[a2]
        v[:, b2] -= mu[:, c2] * r[c2] * inv_m[b2]
    return v


def velocity_verlet_rattle(pos, vel, mass, box, force_fn, dt, n_steps, accel, mols, d_oh,
                           d_hh):
    """Returns dict(pos, vel, traj) with the constraints held every step."""
    x = np.asarray(pos, np.float64).copy()
    v = rattle_velocities(x, vel, mass, box, mols)
    m = np.asarray(mass, np.float64)
    L = np.asarray(box, np.float64)[:, None]
    F = force_fn(x)
    traj = [x.copy()]
    for _ in range(n_steps):
        v = v + 0.5 * dt * accel * F / m[None, :]
        y = x + dt * v
        y2, _ = shake(x, y, m, box, mols, d_oh, d_hh)
        v = v + (y2 - y) / dt
        x = y2 - L * np.floor(y2 / L)
        F = force_fn(x)
        v = v + 0.5 * dt * accel * F / m[None, :]
        v = rattle_velocities(x, v, m, box, mols)
        traj.append(x.copy())
    return dict(pos=x, vel=v, traj=np.array(traj))
