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
* settle: the same position constraints in closed form (the method of
  Miyamoto and Kollman, 1992, as derived below), for molecules with two
  equal hydrogen masses.

SETTLE, derivation. The SHAKE solution moves each atom by a combination of
the old bond vectors, so (1) every displacement lies in the old molecular
plane, (2) the centre of mass stays where the unconstrained step put it, and
(3) sum_i x0_i x m_i (y'_i - y_i) = 0 (each constraint moves its two atoms
by equal and opposite amounts along their old separation). In a frame with
Z normal to the old plane and the origin at the centre of mass, (1) fixes
every atom's Z coordinate at its unconstrained value. The rigid triangle
(O at (0, ra), H at (-+rc, -rb), ra + rb its height h, ra = 2 m_H h / M)
rotated by psi about Y and phi about X has Z coordinates ra sin(phi) (O) and
-rb sin(phi) -+ rc sin(psi) cos(phi) (H1, H2), which give phi and psi; a
rotation by theta about Z changes no Z, and (3)'s Z component,
alpha sin(theta) + beta cos(theta) = gamma with
  alpha = sum m (x0 x2 + y0 y2), beta = sum m (x0 y2 - y0 x2),
  gamma = sum m (x0 y1 - y0 x1)
(x0, y0: old in-plane coordinates, x2, y2: the triangle after phi and psi,
x1, y1: unconstrained, all about the centres of mass), gives theta (the root
next to theta = 0).
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


def settle(x_ref, y, mass, box, mols, d_oh, d_hh):
    """Closed-form solution of the position constraints (see the module
    docstring): the same fixed point as shake(), without iterations."""
    x_ref = np.asarray(x_ref, np.float64)
    y = np.asarray(y, np.float64).copy()
    L = np.asarray(box, np.float64)[:, None]
    m = np.asarray(mass, np.float64)
    mol = np.asarray(mols, np.int64)
    ia, ib, ic = mol[:, 0], mol[:, 1], mol[:, 2]
    mo, mh = m[ia], m[ib]
    M = mo + 2.0 * mh
    rc = 0.5 * d_hh
    h = np.sqrt(d_oh * d_oh - rc * rc)
    ra = 2.0 * mh * h / M
    rb = h - ra
    # old and new geometry relative to O (minimum image), then to the COM
    ob0, oc0 = _mi(x_ref[:, ib] - x_ref[:, ia], L), _mi(x_ref[:, ic] - x_ref[:, ia], L)
    ob1, oc1 = _mi(y[:, ib] - y[:, ia], L), _mi(y[:, ic] - y[:, ia], L)
    com0 = (mh * ob0 + mh * oc0) / M
    com1 = (mh * ob1 + mh * oc1) / M
    old = [-com0, ob0 - com0, oc0 - com0]
    new = [-com1, ob1 - com1, oc1 - com1]
    Z = np.cross(ob0.T, oc0.T).T
    Z /= np.sqrt((Z * Z).sum(axis=0))
    X = np.cross(new[0].T, Z.T).T
    X /= np.sqrt((X * X).sum(axis=0))
    Y = np.cross(Z.T, X.T).T
    to = lambda v: ((v * X).sum(axis=0), (v * Y).sum(axis=0), (v * Z).sum(axis=0))
    o0, n1 = [to(v) for v in old], [to(v) for v in new]
    sphi = n1[0][2] / ra
    cphi = np.sqrt(1.0 - sphi * sphi)
    spsi = (n1[1][2] - n1[2][2]) / (2.0 * rc * cphi)
    cpsi = np.sqrt(1.0 - spsi * spsi)
    t2 = [(0.0 * sphi, ra * cphi),
          (-rc * cpsi, -rb * cphi - rc * spsi * sphi),
          (rc * cpsi, -rb * cphi + rc * spsi * sphi)]
    z2 = [ra * sphi, -rb * sphi + rc * spsi * cphi, -rb * sphi - rc * spsi * cphi]
    w = [mo, mh, mh]
    alpha = sum(wk * (o[0] * t[0] + o[1] * t[1]) for wk, o, t in zip(w, o0, t2))
    beta = sum(wk * (o[0] * t[1] - o[1] * t[0]) for wk, o, t in zip(w, o0, t2))
    gamma = sum(wk * (o[0] * n[1] - o[1] * n[0]) for wk, o, n in zip(w, o0, n1))
    ab = alpha * alpha + beta * beta
    sth = (alpha * gamma - beta * np.sqrt(ab - gamma * gamma)) / ab
    cth = np.sqrt(1.0 - sth * sth)
    cm = y[:, ia] + com1
    for k, atom in enumerate((ia, ib, ic)):
        x3 = t2[k][0] * cth - t2[k][1] * sth
        y3 = t2[k][0] * sth + t2[k][1] * cth
        y[:, atom] = cm + x3 * X + y3 * Y + z2[k] * Z
    return y


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
