"""Harmonic bonds and angles in float64 (paper Sec. II.A.1, Eqs. 1-2).

U_bond  = k (r - r0)^2                 (no factor 1/2, as printed)
U_angle = k (theta - theta0)^2,  theta = arccos(r_hat_ij . r_hat_lj)
with j the vertex atom of the (i, j, l) triple. Distances use the minimum
image, as the paper's edge-list distance helper does.
"""
from __future__ import annotations

import numpy as np

from .nonbonded import displacement


def bonds(pos, box, bond_idx, k, r0):
    pos = np.asarray(pos, np.float64)
    n = pos.shape[1]
    F = np.zeros((3, n))
    b = np.asarray(bond_idx, np.int64).reshape(-1, 2)
    if len(b) == 0:
        return dict(E=0.0, F=F, W=np.zeros((3, 3)))
    i, j = b[:, 0], b[:, 1]
    d = displacement(pos, box, i, j)
    r = np.sqrt((d * d).sum(axis=0))
    k = np.asarray(k, np.float64)
    r0 = np.asarray(r0, np.float64)
    E = k * (r - r0) ** 2
    fj = d * (-2.0 * k * (r - r0) / r)
    for a in range(3):
        F[a] += np.bincount(j, weights=fj[a], minlength=n)
        F[a] -= np.bincount(i, weights=fj[a], minlength=n)
    W = (d[:, None, :] * fj[None, :, :]).sum(axis=2)
    return dict(E=float(E.sum()), F=F, W=W)


def angles(pos, box, angle_idx, k, theta0):
    pos = np.asarray(pos, np.float64)
    n = pos.shape[1]
    F = np.zeros((3, n))
    t = np.asarray(angle_idx, np.int64).reshape(-1, 3)
    if len(t) == 0:
        return dict(E=0.0, F=F, W=np.zeros((3, 3)))
    i, j, l = t[:, 0], t[:, 1], t[:, 2]
    a = displacement(pos, box, j, i)      # x_i - x_j
    b = displacement(pos, box, j, l)      # x_l - x_j
    ra = np.sqrt((a * a).sum(axis=0))
    rb = np.sqrt((b * b).sum(axis=0))
    ah, bh = a / ra, b / rb
    c = np.clip((ah * bh).sum(axis=0), -1.0, 1.0)
    theta = np.arccos(c)
    k = np.asarray(k, np.float64)
    th0 = np.asarray(theta0, np.float64)
    E = k * (theta - th0) ** 2
    dU = 2.0 * k * (theta - th0)
    s = np.sqrt(np.maximum(1.0 - c * c, 1e-300))
    Fi = (dU / s) * (bh - c * ah) / ra
    Fl = (dU / s) * (ah - c * bh) / rb
    Fj = -(Fi + Fl)
    for ax in range(3):
        F[ax] += np.bincount(i, weights=Fi[ax], minlength=n)
        F[ax] += np.bincount(l, weights=Fl[ax], minlength=n)
        F[ax] += np.bincount(j, weights=Fj[ax], minlength=n)
    W = (a[:, None, :] * Fi[None, :, :]).sum(axis=2) + (b[:, None, :] * Fl[None, :, :]).sum(axis=2)
    return dict(E=float(E.sum()), F=F, W=W)
