"""Short-range nonbonded terms in float64 (paper Sec. II.A.2).

* Lennard-Jones 12-6, Eq. (4), with Lorentz-Berthelot mixing, Eq. (5), and the
  optional C2 switching function of Eq. (6) applied to LJ only.
* Real-space Ewald term, the n = 0 (minimum-image) part of the direct sum,
  Eq. (10): k_e q_i q_j erfc(alpha r) / r for every interacting, non-excluded
  pair (the minimum image is the only image inside r_c because r_c < L/2).
* Exclusion correction: excluded pairs are dropped from the list (paper,
  "Exclusions and Exceptions"); since the reciprocal sum still contains their
  smooth erf part, it is removed here: -k_e q_i q_j erf(alpha r)/r, minimum
  image, no cutoff.
* Self energy, Eq. (12), scaled by k_e, and the neutralising-background term
  -k_e pi Q^2 / (2 V alpha^2) for a net charge Q (zero for neutral systems).
* Reaction field, Eq. (8), instead of Ewald when eps_s > 0: k_e q_i q_j
  (1/r + k_RF r^2 - c_RF) for every interacting, non-excluded pair, with the
  solvent dielectric eps_s in both constants (reading: the printed constants
  mix eps and eps_s; with eps_s in both, the pair energy vanishes at r_c);
  eps_s = inf is the conducting limit k_RF = 1/(2 r_c^3), c_RF = 3/(2 r_c).
  Excluded pairs get no term, and there is no self or reciprocal part.

Forces are the analytic negative gradients. The virial tensor is
W_ab = sum_pairs d_a F_b, with d = x_j - x_i (minimum image) and F the force
on j, so that trace(W) = -dU/dlambda under the affine scaling (x, L) -> lambda (x, L).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc


def displacement(pos, box, i, j):
    """Exact float64 minimum-image x_j - x_i (one wrap, positions in [0, L))."""
    pos = np.asarray(pos, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)[:, None]
    d = pos[:, j] - pos[:, i]
    d = np.where(d > 0.5 * L, d - L, np.where(d < -0.5 * L, d + L, d))
    return d


def switch(r, r_s, r_c):
    """S(x) = 1 - 6x^5 + 15x^4 - 10x^3, x = (r - r_s)/(r_c - r_s), Eq. (6); and dS/dr."""
    x = np.clip((r - r_s) / (r_c - r_s), 0.0, 1.0)
    S = 1.0 - 6.0 * x ** 5 + 15.0 * x ** 4 - 10.0 * x ** 3
    dS = (-30.0 * x ** 4 + 60.0 * x ** 3 - 30.0 * x ** 2) / (r_c - r_s)
    inside = (r > r_s) & (r < r_c)
    return np.where(r <= r_s, 1.0, np.where(inside, S, 0.0)), np.where(inside, dS, 0.0)


def _accumulate(n, i, j, fj):
    F = np.zeros((3, n))
    for a in range(3):
        F[a] += np.bincount(j, weights=fj[a], minlength=n)
        F[a] -= np.bincount(i, weights=fj[a], minlength=n)
    return F


def reaction_field_constants(r_cut, eps_s):
    """(k_RF, c_RF) of Eq. (8) for cutoff r_cut and solvent dielectric eps_s."""
    rc = float(r_cut)
    if math.isinf(eps_s):
        return 1.0 / (2.0 * rc ** 3), 3.0 / (2.0 * rc)
    return (eps_s - 1.0) / ((2.0 * eps_s + 1.0) * rc ** 3), 3.0 * eps_s / ((2.0 * eps_s + 1.0) * rc)


def pair_terms(pos, box, pairs, atom_type, type_sigma, type_epsilon, charge,
               alpha, coulomb_k, r_cut=None, switch_r=0.0, rf_epsilon=0.0):
    """LJ and real-space Ewald (or, with rf_epsilon > 0, the reaction field)
    over the given interacting pairs.

    Returns dict(E_lj, E_dir, F [3,N], W [3,3]).
    """
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    if len(pairs) == 0:
        return dict(E_lj=0.0, E_dir=0.0, F=np.zeros((3, n)), W=np.zeros((3, 3)))
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    d = displacement(pos, box, i, j)
    r = np.sqrt((d * d).sum(axis=0))
    t = np.asarray(atom_type)
    sig = np.asarray(type_sigma, np.float64)[t]
    eps = np.asarray(type_epsilon, np.float64)[t]
    sij = 0.5 * (sig[i] + sig[j])                 # Eq. (5)
    eij = np.sqrt(eps[i] * eps[j])                # Eq. (5)
    s6 = (sij / r) ** 6
    u_lj = 4.0 * eij * (s6 * s6 - s6)             # Eq. (4)
    du_lj = 4.0 * eij * (-12.0 * s6 * s6 + 6.0 * s6) / r
    if switch_r and switch_r > 0:
        S, dS = switch(r, float(switch_r), float(r_cut))
        du_lj = du_lj * S + u_lj * dS
        u_lj = u_lj * S
    q = np.asarray(charge, np.float64)
    if rf_epsilon and rf_epsilon > 0 and coulomb_k != 0:
        k_rf, c_rf = reaction_field_constants(r_cut, rf_epsilon)
        qq = coulomb_k * q[i] * q[j]
        u_c = qq * (1.0 / r + k_rf * r * r - c_rf)            # Eq. (8)
        du_c = qq * (-1.0 / r ** 2 + 2.0 * k_rf * r)
    elif alpha > 0 and coulomb_k != 0:
        qq = coulomb_k * q[i] * q[j]
        u_c = qq * erfc(alpha * r) / r            # Eq. (10), n = 0 term
        du_c = -qq * (erfc(alpha * r) / r ** 2
                      + 2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2) / r)
    else:
        u_c = np.zeros_like(r)
        du_c = np.zeros_like(r)
    fmag = -(du_lj + du_c) / r                    # force on j along d
    fj = d * fmag
    W = (d[:, None, :] * fj[None, :, :]).sum(axis=2)
    return dict(E_lj=float(u_lj.sum()), E_dir=float(u_c.sum()),
                F=_accumulate(n, i, j, fj), W=W)


def exclusion_correction(pos, box, exclusions, charge, alpha, coulomb_k):
    """-k_e sum_excl q_i q_j erf(alpha r)/r, minimum image, no cutoff."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    ex = np.asarray(exclusions, dtype=np.int64).reshape(-1, 2)
    if len(ex) == 0 or alpha <= 0:
        return dict(E=0.0, F=np.zeros((3, n)), W=np.zeros((3, 3)))
    i, j = ex[:, 0], ex[:, 1]
    d = displacement(pos, box, i, j)
    r = np.sqrt((d * d).sum(axis=0))
    q = np.asarray(charge, np.float64)
    qq = coulomb_k * q[i] * q[j]
    u = -qq * erf(alpha * r) / r
    du = -qq * (2.0 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2) / r
                - erf(alpha * r) / r ** 2)
    fj = d * (-du / r)
    W = (d[:, None, :] * fj[None, :, :]).sum(axis=2)
    return dict(E=float(u.sum()), F=_accumulate(n, i, j, fj), W=W)


def self_energy(charge, box, alpha, coulomb_k):
    """Eq. (12) times k_e, plus the neutralising term for a net charge."""
    q = np.asarray(charge, np.float64)
    V = float(np.prod(np.asarray(box, np.float64)))
    e_self = -coulomb_k * alpha / math.sqrt(math.pi) * float((q * q).sum())
    Q = float(q.sum())
    e_net = -coulomb_k * math.pi * Q * Q / (2.0 * V * alpha * alpha) if alpha > 0 else 0.0
    return e_self + e_net
