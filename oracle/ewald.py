"""Ewald summation in float64 (paper Sec. II.A.2, Eqs. 9-14).

* alpha_from_tolerance: Eq. (13), alpha = sqrt(-ln(2 delta)) / r_c (natural log).
* kc_from_tolerance: the root of Eq. (14) read as
  delta = k_c sqrt(d alpha)/20 exp(-(pi k_c/(d alpha))^2), on its decreasing branch.
* reciprocal_direct: the reciprocal sum of Eq. (11) in its standard form
  (Eq. 11 as printed lacks the charges and the imaginary unit):
      E = k_e/(2 pi V) sum_{m != 0} exp(-pi^2 |m|^2/alpha^2)/|m|^2 |S(m)|^2,
      S(m) = sum_j q_j exp(2 pi i m . r_j),  m = (n1/L1, n2/L2, n3/L3),
  with tin-foil boundary conditions (no surface-dipole term).
* real_images: the direct sum of Eq. (10) over all periodic images inside a
  radius, excluding i = j in the home cell (the implied prime).
Together with the self term of Eq. (12) these give the full Ewald energy, which
is independent of alpha (the paper's remark after Eq. (12)).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.optimize import brentq
from scipy.special import erfc


def alpha_from_tolerance(delta: float, r_cut: float) -> float:
    return math.sqrt(-math.log(2.0 * delta)) / r_cut


def kc_from_tolerance(delta: float, alpha: float, d: float) -> float:
    f = lambda k: k * math.sqrt(d * alpha) / 20.0 * math.exp(-(math.pi * k / (d * alpha)) ** 2) - delta
    k_peak = d * alpha / (math.pi * math.sqrt(2.0))   # maximum of the printed expression
    hi = k_peak
    while f(hi) > 0:
        hi *= 2.0
    return brentq(f, k_peak, hi, xtol=1e-12)


def reciprocal_direct(pos, charge, box, alpha, coulomb_k, n_max):
    """Returns (E, F [3,N]) summed over integer vectors with |n_d| <= n_max."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(charge, np.float64)
    L = np.asarray(box, np.float64)
    V = float(np.prod(L))
    rng = np.arange(-n_max, n_max + 1)
    nv = np.array(list(itertools.product(rng, rng, rng)), dtype=np.float64)
    nv = nv[np.any(nv != 0, axis=1)]
    m = nv / L[None, :]
    msq = (m * m).sum(axis=1)
    f = np.exp(-np.pi ** 2 * msq / alpha ** 2) / msq
    E = 0.0
    F = np.zeros_like(pos)
    for c0 in range(0, len(m), 4096):
        mc = m[c0:c0 + 4096]
        fc = f[c0:c0 + 4096]
        phase = 2.0 * np.pi * (mc @ pos)                 # [M, N]
        S = (q[None, :] * np.exp(1j * phase)).sum(axis=1)
        E += float((fc * np.abs(S) ** 2).sum())
        # F_i = (2 k_e q_i / V) sum_m f(m) m Im(conj(S) e^{i phase_i})
        im = (np.conj(S)[:, None] * np.exp(1j * phase)).imag   # [M, N]
        F += (2.0 * coulomb_k / V) * q[None, :] * ((fc[:, None] * im).T @ mc).T
    return coulomb_k / (2.0 * np.pi * V) * E, F


def real_images(pos, charge, box, alpha, coulomb_k, r_max, exclusions=()):
    """Eq. (10) over all images with |r_ij + n| < r_max; pairs listed in
    `exclusions` skip only their home-cell (n = 0) term. Returns (E, F)."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(charge, np.float64)
    L = np.asarray(box, np.float64)
    n = pos.shape[1]
    nrep = [int(math.ceil(r_max / L[d])) + 1 for d in range(3)]
    shifts = np.array(list(itertools.product(*[range(-k, k + 1) for k in nrep])), np.float64) * L
    excl = set()
    for a, b in np.asarray(exclusions, np.int64).reshape(-1, 2):
        excl.add((int(a), int(b)))
        excl.add((int(b), int(a)))
    E = 0.0
    F = np.zeros_like(pos)
    for i in range(n):
        d = pos[:, :, None] - pos[:, i, None, None] + shifts.T[:, None, :]   # [3, N, S]
        r = np.sqrt((d * d).sum(axis=0))
        mask = r < r_max
        home = np.all(shifts == 0, axis=1)
        mask[i, home] = False
        for j in range(n):
            if (i, j) in excl:
                mask[j, home] = False
        rr = np.where(mask, r, 1.0)
        qq = coulomb_k * q[i] * q[:, None]
        u = np.where(mask, qq * erfc(alpha * rr) / rr, 0.0)
        du = np.where(mask, -qq * (erfc(alpha * rr) / rr ** 2 + 2 * alpha / math.sqrt(math.pi)
                                   * np.exp(-(alpha * rr) ** 2) / rr), 0.0)
        E += 0.5 * float(u.sum())
        # force on i: -dU/dx_i; d = x_j - x_i + n so dU/dx_i = -du * d/r
        F[:, i] += (du[None, :, :] * d / rr[None, :, :]).sum(axis=(1, 2))
    return E, F


def self_term(charge, alpha, coulomb_k):
    q = np.asarray(charge, np.float64)
    return -coulomb_k * alpha / math.sqrt(math.pi) * float((q * q).sum())
