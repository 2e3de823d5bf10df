"""The Hamiltonian Monte Carlo tuning objective of the paper's Sec. IV, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For replicas i = 1..R from positions x_i,0 with standard normals xi_v[i]
(velocities) and xi_dt[i] (time step), the steps in the paper's order:

  1. velocities from the Maxwell-Boltzmann distribution of the masses:
     v_i,0 = sqrt(kT c / m) xi_v[i];
  2. the time step from the folded normal N_F(mu_dt, 0.01 mu_dt):
     dt_i = |mu_dt (1 + 0.01 xi_dt[i])|;
  3. L_q = the 0.999 quantile of N_F(mu_L, sigma_L) (rounded up) steps of
     velocity Verlet (Sec. II.D.1; a = c F / m);
  4. at every step l: E = U + K with K = sum m v^2 / (2 c), the acceptance
     probability alpha_i,l = min(1, exp(-(E_i,l - E_i,0)/kT)) and the jump
     |x_i,l - x_i,0|^2 (unwrapped positions, all atoms);
  5. L_HMC = (1/R) sum_i sum_l N_F(l; mu_L, sigma_L) alpha_i,l / l jump_i,l.

Everything is complex-safe (the branch of min and of the absolute value is
chosen from the real part; the force field of oracle/adjoint.py), so
derivatives of L_HMC with respect to mu_dt, mu_L or the masses along a
direction are complex steps. The interaction sets of each step are recorded
by the unperturbed run and reused (the frozen-set loss, as in
oracle/adjoint.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import adjoint

H_CS = 1e-30


def folded_normal_pdf(x, mu, sigma):
    c = 1.0 / math.sqrt(2.0 * math.pi * sigma * sigma)
    return c * (np.exp(-(x - mu) ** 2 / (2 * sigma * sigma)) +
                np.exp(-(x + mu) ** 2 / (2 * sigma * sigma)))


def folded_normal_quantile(mu, sigma, q=0.999):
    """x with P(|N(mu, sigma^2)| <= x) = q, by bisection on the CDF
    (1/2)[erf((x - mu)/(sigma sqrt 2)) + erf((x + mu)/(sigma sqrt 2))]."""
    cdf = lambda x: 0.5 * (math.erf((x - mu) / (sigma * math.sqrt(2))) +
                           math.erf((x + mu) / (sigma * math.sqrt(2))))
    lo, hi = 0.0, abs(mu) + 20.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if cdf(mid) < q else (lo, mid)
    return hi


def _cabs(z):
    return z if np.real(z) >= 0 else -z


def _cmin1(z):
    return z if np.real(z) < 1.0 else 1.0 + 0.0 * z


def esjd(ff, x0s, mass, mu_dt, mu_L, xi_v, xi_dt, kT, sigma_dt_rel=0.01, sigma_L=1.0,
         sets=None):
    """(L_HMC, recorded interaction sets [R][L_q + 1], L_q). mass: per-atom
    masses (may be complex); mu_dt, mu_L: scalars (may be complex)."""
    s = ff.sys
    c = float(s.accel)
    p0 = ff.params0()
    m = np.asarray(mass)
    L_q = int(math.ceil(folded_normal_quantile(float(np.real(mu_L)), sigma_L)))
    record = sets is None
    out_sets = []
    total = 0.0
    for i, x0 in enumerate(x0s):
        x0 = np.asarray(x0, np.float64)
        v = np.sqrt(kT * c / m)[None, :] * xi_v[i]
        dt = _cabs(mu_dt * (1.0 + sigma_dt_rel * xi_dt[i]))
        sets_i = [] if record else sets[i]
        if record:
            sets_i.append(ff.interacting_pairs(x0))
        U, F = ff(x0, p0, sets_i[0])
        E0 = U + 0.5 * (m[None, :] * v * v).sum() / c
        x = x0 + 0.0 * dt
        for ell in range(1, L_q + 1):
            v = v + 0.5 * dt * c * F / m[None, :]
            x = x + dt * v
            if record:
                sets_i.append(ff.interacting_pairs(x))
            U, F = ff(x, p0, sets_i[ell])
            v = v + 0.5 * dt * c * F / m[None, :]
            E = U + 0.5 * (m[None, :] * v * v).sum() / c
            alpha = _cmin1(np.exp(-(E - E0) / kT))
            jump = ((x - x0) ** 2).sum()
            total = total + folded_normal_pdf(ell, mu_L, sigma_L) * alpha / ell * jump
        out_sets.append(sets_i)
    return total / len(x0s), out_sets, L_q


def gradients(ff, x0s, mass, mu_dt, mu_L, xi_v, xi_dt, kT, mass_dir, **kw):
    """L_HMC and its derivatives with respect to mu_dt, mu_L and the masses
    along mass_dir, by complex steps over the frozen interaction sets."""
    L, sets, L_q = esjd(ff, x0s, mass, mu_dt, mu_L, xi_v, xi_dt, kT, **kw)
    d_dt = np.imag(esjd(ff, x0s, mass, mu_dt + 1j * H_CS, mu_L, xi_v, xi_dt, kT, sets=sets,
                        **kw)[0]) / H_CS
    d_L = np.imag(esjd(ff, x0s, mass, mu_dt, mu_L + 1j * H_CS, xi_v, xi_dt, kT, sets=sets,
                       **kw)[0]) / H_CS
    d_m = np.imag(esjd(ff, x0s, np.asarray(mass) + 1j * H_CS * np.asarray(mass_dir), mu_dt,
                       mu_L, xi_v, xi_dt, kT, sets=sets, **kw)[0]) / H_CS
    return dict(loss=float(np.real(L)), mu_dt=d_dt, mu_L=d_L, mass_dir=d_m, L_q=L_q, sets=sets)
