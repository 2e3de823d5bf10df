"""Pins of the HMC tuning objective's oracle (oracle/hmc.py): its complex-step
derivatives against central differences of the frozen-set objective, the
mu_L derivative against the folded-normal density's own derivative, free
particles in closed form, and the folded-normal quantile."""
import math

import numpy as np

import synth
from oracle import adjoint, hmc


def _setup(name="water375", R=2, seed=5):
    s = synth.config_system(name)
    ff = adjoint.ForceField(s)
    rng = np.random.default_rng(seed)
    xi_v = [rng.standard_normal((3, s.n_atoms)) for _ in range(R)]
    xi_dt = rng.standard_normal(R)
    x0s = [s.pos.astype(np.float64) for _ in range(R)]
    return s, ff, x0s, xi_v, xi_dt


def test_folded_normal_quantile():
    for mu, sig in ((6.0, 1.0), (0.3, 1.0), (40.0, 2.0)):
        x = hmc.folded_normal_quantile(mu, sig)
        cdf = 0.5 * (math.erf((x - mu) / (sig * math.sqrt(2))) + math.erf((x + mu) / (sig * math.sqrt(2))))
        assert abs(cdf - 0.999) < 1e-12
    # far from zero the fold does not matter: mu + 3.0902 sigma
    assert abs(hmc.folded_normal_quantile(40.0, 2.0) - (40.0 + 3.090232306 * 2.0)) < 1e-6


def test_complex_step_derivatives_match_frozen_set_differences():
    s, ff, x0s, xi_v, xi_dt = _setup()
    kT = 0.0019872041 * 300.0
    m = s.mass.astype(np.float64)
    # repartitioning: one unit from O to each of its H (total mass fixed)
    mdir = np.where(s.atom_type == 0, -2.0, 1.0)
    mu_dt, mu_L = 1.0, 5.0
    g = hmc.gradients(ff, x0s, m, mu_dt, mu_L, xi_v, xi_dt, kT, mdir)
    sets = g["sets"]
    f = lambda **kw: float(np.real(hmc.esjd(ff, x0s, kw.get("m", m), kw.get("dt", mu_dt),
                                            kw.get("L", mu_L), xi_v, xi_dt, kT, sets=sets)[0]))
    h = 1e-5
    assert abs(g["mu_dt"] - (f(dt=mu_dt + h) - f(dt=mu_dt - h)) / (2 * h)) <= 1e-6 * abs(g["mu_dt"])
    assert abs(g["mu_L"] - (f(L=mu_L + h) - f(L=mu_L - h)) / (2 * h)) <= 1e-6 * abs(g["mu_L"])
    # masses of ~1-16 amu: the central difference converges as h^2 to the
    # complex step down to a noise floor near 1e-8; Richardson's combination of
    # h and h/2 removes the h^2 term
    c = lambda hh: (f(m=m + hh * mdir) - f(m=m - hh * mdir)) / (2 * hh)
    fd = (4.0 * c(5e-5) - c(1e-4)) / 3.0
    assert abs(g["mass_dir"] - fd) <= 1e-6 * abs(fd)
    assert g["loss"] > 0


def test_mu_L_derivative_is_the_density_derivative():
    # only the weights depend on mu_L: dL/dmu_L = sum dN_F/dmu alpha/l jump
    s, ff, x0s, xi_v, xi_dt = _setup(R=1)
    kT = 0.0019872041 * 300.0
    m = s.mass.astype(np.float64)
    mu_L, sig = 4.0, 1.0
    g = hmc.gradients(ff, x0s, m, 1.0, mu_L, xi_v, xi_dt, kT, np.zeros_like(m))
    # the same objective with the weight replaced by its mu-derivative
    dpdf = lambda x, mu: (1.0 / math.sqrt(2 * math.pi * sig * sig)) * (
        (x - mu) / sig ** 2 * np.exp(-(x - mu) ** 2 / (2 * sig * sig)) -
        (x + mu) / sig ** 2 * np.exp(-(x + mu) ** 2 / (2 * sig * sig)))
    saved = hmc.folded_normal_pdf
    try:
        hmc.folded_normal_pdf = lambda x, mu, sigma: dpdf(x, mu)
        ref = float(np.real(hmc.esjd(ff, x0s, m, 1.0, mu_L, xi_v, xi_dt, kT, sets=g["sets"])[0]))
    finally:
        hmc.folded_normal_pdf = saved
    assert abs(g["mu_L"] - ref) <= 1e-10 * abs(ref)


def test_free_particles_closed_form():
    # no forces: E is conserved (alpha = 1) and x_l - x_0 = l dt v0, so
    # L = (1/R) sum_i sum_l w_l l dt_i^2 sum_a (kT c / m_a) xi^2
    s = synth.random_box(100, [12.0, 12.0, 12.0], 2.0, 0.5, 3, charged=False)
    s.type_epsilon[:] = 0.0
    ff = adjoint.ForceField(s)
    R = 3
    rng = np.random.default_rng(2)
    xi_v = [rng.standard_normal((3, s.n_atoms)) for _ in range(R)]
    xi_dt = rng.standard_normal(R)
    x0s = [s.pos.astype(np.float64)] * R
    m = s.mass.astype(np.float64)
    kT, c = 1.3, float(s.accel)
    mu_dt, mu_L = 0.01, 6.0
    mdir = rng.standard_normal(s.n_atoms)
    g = hmc.gradients(ff, x0s, m, mu_dt, mu_L, xi_v, xi_dt, kT, mdir)
    L_q = g["L_q"]
    ell = np.arange(1, L_q + 1)
    W = (hmc.folded_normal_pdf(ell, mu_L, 1.0) * ell).sum()
    a = np.array([1.0 + 0.01 * z for z in xi_dt])
    S = np.array([(kT * c / m[None, :] * xi * xi).sum() for xi in xi_v])
    L = W * (mu_dt ** 2 * a ** 2 * S).sum() / R
    assert abs(g["loss"] - L) <= 1e-12 * L
    assert abs(g["mu_dt"] - W * (2 * mu_dt * a ** 2 * S).sum() / R) <= 1e-12 * L / mu_dt
    dS = np.array([(-kT * c / m[None, :] ** 2 * xi * xi * mdir[None, :]).sum() for xi in xi_v])
    assert abs(g["mass_dir"] - W * (mu_dt ** 2 * a ** 2 * dS).sum() / R) <= 1e-10 * abs(L)
