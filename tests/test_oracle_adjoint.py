"""Pins of the FP64 adjoint oracle (oracle/adjoint.py): its force field
against the plain oracle, its Hessian-vector and parameter derivatives
against central differences, and the trajectory gradients against
closed forms (free particles, a harmonic dimer under velocity Verlet) and
against central differences of the frozen-interaction-set loss."""
import numpy as np
import pytest

import synth
from oracle import adjoint, forcefield


def _water():
    s = synth.config_system("water375")
    ff = adjoint.ForceField(s)
    return s, ff, ff.params0(), s.pos.astype(np.float64)


def test_force_field_equals_the_plain_oracle():
    s, ff, p, x = _water()
    U, F = ff(x, p, ff.interacting_pairs(x))
    U_ref, F_ref = forcefield.total_forces_fp64(s, x)
    assert abs(U - U_ref) <= 1e-12 * abs(U_ref)
    assert np.linalg.norm(F - F_ref) <= 1e-12 * np.linalg.norm(F_ref)


@pytest.mark.parametrize("term", ["pairs", "exclusions", "bonds", "angles", "pme"])
def test_hessian_vector_product_matches_differences_of_the_force(term):
    s, ff, p, x = _water()
    pairs = ff.interacting_pairs(x)
    if term != "exclusions":
        ff.ex = ff.ex[:0]
    if term != "bonds":
        ff.bonds = ff.bonds[:0]
    if term != "angles":
        ff.angles = ff.angles[:0]
    ff.has_pme = term == "pme"
    if term != "pairs":
        pairs = pairs[:0]
    u = np.random.default_rng(1).standard_normal(x.shape)
    dF = ff.dforce(x, p, pairs, u)
    h = 1e-5
    fd = (ff(x + h * u, p, pairs)[1] - ff(x - h * u, p, pairs)[1]) / (2 * h)
    assert np.linalg.norm(dF - fd) <= 1e-7 * np.linalg.norm(fd)
    # the Hessian is symmetric: w . (H u) = u . (H w)
    w = np.random.default_rng(2).standard_normal(x.shape)
    assert abs((w * dF).sum() - (u * ff.dforce(x, p, pairs, w)).sum()) <= \
        1e-10 * np.abs(w * dF).sum()


def test_parameter_derivatives_match_differences():
    s, ff, p, x = _water()
    pairs = ff.interacting_pairs(x)
    dq = np.where(s.atom_type == 0, 1.0, -0.5)
    got = ff.dparams(x, p, pairs, dq)
    h = 1e-6
    for (name, e), (dU, dF) in zip(ff.param_directions(dq), got):
        if name != "charge" and e[1] == 1.0:
            continue                      # hydrogen type: eps_H = 0
        Up, Fp = ff(x, adjoint.perturb(p, name, e, h), pairs)
        Um, Fm = ff(x, adjoint.perturb(p, name, e, -h), pairs)
        assert abs(dU - (Up - Um) / (2 * h)) <= 1e-7 * max(abs(dU), 1e-3), name
        fd = (Fp - Fm) / (2 * h)
        assert np.linalg.norm(dF - fd) <= 1e-6 * np.linalg.norm(fd), name


def test_trajectory_gradients_match_frozen_set_differences():
    s, ff, p, x = _water()
    v0 = s.vel.astype(np.float64)
    dq = np.where(s.atom_type == 0, 1.0, -0.5)
    dt, T = 1.0, 20
    g = adjoint.gradients(ff, p, x, v0, dt, T, dq)
    sets = g["traj"]["pair_sets"]
    h = 1e-5
    fl = lambda **kw: adjoint.frozen_loss(ff, kw.get("p", p), kw.get("x", x), kw.get("v", v0),
                                          kw.get("dt", dt), T, sets)
    for k, (name, e) in enumerate(ff.param_directions(dq)):
        if name != "charge" and e[1] == 1.0:
            assert name == "sig" or np.isnan(g["theta"][k])
            continue
        fd = (fl(p=adjoint.perturb(p, name, e, h)) - fl(p=adjoint.perturb(p, name, e, -h))) / (2 * h)
        assert abs(g["theta"][k] - fd) <= 1e-6 * abs(fd), (name, g["theta"][k], fd)
    fd = (fl(dt=dt + h) - fl(dt=dt - h)) / (2 * h)
    assert abs(g["dt"] - fd) <= 1e-6 * abs(fd)
    rng = np.random.default_rng(4)
    for _ in range(2):
        w = rng.standard_normal(x.shape)
        fd = (fl(x=x + h * w) - fl(x=x - h * w)) / (2 * h)
        assert abs((g["x0"] * w).sum() - fd) <= 1e-6 * abs(fd)
    w = rng.standard_normal(x.shape)
    fd = (fl(v=v0 + h * w) - fl(v=v0 - h * w)) / (2 * h)
    assert abs((g["v0"] * w).sum() - fd) <= 1e-5 * abs(fd)


def test_free_particles_closed_form():
    # no forces: x_T = x_0 + T dt v_0, L = T^2 dt^2 sum v0^2 / N
    s = synth.random_box(200, [12.0, 12.0, 12.0], 2.0, 0.5, 8, charged=False)
    s.type_epsilon[:] = 0.0
    ff = adjoint.ForceField(s)
    p = ff.params0()
    x, v = s.pos.astype(np.float64), s.vel.astype(np.float64)
    dt, T, n = 0.01, 30, s.n_atoms
    g = adjoint.gradients(ff, p, x, v, dt, T, np.zeros(n))
    assert abs(g["loss"] - T * T * dt * dt * (v * v).sum() / n) <= 1e-12 * g["loss"]
    assert np.abs(g["x0"]).max() <= 1e-14
    ref = 2.0 * T * T * dt * dt * v / n
    assert np.abs(g["v0"] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(g["dt"] - 2.0 * T * T * dt * (v * v).sum() / n) <= 1e-12 * abs(g["dt"])


def _dimer(k=2.0, r0=1.0):
    s = synth.random_box(2, [20.0, 20.0, 20.0], 2.0, 0.5, 5, n_types=1, charged=False,
                         n_excl_per_atom=0)
    s.type_epsilon[:] = 0.0
    s.pos = np.array([[5.0, 6.1], [5.0, 5.0], [5.0, 5.0]], np.float32)
    s.vel = np.array([[0.3, -0.2], [0.0, 0.0], [0.0, 0.0]], np.float32)
    s.mass = np.array([1.0, 3.0], np.float32)
    s.bonds = np.array([[0, 1]], np.int32)
    s.bond_k = np.array([k], np.float32)
    s.bond_r0 = np.array([r0], np.float32)
    s.exclusions = np.array([[0, 1]], np.int32)
    return s


def _dimer_loss_closed_form(s, dt, shift, T):
    """Velocity Verlet of U = k (r - r0)^2 along x written out as the 2 x 2
    linear map of (y, w) = (r - r0, v1 - v0) and free centre-of-mass motion;
    `shift` moves atom 0 along x. Complex-safe in dt and shift."""
    k, r0 = float(s.bond_k[0]), float(s.bond_r0[0])
    m0, m1 = (float(m) for m in s.mass)
    M, mu = m0 + m1, m0 * m1 / (m0 + m1)
    w2 = 2.0 * k / mu
    x0, x1 = float(s.pos[0, 0]) + shift, float(s.pos[0, 1])
    v0, v1 = (float(v) for v in s.vel[0])
    A = np.array([[1.0 - 0.5 * w2 * dt * dt, dt],
                  [-w2 * dt * (1.0 - 0.25 * w2 * dt * dt), 1.0 - 0.5 * w2 * dt * dt]])
    yw = np.linalg.matrix_power(A, T) @ np.array([x1 - x0 - r0, v1 - v0])
    X = (m0 * x0 + m1 * x1) / M + T * dt * (m0 * v0 + m1 * v1) / M
    r = r0 + yw[0]
    xa, xb = X - (m1 / M) * r, X + (m0 / M) * r
    return (k * yw[0] ** 2 + (xa - x0) ** 2 + (xb - x1) ** 2) / 2.0


def test_harmonic_dimer_closed_form():
    s = _dimer()
    ff = adjoint.ForceField(s)
    p = ff.params0()
    dt, T = 0.05, 60
    g = adjoint.gradients(ff, p, s.pos.astype(np.float64), s.vel.astype(np.float64), dt, T,
                          np.zeros(2))
    L = _dimer_loss_closed_form(s, dt, 0.0, T)
    assert abs(g["loss"] - L) <= 1e-12 * abs(L)
    h = 1e-30      # complex step of the closed form
    dL_ddt = np.imag(_dimer_loss_closed_form(s, dt + 1j * h, 0.0, T)) / h
    dL_dx = np.imag(_dimer_loss_closed_form(s, dt, 1j * h, T)) / h
    assert abs(g["dt"] - dL_ddt) <= 1e-10 * abs(dL_ddt), (g["dt"], dL_ddt)
    assert abs(g["x0"][0, 0] - dL_dx) <= 1e-10 * abs(dL_dx), (g["x0"][0, 0], dL_dx)
