"""Pins for the rigid-water constraint oracle (SHAKE positions, RATTLE
velocities, the constrained velocity-Verlet step)."""
import math

import numpy as np
import pytest

import synth
from oracle import constraints, forcefield

W = synth.systems.WATER
D_OH = W["bond_r0"]
D_HH = 2.0 * D_OH * math.sin(math.radians(W["angle_theta0_deg"]) / 2.0)


def _water(name="water375"):
    s = synth.config_system(name)
    mols = np.arange(s.n_atoms).reshape(-1, 3)      # O, H, H per molecule
    return s, mols


def _dists(x, box, mols):
    L = np.asarray(box, np.float64)[:, None]
    out = []
    for a, b in constraints._pairs(mols):
        d = x[:, a] - x[:, b]
        d -= L * np.round(d / L)
        out.append(np.sqrt((d * d).sum(axis=0)))
    return out


def test_shake_restores_the_geometry_and_conserves_momentum():
    s, mols = _water()
    x = s.pos.astype(np.float64)
    x, _ = constraints.shake(x, x, s.mass, s.box, mols, D_OH, D_HH)   # exact geometry
    rng = np.random.default_rng(1)
    v = rng.normal(0.0, 0.02, x.shape)
    y = x + v                                     # one unconstrained drift
    y2, iters = constraints.shake(x, y, s.mass, s.box, mols, D_OH, D_HH)
    doh1, doh2, dhh = _dists(y2, s.box, mols)
    assert np.abs(doh1 / D_OH - 1).max() < 1e-11 and np.abs(doh2 / D_OH - 1).max() < 1e-11
    assert np.abs(dhh / D_HH - 1).max() < 1e-11
    m = s.mass.astype(np.float64)
    p0 = (m * (y - x)).sum(axis=1)
    p1 = (m * (y2 - x)).sum(axis=1)
    assert np.abs(p1 - p0).max() < 1e-12 * np.abs(m * (y - x)).sum()
    # a molecule that already satisfies the constraints is left as it is
    y3, _ = constraints.shake(x, x + 0.0, s.mass, s.box, mols, D_OH, D_HH)
    assert np.abs(y3 - x).max() < 1e-13


def test_rattle_removes_bond_parallel_velocities_only():
    s, mols = _water()
    x, _ = constraints.shake(s.pos, s.pos.astype(np.float64), s.mass, s.box, mols, D_OH, D_HH)
    rng = np.random.default_rng(2)
    v = rng.normal(0.0, 1.0, x.shape)
    v2 = constraints.rattle_velocities(x, v, s.mass, s.box, mols)
    L = s.box.astype(np.float64)[:, None]
    for a, b in constraints._pairs(mols):
        r = x[:, a] - x[:, b]
        r -= L * np.round(r / L)
        rel = (r * (v2[:, a] - v2[:, b])).sum(axis=0)
        assert np.abs(rel).max() < 1e-12
    m = s.mass.astype(np.float64)
    assert np.abs((m * v2).sum(axis=1) - (m * v).sum(axis=1)).max() < 1e-10
    ke = lambda u: 0.5 * float((m * u * u).sum())
    assert ke(v2) <= ke(v)                        # a projection removes energy
    # projecting twice changes nothing
    assert np.abs(constraints.rattle_velocities(x, v2, s.mass, s.box, mols) - v2).max() < 1e-12


def test_free_rigid_molecule_keeps_energy_and_angular_momentum():
    m = np.array([W["m_O"], W["m_H"], W["m_H"]])
    th = math.radians(W["angle_theta0_deg"]) / 2.0
    x = np.array([[0.0, D_OH * math.sin(th), -D_OH * math.sin(th)],
                  [0.0, D_OH * math.cos(th), D_OH * math.cos(th)],
                  [0.0, 0.0, 0.0]]) + 10.0
    rng = np.random.default_rng(3)
    v = rng.normal(0.0, 0.01, (3, 3))
    box = np.array([40.0, 40.0, 40.0])
    mols = np.array([[0, 1, 2]])
    zero = lambda p: np.zeros_like(p)
    r = constraints.velocity_verlet_rattle(x, v, m, box, zero, 0.5, 4000, 1.0, mols, D_OH, D_HH)
    v0 = constraints.rattle_velocities(x, v, m, box, mols)
    ke = lambda u: 0.5 * float((m * u * u).sum())
    com = lambda p: (m * p).sum(axis=1) / m.sum()

    def ang(p, u):
        c = com(p)
        return sum(m[k] * np.cross(p[:, k] - c, u[:, k]) for k in range(3))
    assert abs(ke(r["vel"]) / ke(v0) - 1.0) < 1e-6
    assert np.abs(ang(r["pos"], r["vel"]) - ang(x, v0)).max() < 1e-9 * np.abs(ang(x, v0)).max()
    for d, ref in zip(_dists(r["pos"], box, mols), (D_OH, D_OH, D_HH)):
        assert abs(float(d[0]) / ref - 1.0) < 1e-11


def test_rigid_water_conserves_energy_at_two_femtoseconds():
    # intermolecular LJ + reaction field, rigid molecules (no bond or angle
    # terms), dt = 2 fs: the total energy stays within 2 % of the kinetic
    s, mols = _water()
    s.bond_k[:] = 0.0
    s.angle_k[:] = 0.0
    s.rf_epsilon, s.ewald_delta, s.pme_grid = math.inf, 0.0, (0, 0, 0)
    x, _ = constraints.shake(s.pos, s.pos.astype(np.float64), s.mass, s.box, mols, D_OH, D_HH)
    E = lambda p: forcefield.total_forces_fp64(s, p)
    F = lambda p: E(p)[1]
    n_steps, dt = 60, 2.0
    r = constraints.velocity_verlet_rattle(x, s.vel, s.mass, s.box, F, dt, n_steps,
                                           float(s.accel), mols, D_OH, D_HH)
    m = s.mass.astype(np.float64)
    acc = float(s.accel)
    v0 = constraints.rattle_velocities(x, s.vel, s.mass, s.box, mols)
    e0 = E(x)[0] + 0.5 * float((m * v0 * v0).sum()) / acc
    ke1 = 0.5 * float((m * r["vel"] ** 2).sum()) / acc
    e1 = E(r["pos"])[0] + ke1
    assert abs(e1 - e0) < 0.02 * ke1, (e0, e1, ke1)


@pytest.mark.parametrize("scale", [0.01, 0.1])
def test_settle_closed_form_equals_converged_shake(scale):
    # SETTLE and SHAKE solve the same equations (displacements along the old
    # bond vectors); the closed form must land on SHAKE's fixed point, keep
    # the centre of mass, move atoms only within the old plane, and satisfy
    # the constraints to rounding
    s, mols = _water()
    x = s.pos.astype(np.float64)
    x, _ = constraints.shake(x, x, s.mass, s.box, mols, D_OH, D_HH)
    y = x + np.random.default_rng(7).normal(0.0, scale, x.shape)
    ys, _ = constraints.shake(x, y, s.mass, s.box, mols, D_OH, D_HH)
    yt = constraints.settle(x, y, s.mass, s.box, mols, D_OH, D_HH)
    assert np.abs(yt - ys).max() < 1e-10
    doh1, doh2, dhh = _dists(yt, s.box, mols)
    for d, ref in ((doh1, D_OH), (doh2, D_OH), (dhh, D_HH)):
        assert np.abs(d / ref - 1).max() < 1e-13
    m = s.mass.astype(np.float64)
    a, b, c = mols[:, 0], mols[:, 1], mols[:, 2]
    com = lambda z: m[a] * z[:, a] + m[b] * z[:, b] + m[c] * z[:, c]
    assert np.abs(com(yt) - com(y)).max() < 1e-12 * np.abs(com(y)).max()
    L = s.box.astype(np.float64)[:, None]
    mi = lambda d: d - L * np.round(d / L)
    nrm = np.cross(mi(x[:, b] - x[:, a]).T, mi(x[:, c] - x[:, a]).T).T
    for k in (a, b, c):
        assert np.abs((nrm * (yt[:, k] - y[:, k])).sum(axis=0)).max() < 1e-12
