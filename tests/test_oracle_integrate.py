"""Pins for the oracle's velocity Verlet (Sec. II.D.1)."""
import math

import numpy as np
import pytest

import synth
from oracle import bonded, forcefield, integrate


def test_harmonic_dimer_matches_closed_form_recurrence():
    # U = k (r - r0)^2 on a 1-D dimer of equal masses m: the bond length obeys a
    # linear oscillator with omega^2 = 4 k c / m. Velocity Verlet on a linear
    # oscillator is exactly x_n = A cos(n w~ dt) with cos(w~ dt) = 1 - (omega dt)^2 / 2.
    k, r0, m, c = 3.0, 1.5, 2.0, 1.0
    box = np.array([50.0, 50.0, 50.0])
    d0 = 0.01
    pos = np.array([[10.0, 10.0 + r0 + d0], [10.0, 10.0], [10.0, 10.0]])
    vel = np.zeros((3, 2))
    F = lambda p: bonded.bonds(p, box, [[0, 1]], [k], [r0])["F"]
    dt, n = 0.05, 200
    out = integrate.velocity_verlet(pos, vel, [m, m], box, F, dt, n, c)
    omega = math.sqrt(4 * k * c / m)
    wt = math.acos(1 - (omega * dt) ** 2 / 2)
    bond = out["traj"][:, 0, 1] - out["traj"][:, 0, 0] - r0
    expect = d0 * np.cos(wt * np.arange(n + 1))
    assert np.abs(bond - expect).max() < 1e-12


def test_time_reversibility_fp64():
    s = synth.lj_fluid(4, 0.8, 0.1, 1.8, 0.2, 1.0, 5)   # 64 atoms, L = 4.31
    F = lambda p: forcefield.total_forces_fp64(s, p)[1]
    out = integrate.velocity_verlet(s.pos, s.vel, s.mass, s.box, F, 0.002, 40, 1.0)
    back = integrate.velocity_verlet(out["pos"], -out["vel"], s.mass, s.box, F, 0.002, 40, 1.0)
    d = back["pos"] - s.pos.astype(np.float64)
    d -= s.box[:, None] * np.round(d / s.box[:, None])
    assert np.abs(d).max() < 1e-10


def test_energy_fluctuation_scales_as_dt_squared():
    s = synth.lj_fluid(4, 0.8, 0.1, 1.8, 0.2, 0.5, 6)
    s.switch_r = np.float32(1.4)        # smooth potential: shadow Hamiltonian holds
    U = lambda p: forcefield.total_forces_fp64(s, p)[0]
    F = lambda p: forcefield.total_forces_fp64(s, p)[1]
    amp = []
    for dt, n in ((0.004, 100), (0.002, 200)):
        e = np.array(integrate.velocity_verlet(s.pos, s.vel, s.mass, s.box, F, dt, n, 1.0,
                                               energy_fn=U)["etot"])
        amp.append(e.std())
    assert 3.0 < amp[0] / amp[1] < 5.0


def test_fp32_emulation_tracks_fp64_briefly():
    s = synth.lj_fluid(4, 0.8, 0.1, 1.8, 0.2, 1.0, 7)
    F = lambda p: forcefield.total_forces_fp64(s, p)[1]
    a = integrate.velocity_verlet(s.pos, s.vel, s.mass, s.box, F, 0.005, 20, 1.0)
    b = integrate.velocity_verlet_f32(s.pos, s.vel, s.mass, s.box, F, 0.005, 20, 1.0)
    d = a["traj"] - b["traj"]
    d -= s.box[None, :, None] * np.round(d / s.box[None, :, None])
    assert np.abs(d).max() < 1e-4
