"""Velocity Verlet (paper Sec. II.D.1, the listed update steps 1, 2, 4, 5;
constraints, thermostat and measurement steps are empty here).

    v(t + dt/2) = v(t) + (dt/2) a(t)
    x(t + dt)   = x(t) + dt v(t + dt/2)
    a(t + dt)   = c F(x(t + dt)) / m
    v(t + dt)   = v(t + dt/2) + (dt/2) a(t + dt)

c converts force/mass into acceleration (1 in reduced units). Positions are
wrapped back into [0, L) after each drift; with minimum-image forces this
changes nothing physical, and `image` counts the wraps so unwrapped
coordinates are x + image * L.
"""
from __future__ import annotations

import numpy as np


def kinetic_energy(vel, mass, accel):
    v = np.asarray(vel, np.float64)
    m = np.asarray(mass, np.float64)
    return 0.5 * float((m[None, :] * v * v).sum()) / accel


def velocity_verlet(pos, vel, mass, box, force_fn, dt, n_steps, accel,
                    energy_fn=None):
    """float64 trajectory. force_fn(pos) -> F [3,N]; energy_fn(pos) -> U.

    Returns dict(pos, vel, image, traj [n_steps+1,3,N], etot list or None).
    """
    x = np.asarray(pos, np.float64).copy()
    v = np.asarray(vel, np.float64).copy()
    m = np.asarray(mass, np.float64)
    L = np.asarray(box, np.float64)[:, None]
    img = np.zeros(x.shape, np.int64)
    F = force_fn(x)
    traj = [x.copy()]
    etot = [] if energy_fn is not None else None
    if energy_fn is not None:
        etot.append(energy_fn(x) + kinetic_energy(v, m, accel))
    for _ in range(n_steps):
        v = v + 0.5 * dt * accel * F / m[None, :]
        x = x + dt * v
        shift = np.floor(x / L)
        x = x - shift * L
        img += shift.astype(np.int64)
        F = force_fn(x)
        v = v + 0.5 * dt * accel * F / m[None, :]
        traj.append(x.copy())
        if energy_fn is not None:
            etot.append(energy_fn(x) + kinetic_energy(v, m, accel))
    return dict(pos=x, vel=v, image=img, traj=np.array(traj), etot=etot)


def velocity_verlet_f32(pos, vel, mass, box, force_fn, dt, n_steps, accel):
    """Same scheme with float32 state and float32 update arithmetic (forces
    evaluated in float64 and rounded): calibrates how far a float32 run is
    expected to drift from the float64 one."""
    f32 = np.float32
    x = np.asarray(pos, f32).copy()
    v = np.asarray(vel, f32).copy()
    h = (f32(0.5) * f32(dt) * f32(accel) / np.asarray(mass, f32)).astype(f32)
    L = np.asarray(box, f32)[:, None]
    F = force_fn(x.astype(np.float64)).astype(f32)
    traj = [x.astype(np.float64)]
    for _ in range(n_steps):
        v = (v + h[None, :] * F).astype(f32)
        x = (x + f32(dt) * v).astype(f32)
        x = np.where(x >= L, x - L, np.where(x < 0, x + L, x)).astype(f32)
        F = force_fn(x.astype(np.float64)).astype(f32)
        v = (v + h[None, :] * F).astype(f32)
        traj.append(x.astype(np.float64))
    return dict(pos=x, vel=v, traj=np.array(traj))


def langevin_baoab(pos, vel, mass, box, force_fn, dt, n_steps, accel, kT, gamma, seed,
                   step0=0):
    """Langevin dynamics, float64: the paper's adapted splitting read as the
    'middle' scheme (BAOAB):

        v += (dt/2) a;  x += (dt/2) v;
        v  = c1 v + c2 sqrt(kT c / m) xi,   c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2);
        x += (dt/2) v (wrapped);  a = c F(x) / m;  v += (dt/2) a

    with xi three standard normals per atom from rng.normals3(atom, step,
    seed), step = step0, step0 + 1, ... Returns dict(pos, vel, image).
    """
    from . import rng
    x = np.asarray(pos, np.float64).copy()
    v = np.asarray(vel, np.float64).copy()
    m = np.asarray(mass, np.float64)
    L = np.asarray(box, np.float64)[:, None]
    img = np.zeros(x.shape, np.int64)
    n = x.shape[1]
    c1 = float(np.exp(-gamma * dt))
    c2 = float(np.sqrt(1.0 - c1 * c1))
    sig = np.sqrt(kT * accel / m)[None, :]
    F = force_fn(x)
    atoms = np.arange(n)
    for s in range(n_steps):
        v = v + 0.5 * dt * accel * F / m[None, :]
        x = x + 0.5 * dt * v
        v = c1 * v + c2 * sig * rng.normals3(atoms, step0 + s, seed)
        x = x + 0.5 * dt * v
        shift = np.floor(x / L)
        x = x - shift * L
        img += shift.astype(np.int64)
        F = force_fn(x)
        v = v + 0.5 * dt * accel * F / m[None, :]
    return dict(pos=x, vel=v, image=img)
