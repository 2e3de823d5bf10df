"""Pins for the counter-based generator and the Langevin (BAOAB) oracle."""
import numpy as np
import pytest

from oracle import integrate, rng


@pytest.mark.parametrize("ctr,key", [(0, (0, 0)), (5, (123, 456)),
                                     (2 ** 63, (2 ** 64 - 1, 77))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox is the same Philox4x64-10; it advances the counter
    # before drawing, so its first block is ours at counter + 1
    bg = np.random.Philox(counter=np.array([ctr, 0, 0, 0], np.uint64),
                          key=np.array(key, np.uint64))
    ref = [int(v) for v in bg.random_raw(4)]
    assert rng.philox4x64_10([ctr + 1, 0, 0, 0], key) == ref


def test_vectorised_blocks_match_scalar_reference():
    atoms = np.array([0, 1, 7, 12345, 2 ** 31])
    seed = (99 << 64) | 31337
    got = rng.philox_blocks(atoms, 42, seed)
    for k, a in enumerate(atoms):
        assert [int(v) for v in got[:, k]] == rng.philox4x64_10([a, 42, 0, 0], (31337, 99))


def test_normals_are_standard():
    z = rng.normals3(np.arange(100000), 3, 2024)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    # distinct steps and seeds give different streams
    assert not np.array_equal(z, rng.normals3(np.arange(100000), 4, 2024))
    assert not np.array_equal(z, rng.normals3(np.arange(100000), 3, 2025))


def _harmonic(k):
    return lambda x: -k * (x - 50.0)


def test_zero_friction_is_velocity_verlet():
    r = np.random.default_rng(0)
    x0 = 50.0 + r.normal(0, 1, (3, 50))
    v0 = r.normal(0, 1, (3, 50))
    m = r.uniform(1, 2, 50)
    box = np.array([100.0, 100.0, 100.0])
    a = integrate.langevin_baoab(x0, v0, m, box, _harmonic(1.0), 0.05, 200, 1.0, 1.0, 0.0, 7)
    b = integrate.velocity_verlet(x0, v0, m, box, _harmonic(1.0), 0.05, 200, 1.0)
    assert np.abs(a["pos"] - b["pos"]).max() < 1e-10
    assert np.abs(a["vel"] - b["vel"]).max() < 1e-10


def test_free_particles_relax_to_maxwell_boltzmann():
    n, kT, m = 20000, 2.5, 3.0
    x0 = np.full((3, n), 50.0)
    v0 = np.zeros((3, n))
    r = integrate.langevin_baoab(x0, v0, np.full(n, m), np.array([100.0] * 3),
                                 lambda x: np.zeros_like(x), 0.1, 30, 1.0, kT, 2.0, 11)
    assert abs(r["vel"].var() / (kT / m) - 1.0) < 0.02
    assert abs(r["vel"].mean()) < 0.01 * np.sqrt(kT / m)


def test_harmonic_configurational_variance_is_exact():
    # BAOAB samples a harmonic oscillator's positions without time-step bias
    # (variance kT/k for any stable dt; the ABOBA ordering would be off by
    # 1/(1 - (w dt)^2/4) = 1.19 at w dt = 0.8)
    n, kT, k, m = 20000, 1.0, 4.0, 1.0
    dt = 0.8 / np.sqrt(k / m)
    x0 = np.full((3, n), 50.0)
    v0 = np.zeros((3, n))
    r = integrate.langevin_baoab(x0, v0, np.full(n, m), np.array([100.0] * 3), _harmonic(k),
                                 dt, 60, 1.0, kT, 1.5, 5)
    assert abs((r["pos"] - 50.0).var() / (kT / k) - 1.0) < 0.02
