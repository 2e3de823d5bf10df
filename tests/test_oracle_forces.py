"""Pins for the oracle's short-range and bonded terms (Sec. II.A.1-2)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import bonded, ewald, forcefield, neighbors, nonbonded

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _two_atoms(r, sig=(1.0, 1.0), eps=(1.0, 1.0), q=(0.0, 0.0), L=20.0):
    box = np.array([L, L, L])
    pos = np.array([[5.0, 5.0 + r], [5.0, 5.0], [5.0, 5.0]])
    return box, pos, np.array([0, 1]), np.array(sig), np.array(eps), np.array(q)


def test_lj_closed_form_minimum_and_zero():
    rmin = 2.0 ** (1 / 6)
    box, pos, t, sig, eps, q = _two_atoms(rmin)
    p = nonbonded.pair_terms(pos, box, np.array([[0, 1]]), t, sig, eps, q, 0.0, 0.0)
    assert p["E_lj"] == pytest.approx(-1.0, rel=1e-13)
    assert np.abs(p["F"]).max() < 1e-12
    box, pos, *_ = _two_atoms(1.0)
    p = nonbonded.pair_terms(pos, box, np.array([[0, 1]]), t, sig, eps, q, 0.0, 0.0)
    assert abs(p["E_lj"]) < 1e-14


def test_lorentz_berthelot_mixing():
    # sigma_ij = (s_i + s_j)/2, eps_ij = sqrt(e_i e_j): minimum at 2^(1/6) sigma_ij, depth eps_ij
    sig, eps = (1.0, 2.0), (0.25, 4.0)
    rmin = 2.0 ** (1 / 6) * 1.5
    box, pos, t, s_, e_, q = _two_atoms(rmin, sig, eps)
    p = nonbonded.pair_terms(pos, box, np.array([[0, 1]]), t, s_, e_, q, 0.0, 0.0)
    assert p["E_lj"] == pytest.approx(-1.0, rel=1e-13)
    assert np.abs(p["F"]).max() < 1e-12


def test_real_space_plus_excluded_erf_is_plain_coulomb():
    # erfc + erf = 1: the listed real-space term minus the exclusion correction
    # of the same pair reproduces the plain Coulomb law, Eq. (7)
    r, kq = 2.7, 332.0637
    box, pos, t, sig, eps, q = _two_atoms(r, eps=(0.0, 0.0), q=(0.8, -0.6))
    for alpha in (0.1, 0.3, 0.9):
        p = nonbonded.pair_terms(pos, box, np.array([[0, 1]]), t, sig, eps, q, alpha, kq)
        e = nonbonded.exclusion_correction(pos, box, np.array([[0, 1]]), q, alpha, kq)
        assert p["E_dir"] - e["E"] == pytest.approx(kq * 0.8 * -0.6 / r, rel=1e-13)
        fx = p["F"][0, 1] - e["F"][0, 1]
        assert fx == pytest.approx(kq * 0.8 * -0.6 / r ** 2, rel=1e-12)
    # alpha -> 0 leaves only the bare Coulomb term in real space
    p = nonbonded.pair_terms(pos, box, np.array([[0, 1]]), t, sig, eps, q, 1e-9, kq)
    assert p["E_dir"] == pytest.approx(kq * 0.8 * -0.6 / r, rel=1e-8)


def _fd_check(energy_fn, pos, force, idx, h=1e-5, rtol=1e-6):
    for a, i in idx:
        pp = pos.copy(); pp[a, i] += h
        pm = pos.copy(); pm[a, i] -= h
        fd = -(energy_fn(pp) - energy_fn(pm)) / (2 * h)
        assert fd == pytest.approx(force[a, i], rel=rtol, abs=1e-7 * max(1.0, abs(fd)))


def test_pair_forces_are_negative_gradient_and_sum_to_zero():
    s = synth.random_box(120, [6.0, 6.5, 7.0], 2.4, 0.3, 21, min_dist=0.7)
    s.switch_r = np.float32(2.0)
    pos = s.pos.astype(np.float64)
    pairs = neighbors.brute_force_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    inter = pairs[neighbors.interacting(s.pos, s.box, s.r_cut, s.r_ghost, pairs)]
    alpha = 0.9

    def terms(p):
        return nonbonded.pair_terms(p, s.box, inter, s.atom_type, s.type_sigma, s.type_epsilon,
                                    s.charge, alpha, 1.0, r_cut=float(s.r_cut),
                                    switch_r=float(s.switch_r))
    base = terms(pos)
    E = lambda p: (lambda d: d["E_lj"] + d["E_dir"])(terms(p))
    rng = np.random.default_rng(3)
    idx = [(int(rng.integers(3)), int(rng.integers(s.n_atoms))) for _ in range(12)]
    _fd_check(E, pos, base["F"], idx)
    assert np.abs(base["F"].sum(axis=1)).max() < 1e-9 * np.abs(base["F"]).max()


def test_switch_function_shape():
    r = np.array([0.5, 1.0, 1.5, 2.0, 2.5])
    S, dS = nonbonded.switch(r, 1.0, 2.0)
    assert S[0] == 1.0 and S[1] == 1.0 and S[3] == 0.0 and S[4] == 0.0
    assert S[2] == pytest.approx(0.5)
    eps = 1e-6
    for x0 in (1.0, 2.0):  # C1 at both ends: derivative vanishes
        Sp, _ = nonbonded.switch(np.array([x0 + eps, x0 - eps]), 1.0, 2.0)
        assert abs(Sp[0] - Sp[1]) / (2 * eps) < 1e-4


def test_exclusion_correction_gradient():
    s = synth.config_system("water375")
    pos = s.pos.astype(np.float64)
    a = forcefield.alpha(s)
    f = nonbonded.exclusion_correction(pos, s.box, s.exclusions, s.charge, a, s.coulomb_k)
    E = lambda p: nonbonded.exclusion_correction(p, s.box, s.exclusions, s.charge, a,
                                                 s.coulomb_k)["E"]
    _fd_check(E, pos, f["F"], [(0, 0), (1, 1), (2, 2), (0, 5), (2, 301)])
    assert np.abs(f["F"].sum(axis=1)).max() < 1e-9


def test_bonded_equilibrium_and_closed_forms():
    box = np.array([30.0, 30.0, 30.0])
    r0, th0 = 0.9572, math.radians(104.52)
    O = np.array([10.0, 10.0, 10.0])
    H1 = O + r0 * np.array([math.sin(th0 / 2), 0.0, math.cos(th0 / 2)])
    H2 = O + r0 * np.array([-math.sin(th0 / 2), 0.0, math.cos(th0 / 2)])
    pos = np.stack([O, H1, H2], axis=1)
    b = bonded.bonds(pos, box, [[0, 1], [0, 2]], [450.0, 450.0], [r0, r0])
    an = bonded.angles(pos, box, [[1, 0, 2]], [55.0], [th0])
    assert abs(b["E"]) < 1e-20 and abs(an["E"]) < 1e-20
    assert np.abs(b["F"]).max() < 1e-10 and np.abs(an["F"]).max() < 1e-10
    # stretched bond: E = k dr^2, |F| = 2 k dr
    pos2 = np.stack([O, O + np.array([r0 + 0.1, 0, 0])], axis=1)
    b = bonded.bonds(pos2, box, [[0, 1]], [450.0], [r0])
    assert b["E"] == pytest.approx(450.0 * 0.01, rel=1e-12)
    assert b["F"][0, 1] == pytest.approx(-2 * 450.0 * 0.1, rel=1e-12)
    # right angle: E = k (pi/2 - theta0)^2
    pos3 = np.stack([O, O + np.array([1.0, 0, 0]), O + np.array([0, 1.3, 0])], axis=1)
    an = bonded.angles(pos3, box, [[1, 0, 2]], [55.0], [th0])
    assert an["E"] == pytest.approx(55.0 * (math.pi / 2 - th0) ** 2, rel=1e-12)


def test_bonded_gradient_and_momentum():
    s = synth.config_system("water375")
    rng = np.random.default_rng(9)
    pos = s.pos.astype(np.float64) + rng.normal(0, 0.05, s.pos.shape)
    def E(p):
        return (bonded.bonds(p, s.box, s.bonds, s.bond_k, s.bond_r0)["E"]
                + bonded.angles(p, s.box, s.angles, s.angle_k, s.angle_theta0)["E"])
    F = (bonded.bonds(pos, s.box, s.bonds, s.bond_k, s.bond_r0)["F"]
         + bonded.angles(pos, s.box, s.angles, s.angle_k, s.angle_theta0)["F"])
    _fd_check(E, pos, F, [(0, 0), (1, 1), (2, 2), (0, 4), (1, 200)], h=1e-6, rtol=1e-5)
    assert np.abs(F.sum(axis=1)).max() < 1e-9


def test_virial_trace_is_minus_dU_dlambda():
    s = synth.random_box(100, [6.0, 6.0, 6.0], 2.4, 0.3, 31, min_dist=0.8)
    pos = s.pos.astype(np.float64)
    box = s.box.astype(np.float64)
    pairs = neighbors.brute_force_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    inter = pairs[neighbors.interacting(s.pos, s.box, s.r_cut, s.r_ghost, pairs)]
    alpha = 0.9
    def E(lam):
        d = nonbonded.pair_terms(pos * lam, box * lam, inter, s.atom_type, s.type_sigma,
                                 s.type_epsilon, s.charge, alpha, 1.0)
        return d["E_lj"] + d["E_dir"]
    W = nonbonded.pair_terms(pos, s.box, inter, s.atom_type, s.type_sigma, s.type_epsilon,
                             s.charge, alpha, 1.0)["W"]
    h = 1e-6
    dU = (E(1 + h) - E(1 - h)) / (2 * h)
    assert np.trace(W) == pytest.approx(-dU, rel=1e-7)


def test_alpha_heuristic_golden():
    g = json.load(open(os.path.join(GOLD, "ewald_alpha.json")))
    assert ewald.alpha_from_tolerance(g["delta"], g["r_cut"]) == pytest.approx(g["alpha"], rel=1e-14)


def test_energy_components_water_signs():
    s = synth.config_system("water375")
    nb = forcefield.nonbonded_terms(s)
    E = dict(zip(forcefield.ENERGY_NAMES, nb["E"]))
    assert E["lj"] > 0           # O-O repulsion dominates at liquid density
    assert E["coul_self"] < 0 and E["coul_excl"] > 0
    # rigid equilibrium geometry: bonded energy is rounding noise
    assert abs(E["bond"]) < 1e-6 and abs(E["angle"]) < 1e-6
    assert np.abs(nb["F"].sum(axis=1)).max() < 1e-8 * np.abs(nb["F"]).max()


def _axis_scaled(pos, box, axis, lam):
    s = np.ones(3)
    s[axis] = lam
    return pos * s[:, None], box * s


def _term_energy(d):
    return d["E_lj"] + d["E_dir"] if "E_lj" in d else d["E"]


def _virial_terms(s, inter, alpha, k):
    return {
        "pair": lambda p, b: nonbonded.pair_terms(p, b, inter, s.atom_type, s.type_sigma,
                                                  s.type_epsilon, s.charge, alpha, k),
        "excl": lambda p, b: nonbonded.exclusion_correction(p, b, s.exclusions, s.charge,
                                                            alpha, k),
        "bond": lambda p, b: bonded.bonds(p, b, s.bonds, s.bond_k, s.bond_r0),
        "angle": lambda p, b: bonded.angles(p, b, s.angles, s.angle_k, s.angle_theta0),
    }


def test_virial_diagonal_is_minus_axis_strain_derivative():
    # W_aa = -dU/d(eps_a) when the box and every coordinate along a are
    # scaled by 1 + eps_a (fixed interaction set, water off its equilibrium)
    s = synth.config_system("water375")
    pos = s.pos.astype(np.float64) + np.random.default_rng(5).normal(0.0, 0.03, s.pos.shape)
    box = s.box.astype(np.float64)
    p32 = pos.astype(np.float32)
    pairs = neighbors.brute_force_pairs(p32, s.box, s.r_cut, s.r_ghost, s.exclusions)
    inter = pairs[neighbors.interacting(p32, s.box, s.r_cut, s.r_ghost, pairs)]
    h = 1e-6
    for name, fn in _virial_terms(s, inter, forcefield.alpha(s), float(s.coulomb_k)).items():
        W = fn(pos, box)["W"]
        assert np.abs(W).max() > 0, name
        for ax in range(3):
            ep = _term_energy(fn(*_axis_scaled(pos, box, ax, 1 + h)))
            em = _term_energy(fn(*_axis_scaled(pos, box, ax, 1 - h)))
            fd = -(ep - em) / (2 * h)
            assert W[ax, ax] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(W).max()), (name, ax)


def test_virial_off_diagonal_is_minus_shear_derivative():
    # an isolated cluster (no periodic image within reach): shearing every
    # coordinate r_a += eps r_b gives -dU/d(eps) = W_ba
    rng = np.random.default_rng(8)
    n = 36
    pos = 46.0 + 8.0 * rng.random((3, n))
    box = np.full(3, 100.0)
    s = synth.random_box(n, [100.0, 100.0, 100.0], 20.0, 0.0, 9)
    s.charge = rng.choice([-0.5, 0.5], n).astype(np.float32)
    s.bonds = np.stack([np.arange(0, n - 1, 3), np.arange(1, n, 3)], 1).astype(np.int32)
    s.bond_k = np.full(len(s.bonds), 300.0, np.float32)
    s.bond_r0 = np.full(len(s.bonds), 1.2, np.float32)
    s.angles = np.stack([np.arange(0, n - 2, 3), np.arange(1, n - 1, 3),
                         np.arange(2, n, 3)], 1).astype(np.int32)
    s.angle_k = np.full(len(s.angles), 40.0, np.float32)
    s.angle_theta0 = np.full(len(s.angles), 1.8, np.float32)
    s.exclusions = s.bonds.copy()
    i, j = np.triu_indices(n, 1)
    keep = ~np.isin(i * n + j, s.exclusions[:, 0] * n + s.exclusions[:, 1])
    inter = np.stack([i[keep], j[keep]], 1)
    h = 1e-6
    for name, fn in _virial_terms(s, inter, 0.3, 1.0).items():
        W = fn(pos, box)["W"]
        assert np.abs(W).max() > 0, name
        for a, b in ((0, 1), (0, 2), (1, 2), (1, 0), (2, 0), (2, 1)):
            pp, pm = pos.copy(), pos.copy()
            pp[a] += h * pos[b]
            pm[a] -= h * pos[b]
            fd = -(_term_energy(fn(pp, box)) - _term_energy(fn(pm, box))) / (2 * h)
            assert W[b, a] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(W).max()), (name, a, b)
