"""Pins for the oracle's Ewald and smooth-PME reciprocal space (Sec. II.A.2,
Eqs. 9-14 and the PME paragraph)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import bspline, ewald, forcefield, nonbonded, pme

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bspline_golden_values_and_closed_form():
    g = json.load(open(os.path.join(GOLD, "bspline_m4.json")))
    assert np.allclose(bspline.M(4, np.array(g["integer_points"], float)), g["values"],
                       rtol=0, atol=1e-15)
    w = np.linspace(0.0, 3.999, 400)
    k = np.floor(w).astype(int)
    c = np.array(g["piecewise_coefficients_times_6"], float)[k]
    closed = (c[:, 0] + c[:, 1] * w + c[:, 2] * w ** 2 + c[:, 3] * w ** 3) / 6.0
    assert np.allclose(bspline.M(4, w), closed, atol=1e-14)


def test_bspline_partition_of_unity_symmetry_derivative():
    f = np.linspace(0.0, 1.0, 37)
    t = np.arange(4)
    Ms = bspline.M(4, f[:, None] + t[None, :])
    assert np.allclose(Ms.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(bspline.dM(4, f[:, None] + t[None, :]).sum(axis=1), 0.0, atol=1e-13)
    w = np.linspace(0, 4, 101)
    assert np.allclose(bspline.M(4, w), bspline.M(4, 4 - w), atol=1e-14)
    h = 1e-6
    w = np.linspace(0.05, 3.95, 50)
    fd = (bspline.M(4, w + h) - bspline.M(4, w - h)) / (2 * h)
    assert np.allclose(bspline.dM(4, w), fd, atol=1e-8)


def _nacl(a=5.64, nrep=1):
    na = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cl = na + np.array([0.5, 0, 0])
    frac = np.concatenate([na, cl]) % 1.0
    q = np.array([1.0] * 4 + [-1.0] * 4)
    box = np.array([a, a, a])
    return (frac * a).T + 0.01, q, box   # small shift keeps atoms off exact grid points


def test_madelung_constant_by_ewald():
    g = json.load(open(os.path.join(GOLD, "madelung_nacl.json")))
    pos, q, box = _nacl()
    a = box[0]
    expect = -4.0 * g["madelung"] / (a / 2)
    for alpha in (0.6, 0.9):
        Er, _ = ewald.real_images(pos, q, box, alpha, 1.0, r_max=8.0 / alpha)
        Ek, _ = ewald.reciprocal_direct(pos, q, box, alpha, 1.0, n_max=int(3 * alpha * a) + 3)
        Es = ewald.self_term(q, alpha, 1.0)
        assert Er + Ek + Es == pytest.approx(expect, rel=1e-10)


def test_ewald_total_is_alpha_invariant_and_forces_agree():
    s = synth.random_box(24, [7.0, 7.5, 8.0], 3.0, 0.1, 41, min_dist=1.0)
    pos, q, box = s.pos.astype(np.float64), s.charge.astype(np.float64), s.box.astype(np.float64)
    tot, forces = [], []
    for alpha in (0.5, 0.7, 0.9):
        Er, Fr = ewald.real_images(pos, q, box, alpha, 1.0, r_max=7.0 / alpha)
        Ek, Fk = ewald.reciprocal_direct(pos, q, box, alpha, 1.0, n_max=int(2.5 * alpha * 8) + 3)
        tot.append(Er + Ek + ewald.self_term(q, alpha, 1.0))
        forces.append(Fr + Fk)
    assert max(tot) - min(tot) < 1e-10 * abs(tot[0])
    for F in forces[1:]:
        assert np.abs(F - forces[0]).max() < 1e-9 * np.abs(forces[0]).max()


def test_reciprocal_direct_forces_fd():
    s = synth.random_box(12, [6.0, 6.0, 6.0], 2.5, 0.1, 43, min_dist=1.0)
    pos, q, box = s.pos.astype(np.float64), s.charge.astype(np.float64), s.box.astype(np.float64)
    E0, F = ewald.reciprocal_direct(pos, q, box, 0.8, 1.0, 8)
    h = 1e-6
    for a, i in [(0, 0), (1, 3), (2, 7)]:
        pp = pos.copy(); pp[a, i] += h
        pm = pos.copy(); pm[a, i] -= h
        fd = -(ewald.reciprocal_direct(pp, q, box, 0.8, 1.0, 8)[0]
               - ewald.reciprocal_direct(pm, q, box, 0.8, 1.0, 8)[0]) / (2 * h)
        assert fd == pytest.approx(F[a, i], rel=1e-6, abs=1e-9)


def test_spme_converges_to_ewald():
    # order-4 splines: energy error ~ h^4, force error (differentiated splines) at least ~ h^3
    s = synth.random_box(40, [8.0, 8.0, 8.0], 3.0, 0.1, 47, min_dist=1.0)
    pos, q, box = s.pos.astype(np.float64), s.charge.astype(np.float64), s.box.astype(np.float64)
    alpha = 0.7
    Ek, Fk = ewald.reciprocal_direct(pos, q, box, alpha, 1.0, n_max=14)
    ferr, eerr = [], []
    for K in (12, 24, 48):
        r = pme.spme(pos, q, box, (K, K, K), alpha, 1.0)
        ferr.append(np.linalg.norm(r["F"] - Fk) / np.linalg.norm(Fk))
        eerr.append(abs(r["E"] - Ek) / abs(Ek))
    assert ferr[2] < 1e-4 and eerr[2] < 1e-5
    assert eerr[0] / eerr[1] > 12.0 and eerr[1] / eerr[2] > 12.0
    assert ferr[0] / ferr[1] > 7.0 and ferr[1] / ferr[2] > 7.0


def test_spme_energy_spectral_equals_real_space_and_fd():
    s = synth.config_system("water375")
    a = forcefield.alpha(s)
    pos = s.pos.astype(np.float64)
    r = pme.spme(pos, s.charge, s.box, s.pme_grid, a, s.coulomb_k)
    assert 0.5 * s.coulomb_k * float((r["Q"] * r["phi"]).sum()) == pytest.approx(r["E"], rel=1e-11)
    h = 1e-5
    for ax, i in [(0, 0), (1, 1), (2, 2), (0, 200)]:
        pp = pos.copy(); pp[ax, i] += h
        pm = pos.copy(); pm[ax, i] -= h
        fd = -(pme.spme(pp, s.charge, s.box, s.pme_grid, a, s.coulomb_k)["E"]
               - pme.spme(pm, s.charge, s.box, s.pme_grid, a, s.coulomb_k)["E"]) / (2 * h)
        assert fd == pytest.approx(r["F"][ax, i], rel=1e-6, abs=1e-6)


def test_spme_virial_trace():
    s = synth.config_system("water375")
    a = forcefield.alpha(s)
    pos = s.pos.astype(np.float64)
    box = s.box.astype(np.float64)
    W = pme.spme(pos, s.charge, box, s.pme_grid, a, s.coulomb_k)["W"]
    h = 1e-5
    Ep = pme.spme(pos * (1 + h), s.charge, box * (1 + h), s.pme_grid, a, s.coulomb_k)["E"]
    Em = pme.spme(pos * (1 - h), s.charge, box * (1 - h), s.pme_grid, a, s.coulomb_k)["E"]
    assert np.trace(W) == pytest.approx(-(Ep - Em) / (2 * h), rel=1e-8)


def test_spme_water_matches_direct_ewald_within_tolerance():
    # delta = 5e-4 with the mesh heuristic n = 2 alpha d / (3 delta^(1/5)): the reciprocal
    # error relative to the total nonbonded force stays within a few delta
    s = synth.config_system("water375")
    a = forcefield.alpha(s)
    n_mesh = int(math.ceil(2 * a * float(s.box[0]) / (3 * 5e-4 ** 0.2)))
    pos = s.pos.astype(np.float64)
    Ek, Fk = ewald.reciprocal_direct(pos, s.charge, s.box, a, s.coulomb_k, n_max=12)
    r = pme.spme(pos, s.charge, s.box, (n_mesh,) * 3, a, s.coulomb_k)
    Fsr = forcefield.nonbonded_terms(s)["F"]
    assert np.linalg.norm(r["F"] - Fk) / np.linalg.norm(Fk + Fsr) < 4 * 5e-4
    assert abs(r["E"] - Ek) / abs(Ek) < 10 * 5e-4
    # the net reciprocal force is not zero for SPME but is small
    assert np.linalg.norm(r["F"].sum(axis=1)) < 0.05 * np.abs(r["F"]).max()


def test_excluded_molecule_reciprocal_cancels_erf_terms():
    # One neutral, fully excluded water molecule: E_rec + E_self + E_excl -> 0 as the box
    # grows (only the O(1/L^3) dipole remainder survives).
    r0, th0 = 0.9572, math.radians(104.52)
    q = np.array([-0.834, 0.417, 0.417])
    ex = np.array([[0, 1], [0, 2], [1, 2]])
    res = []
    for L in (10.0, 20.0, 40.0):
        O = np.array([L / 2 + 0.1, L / 2 + 0.2, L / 2 + 0.3])
        H1 = O + r0 * np.array([math.sin(th0 / 2), 0.0, math.cos(th0 / 2)])
        H2 = O + r0 * np.array([-math.sin(th0 / 2), 0.0, math.cos(th0 / 2)])
        pos = np.stack([O, H1, H2], axis=1)
        box = np.array([L, L, L])
        alpha = 0.45
        Ek, _ = ewald.reciprocal_direct(pos, q, box, alpha, 1.0, n_max=int(2.2 * alpha * L) + 2)
        Ex = nonbonded.exclusion_correction(pos, box, ex, q, alpha, 1.0)["E"]
        res.append(abs(Ek + Ex + ewald.self_term(q, alpha, 1.0)))
    assert res[1] < res[0] / 6 and res[2] < res[1] / 6
    assert res[2] < 1e-4


def test_kc_root_satisfies_eq14():
    kc = ewald.kc_from_tolerance(5e-4, 0.292029, 44.8)
    d, a = 44.8, 0.292029
    val = kc * math.sqrt(d * a) / 20 * math.exp(-(math.pi * kc / (d * a)) ** 2)
    assert val == pytest.approx(5e-4, rel=1e-9)
    assert kc > d * a / (math.pi * math.sqrt(2))


def test_spme_virial_diagonal_per_axis():
    # W_aa = -dE_rec/d(eps_a): box length and coordinates along a scaled by
    # 1 + eps_a (the grid counts stay, as for a box deformation)
    s = synth.config_system("water375")
    a = forcefield.alpha(s)
    pos = s.pos.astype(np.float64)
    box = s.box.astype(np.float64)
    W = pme.spme(pos, s.charge, box, s.pme_grid, a, s.coulomb_k)["W"]
    h = 1e-5
    for ax in range(3):
        sc = np.ones(3)
        sc[ax] = 1 + h
        Ep = pme.spme(pos * sc[:, None], s.charge, box * sc, s.pme_grid, a, s.coulomb_k)["E"]
        sc[ax] = 1 - h
        Em = pme.spme(pos * sc[:, None], s.charge, box * sc, s.pme_grid, a, s.coulomb_k)["E"]
        assert W[ax, ax] == pytest.approx(-(Ep - Em) / (2 * h), rel=1e-7, abs=1e-8 * abs(W).max())
    assert np.allclose(W, W.T, rtol=0, atol=1e-12 * np.abs(W).max())


def test_self_energy_madelung_and_net_charge_alpha_invariance():
    """nonbonded.self_energy (Eq. 12 plus the neutralising background for a
    net charge Q): the NaCl Madelung energy through it, and the Ewald total of a
    net-charged box independent of alpha (the remark after Eq. 12) only with the
    background term -pi Q^2 / (2 V alpha^2)."""
    g = json.load(open(os.path.join(GOLD, "madelung_nacl.json")))
    pos, q, box = _nacl()
    a = box[0]
    alpha = 0.8
    Er, _ = ewald.real_images(pos, q, box, alpha, 1.0, r_max=8.0 / alpha)
    Ek, _ = ewald.reciprocal_direct(pos, q, box, alpha, 1.0, n_max=int(3 * alpha * a) + 3)
    Es = nonbonded.self_energy(q, box, alpha, 1.0)
    assert Er + Ek + Es == pytest.approx(-4.0 * g["madelung"] / (a / 2), rel=1e-10)

    rng = np.random.default_rng(7)
    box = np.array([6.0, 6.5, 7.0])
    pos = rng.uniform(0.0, 1.0, (3, 5)) * box[:, None]
    q = np.array([1.0, -0.4, 0.9, 0.5, -0.7])          # Q = +1.3
    k_e = 332.0637
    tot, tot_without_net = [], []
    for alpha in (0.5, 0.7, 0.9):
        Er, _ = ewald.real_images(pos, q, box, alpha, k_e, r_max=8.0 / alpha)
        Ek, _ = ewald.reciprocal_direct(pos, q, box, alpha, k_e,
                                        n_max=int(3 * alpha * box.max()) + 3)
        Es = nonbonded.self_energy(q, box, alpha, k_e)
        tot.append(Er + Ek + Es)
        tot_without_net.append(Er + Ek + ewald.self_term(q, alpha, k_e))
    assert max(tot) - min(tot) < 1e-10 * abs(tot[0])
    # the background term is what removes the alpha dependence here
    assert max(tot_without_net) - min(tot_without_net) > 1e-2 * abs(tot[0])
