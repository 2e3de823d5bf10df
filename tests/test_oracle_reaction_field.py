"""Pins for the oracle's reaction-field Coulomb term, Eq. (8), read with the
solvent dielectric eps_s in both constants."""
import math

import numpy as np
import pytest

import synth
from oracle import forcefield, nonbonded

KE = 332.0637132991921   # any positive constant: the pins are relative


def _pair(r, eps_s, r_cut=9.0, q=(0.8, -0.6)):
    box = np.array([40.0, 40.0, 40.0])
    pos = np.array([[5.0, 5.0 + r], [5.0, 5.0], [5.0, 5.0]])
    return nonbonded.pair_terms(pos, box, np.array([[0, 1]]), np.array([0, 0]),
                                np.array([1.0]), np.array([0.0]), np.array(q), 0.0, KE,
                                r_cut=r_cut, rf_epsilon=eps_s)


@pytest.mark.parametrize("eps_s", [1.0, 4.0, 78.5, math.inf])
def test_energy_vanishes_at_the_cutoff(eps_s):
    # the defining property of k_RF, c_RF with eps_s in both: U(r_c) = 0
    p = _pair(9.0, eps_s)
    assert abs(p["E_dir"]) < 1e-12 * KE


def test_vacuum_dielectric_is_the_shifted_coulomb_potential():
    # eps_s = 1: k_RF = 0, c_RF = 1/r_c, U = k_e q q (1/r - 1/r_c)
    p = _pair(3.0, 1.0)
    assert p["E_dir"] == pytest.approx(KE * 0.8 * -0.6 * (1 / 3.0 - 1 / 9.0), rel=1e-14)
    f = p["F"][0, 1]   # along +x on atom 1 (x_j - x_i = +r)
    assert f == pytest.approx(KE * 0.8 * -0.6 / 9.0, rel=1e-14)


def test_conducting_limit_force_vanishes_at_the_cutoff():
    p = _pair(9.0, math.inf)
    assert np.abs(p["F"]).max() < 1e-12 * KE
    k, c = nonbonded.reaction_field_constants(9.0, math.inf)
    k2, c2 = nonbonded.reaction_field_constants(9.0, 1e12)
    assert k == pytest.approx(k2, rel=1e-9) and c == pytest.approx(c2, rel=1e-9)


@pytest.mark.parametrize("r", [2.5, 5.0, 8.7])
def test_force_is_minus_the_energy_gradient(r):
    h = 1e-5
    e_p = _pair(r + h, 78.5)["E_dir"]
    e_m = _pair(r - h, 78.5)["E_dir"]
    f = _pair(r, 78.5)["F"]
    assert f[0, 1] == pytest.approx(-(e_p - e_m) / (2 * h), rel=1e-7)
    assert np.allclose(f[:, 0], -f[:, 1], rtol=0, atol=1e-12 * KE)


def test_large_cutoff_tends_to_plain_coulomb():
    p = _pair(3.0, 78.5, r_cut=1.0e5)
    assert p["E_dir"] == pytest.approx(KE * 0.8 * -0.6 / 3.0, rel=1e-4)


def test_water_box_has_no_ewald_parts():
    s = synth.config_system("water375")
    s.rf_epsilon = 78.5
    s.ewald_delta = 0.0
    s.pme_grid = (0, 0, 0)
    t = forcefield.nonbonded_terms(s)
    assert t["E"][2] == 0.0 and t["E"][3] == 0.0          # exclusion, self
    assert t["E"][1] != 0.0
    assert np.abs(t["F"].sum(axis=1)).max() < 1e-9 * np.abs(t["F"]).max()
