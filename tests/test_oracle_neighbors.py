"""Pins for the oracle's Verlet list (Sec. II.A.2, "Neighborlists")."""
import numpy as np
import pytest

import synth
from oracle import neighbors


def _naive_fp64_pairs(pos, box, r_nl):
    """Textbook all-pairs list in float64 (independent of the float32 predicate)."""
    p = pos.astype(np.float64)
    L = box.astype(np.float64)
    n = p.shape[1]
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            d = p[:, j] - p[:, i]
            d -= L * np.round(d / L)
            if d @ d < r_nl * r_nl:
                out.append((i, j))
    return np.array(out, np.int32).reshape(-1, 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_matches_tree_seeded(seed):
    s = synth.random_box(600, [9.0, 10.0, 11.0], 2.5, 0.4, seed, n_excl_per_atom=2)
    bf = neighbors.brute_force_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    tr = neighbors.tree_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    assert len(bf) > 1000
    assert np.array_equal(bf, tr)


def test_fp32_predicate_agrees_with_fp64_away_from_rnl():
    s = synth.random_box(300, [7.0, 7.0, 7.0], 2.0, 0.5, 11, n_excl_per_atom=0)
    f32 = neighbors.brute_force_pairs(s.pos, s.box, s.r_cut, s.r_ghost)
    rnl = float(np.float32(s.r_cut + s.r_ghost))
    f64 = _naive_fp64_pairs(s.pos, s.box, rnl)
    a = {tuple(p) for p in f32}
    b = {tuple(p) for p in f64}
    diff = a ^ b
    for i, j in diff:   # only pairs within rounding of r_nl may differ
        d = s.pos[:, j].astype(np.float64) - s.pos[:, i]
        d -= s.box * np.round(d / s.box)
        assert abs(np.sqrt(d @ d) - rnl) < 1e-5
    assert len(a) > 500


def test_list_invariant_under_relabelling():
    s = synth.random_box(400, [8.0, 8.0, 8.0], 2.2, 0.3, 5, n_excl_per_atom=1)
    base = neighbors.brute_force_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    perm = np.random.default_rng(0).permutation(s.n_atoms)
    inv = np.argsort(perm)
    pos2 = s.pos[:, perm]
    ex2 = inv[s.exclusions]
    got = neighbors.brute_force_pairs(pos2, s.box, s.r_cut, s.r_ghost, ex2)
    mapped = perm[got]
    mapped = np.sort(mapped, axis=1)
    mapped = mapped[np.lexsort((mapped[:, 1], mapped[:, 0]))]
    assert np.array_equal(mapped, base)


def test_predicate_symmetric_and_periodic_hand_case():
    box = np.array([10.0, 10.0, 10.0], np.float32)
    pos = np.array([[0.25, 9.75, 5.0, 5.0],
                    [5.0, 5.0, 0.1, 5.0],
                    [5.0, 5.0, 5.0, 5.0]], np.float32)
    # atoms 0,1 are 0.5 apart through the x boundary; atoms 2,3 are 4.9 apart
    pairs = neighbors.brute_force_pairs(pos, box, 1.0, 0.0)
    assert [tuple(p) for p in pairs] == [(0, 1)]
    pairs = neighbors.brute_force_pairs(pos, box, 4.0, 1.0)   # r_nl = 5
    assert (2, 3) in {tuple(p) for p in pairs}
    i = np.array([0, 1, 2, 3, 0])
    j = np.array([1, 0, 3, 2, 3])
    r2 = neighbors.r2_f32(pos, box, i, j)
    assert r2[0] == r2[1] and r2[2] == r2[3]
    assert abs(float(r2[0]) - 0.25) < 1e-6


def test_exclusions_removed_and_rows_consistent():
    s = synth.config_system("water375")
    full = neighbors.tree_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    keys = set(map(tuple, full))
    for a, b in s.exclusions:
        assert (min(a, b), max(a, b)) not in keys
    for i in (0, 1, 2, 100, 374):
        row = neighbors.neighbors_of(s.pos, s.box, s.r_cut, s.r_ghost, i, s.exclusions)
        expect = np.sort(np.concatenate([full[full[:, 0] == i, 1], full[full[:, 1] == i, 0]]))
        assert np.array_equal(row, expect)


def test_interaction_set_is_subset_with_rc():
    s = synth.config_system("water375")
    full = neighbors.tree_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)
    m = neighbors.interacting(s.pos, s.box, s.r_cut, s.r_ghost, full)
    d = s.pos[:, full[:, 1]].astype(np.float64) - s.pos[:, full[:, 0]]
    d -= s.box[:, None] * np.round(d / s.box[:, None])
    r = np.sqrt((d * d).sum(0))
    far = np.abs(r - float(s.r_cut)) > 1e-5
    assert np.array_equal(m[far], (r < float(s.r_cut))[far])
    # the ghost shell holds the expected share of pairs for a uniform fluid
    frac = m.mean()
    rnl = float(s.r_cut + s.r_ghost)
    assert abs(frac - (float(s.r_cut) / rnl) ** 3) < 0.08


def test_min_image_f32_accurate_and_antisymmetric():
    rng = np.random.default_rng(12)
    L = np.float32(98.6)
    xi = (rng.random(20000) * np.float64(L)).astype(np.float32)
    xj = (rng.random(20000) * np.float64(L)).astype(np.float32)
    d = neighbors.min_image_f32(xi, xj, L)
    d_rev = neighbors.min_image_f32(xj, xi, L)
    assert np.array_equal(d, -d_rev)
    exact = xj.astype(np.float64) - xi.astype(np.float64)
    exact = np.where(exact > L / 2, exact - np.float64(L), np.where(exact < -L / 2, exact + np.float64(L), exact))
    err = np.abs(d.astype(np.float64) - exact)
    assert np.all(err <= 0.5 * np.spacing(np.abs(d)) + 1e-30)
