"""Sums the oracle's components for a system object.

The system object carries the fields of synth.System (float32 positions and
parameters, int32 topology); everything is widened to float64 here.

Energy slots, in order: LJ, Coulomb real-space, exclusion correction,
self (+ neutralising) term, bonds, angles; the reciprocal PME energy is
returned separately.
"""
from __future__ import annotations

import numpy as np

from . import bonded, ewald, neighbors, nonbonded, pme

ENERGY_NAMES = ("lj", "coul_dir", "coul_excl", "coul_self", "bond", "angle")


def alpha(sys) -> float:
    if getattr(sys, "rf_epsilon", 0.0) > 0:
        return 0.0   # reaction field: no Ewald split
    if not sys.ewald_delta or sys.ewald_delta <= 0:
        return 0.0
    return ewald.alpha_from_tolerance(float(sys.ewald_delta), float(sys.r_cut))


def neighbor_list(sys, pos=None, method="tree"):
    pos = sys.pos if pos is None else pos
    fn = neighbors.tree_pairs if method == "tree" else neighbors.brute_force_pairs
    return fn(pos, sys.box, sys.r_cut, sys.r_ghost, sys.exclusions)


def nonbonded_terms(sys, pos=None, pairs=None):
    """Short-range terms with the float32 interaction decision on `pos`.

    pos: float32 [3,N] (defaults to sys.pos); pairs: the Verlet list to draw
    interacting pairs from (defaults to the list built at `pos`).
    Returns dict(E [6], F [3,N], W [3,3], n_interacting).
    """
    pos = np.asarray(sys.pos if pos is None else pos, np.float32)
    if pairs is None:
        pairs = neighbor_list(sys, pos)
    inter = pairs[neighbors.interacting(pos, sys.box, sys.r_cut, sys.r_ghost, pairs)]
    a = alpha(sys)
    p64 = pos.astype(np.float64)
    pt = nonbonded.pair_terms(p64, sys.box, inter, sys.atom_type, sys.type_sigma,
                              sys.type_epsilon, sys.charge, a, sys.coulomb_k,
                              r_cut=float(sys.r_cut), switch_r=float(sys.switch_r),
                              rf_epsilon=float(getattr(sys, "rf_epsilon", 0.0)))
    ex = nonbonded.exclusion_correction(p64, sys.box, sys.exclusions, sys.charge, a,
                                        sys.coulomb_k)
    e_self = nonbonded.self_energy(sys.charge, sys.box, a, sys.coulomb_k) if a > 0 else 0.0
    bo = bonded.bonds(p64, sys.box, sys.bonds, sys.bond_k, sys.bond_r0)
    an = bonded.angles(p64, sys.box, sys.angles, sys.angle_k, sys.angle_theta0)
    E = np.array([pt["E_lj"], pt["E_dir"], ex["E"], e_self, bo["E"], an["E"]])
    F = pt["F"] + ex["F"] + bo["F"] + an["F"]
    W = pt["W"] + ex["W"] + bo["W"] + an["W"]
    return dict(E=E, F=F, W=W, n_interacting=len(inter), n_listed=len(pairs),
                parts=dict(pair=pt, excl=ex, bond=bo, angle=an))


def pme_terms(sys, pos=None, order=4):
    pos = np.asarray(sys.pos if pos is None else pos, np.float32)
    return pme.spme(pos.astype(np.float64), sys.charge, sys.box, sys.pme_grid, alpha(sys),
                    sys.coulomb_k, order)


def total_forces_fp64(sys, pos64):
    """All terms at float64 positions with a float64 cutoff (no list): the
    plain definition used for trajectories."""
    from scipy.spatial import cKDTree
    pos64 = np.asarray(pos64, np.float64)
    L = np.asarray(sys.box, np.float64)
    tree = cKDTree(np.mod(pos64.T, L), boxsize=L)
    pairs = tree.query_pairs(float(sys.r_cut), output_type="ndarray")
    if len(pairs) and len(sys.exclusions):
        n = pos64.shape[1]
        keys = pairs.min(1).astype(np.int64) * n + pairs.max(1)
        ex = np.asarray(sys.exclusions, np.int64)
        ekeys = ex.min(1) * n + ex.max(1)
        pairs = pairs[~np.isin(keys, ekeys)]
    pairs = np.sort(pairs, axis=1) if len(pairs) else np.zeros((0, 2), np.int64)
    a = alpha(sys)
    pt = nonbonded.pair_terms(pos64, sys.box, pairs, sys.atom_type, sys.type_sigma,
                              sys.type_epsilon, sys.charge, a, sys.coulomb_k,
                              r_cut=float(sys.r_cut), switch_r=float(sys.switch_r),
                              rf_epsilon=float(getattr(sys, "rf_epsilon", 0.0)))
    ex = nonbonded.exclusion_correction(pos64, sys.box, sys.exclusions, sys.charge, a,
                                        sys.coulomb_k)
    bo = bonded.bonds(pos64, sys.box, sys.bonds, sys.bond_k, sys.bond_r0)
    an = bonded.angles(pos64, sys.box, sys.angles, sys.angle_k, sys.angle_theta0)
    e_self = nonbonded.self_energy(sys.charge, sys.box, a, sys.coulomb_k) if a > 0 else 0.0
    U = pt["E_lj"] + pt["E_dir"] + ex["E"] + bo["E"] + an["E"] + e_self
    F = pt["F"] + ex["F"] + bo["F"] + an["F"]
    if a > 0 and sum(sys.pme_grid) > 0:
        r = pme.spme(pos64, sys.charge, sys.box, sys.pme_grid, a, sys.coulomb_k)
        U += r["E"]
        F = F + r["F"]
    return U, F
