"""Verlet neighbour list, oracle side (paper Sec. II.A.2, "Neighborlists").

The list holds every non-excluded pair closer than r_nl = r_c + r_g
(Sec. II.A.2; exclusions are removed at list level, "Exclusions and
Exceptions" paragraph). Because several lists are "correct" within rounding
of r_nl, the inclusion test is pinned to one IEEE float32 expression:

    s    = fl32(x_j - x_i)                                   per dimension
    d    = s                        if -L/2 <= s <= L/2
         = fl32(fl32(x_j - L) - x_i) if s > L/2
         = fl32(x_j + fl32(L - x_i)) if s < -L/2
    r2   = fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz))
    keep iff r2 < fl32(r_nl * r_nl),  r_nl = fl32(r_c + r_g)

(The wrapped branches subtract the box from the coordinate that lies in the
far half first, which is exact, so d is within half an ulp of the exact
minimum-image displacement instead of half an ulp of L; the expression is
antisymmetric in i, j, so the predicate is symmetric.)

and a pair *interacts* iff it is listed and r2 < fl32(r_c * r_c) under the
same expression. numpy float32 arithmetic is correctly rounded and never
fused, so this module reproduces the predicate exactly.

Lists are returned as int32 [P, 2] arrays of (i, j), i < j, sorted
lexicographically.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def cutoffs_f32(r_cut, r_ghost):
    """(rnl2, rc2) float32 thresholds of the predicate."""
    rc = F32(r_cut)
    rnl = F32(rc + F32(r_ghost))
    return F32(rnl * rnl), F32(rc * rc)


def min_image_f32(xi, xj, L):
    """Per-dimension float32 minimum-image displacement x_j - x_i (one wrap)."""
    L = F32(L)
    hL = F32(L * F32(0.5))
    xi = np.asarray(xi, F32)
    xj = np.asarray(xj, F32)
    s = (xj - xi).astype(F32)
    up = ((xj - L).astype(F32) - xi).astype(F32)      # s > L/2
    dn = (xj + (L - xi).astype(F32)).astype(F32)      # s < -L/2
    d = np.where(s > hL, up, np.where(s < -hL, dn, s))
    return d.astype(F32)


def r2_f32(pos, box, i, j):
    """float32 squared distances of pairs (i[k], j[k]); pos is float32 [3, N]."""
    dx = min_image_f32(pos[0, i], pos[0, j], box[0])
    dy = min_image_f32(pos[1, i], pos[1, j], box[1])
    dz = min_image_f32(pos[2, i], pos[2, j], box[2])
    return ((dx * dx).astype(F32) + (dy * dy).astype(F32)).astype(F32) + (dz * dz).astype(F32)


def _exclusion_keys(exclusions, n):
    ex = np.asarray(exclusions, dtype=np.int64).reshape(-1, 2)
    lo, hi = np.minimum(ex[:, 0], ex[:, 1]), np.maximum(ex[:, 0], ex[:, 1])
    return np.unique(lo * n + hi)


def _drop_excluded(pairs, exclusions, n):
    if len(pairs) == 0 or len(exclusions) == 0:
        return pairs
    keys = pairs[:, 0].astype(np.int64) * n + pairs[:, 1]
    return pairs[~np.isin(keys, _exclusion_keys(exclusions, n))]


def _canonical(i, j):
    pairs = np.stack([np.minimum(i, j), np.maximum(i, j)], axis=1).astype(np.int32)
    if len(pairs) == 0:
        return pairs.reshape(0, 2)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order]


def brute_force_pairs(pos, box, r_cut, r_ghost, exclusions=()):
    """O(N^2) list: every i<j tested with the float32 predicate."""
    pos = np.asarray(pos, dtype=F32)
    n = pos.shape[1]
    rnl2, _ = cutoffs_f32(r_cut, r_ghost)
    out_i, out_j = [], []
    for i in range(n - 1):
        j = np.arange(i + 1, n)
        r2 = r2_f32(pos, box, np.full(j.size, i), j)
        keep = j[r2 < rnl2]
        out_i.append(np.full(keep.size, i))
        out_j.append(keep)
    if not out_i:
        return np.zeros((0, 2), np.int32)
    pairs = _canonical(np.concatenate(out_i), np.concatenate(out_j))
    return _drop_excluded(pairs, exclusions, n)


def tree_pairs(pos, box, r_cut, r_ghost, exclusions=(), margin=1e-3):
    """Same list as brute_force_pairs for large N.

    Candidates come from scipy's periodic k-d tree at radius r_nl + margin
    (float64 geometry, a library primitive); the float32 predicate then
    decides. The margin is far wider than float32 rounding of distances
    below the box size, so no predicate-true pair is missed.
    """
    from scipy.spatial import cKDTree
    pos = np.asarray(pos, dtype=F32)
    n = pos.shape[1]
    box64 = np.asarray(box, dtype=np.float64)
    rnl2, _ = cutoffs_f32(r_cut, r_ghost)
    rnl64 = float(F32(F32(r_cut) + F32(r_ghost)))
    tree = cKDTree(pos.T.astype(np.float64), boxsize=box64)
    cand = tree.query_pairs(rnl64 + margin, output_type="ndarray")
    if cand.size == 0:
        return np.zeros((0, 2), np.int32)
    r2 = r2_f32(pos, box, cand[:, 0], cand[:, 1])
    cand = cand[r2 < rnl2]
    pairs = _canonical(cand[:, 0], cand[:, 1])
    return _drop_excluded(pairs, exclusions, n)


def neighbors_of(pos, box, r_cut, r_ghost, i, exclusions=()):
    """Sorted partner indices of atom i (both directions) by brute force."""
    pos = np.asarray(pos, dtype=F32)
    n = pos.shape[1]
    rnl2, _ = cutoffs_f32(r_cut, r_ghost)
    j = np.arange(n)
    j = j[j != i]
    r2 = r2_f32(pos, box, np.full(j.size, i), j)
    nb = j[r2 < rnl2]
    if len(exclusions):
        ex = np.asarray(exclusions).reshape(-1, 2)
        partners = np.concatenate([ex[ex[:, 0] == i, 1], ex[ex[:, 1] == i, 0]])
        nb = nb[~np.isin(nb, partners)]
    return np.sort(nb).astype(np.int32)


def interacting(pos, box, r_cut, r_ghost, pairs):
    """Mask of listed pairs that interact: float32 r2 < fl32(r_c^2)."""
    _, rc2 = cutoffs_f32(r_cut, r_ghost)
    if len(pairs) == 0:
        return np.zeros(0, bool)
    return r2_f32(np.asarray(pos, F32), box, pairs[:, 0], pairs[:, 1]) < rc2
