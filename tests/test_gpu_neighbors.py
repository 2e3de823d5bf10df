"""GPU parity: Verlet list from the HIP cell-list build vs the oracle (bit-exact)."""
import numpy as np
import pytest

import synth
from oracle import neighbors
from helpers import announce, gpu_context

pytestmark = pytest.mark.gpu


def _oracle_pairs(s):
    return neighbors.tree_pairs(s.pos, s.box, s.r_cut, s.r_ghost, s.exclusions)


@pytest.mark.parametrize("options", [0, 1, 2], ids=["full", "half", "cooperative-build"])
@pytest.mark.parametrize("name", ["lj1k", "water375", "water9k"])
def test_list_exact(name, options):
    s = synth.config_system(name)
    announce(f"list {name} N={s.n_atoms} options={options}")
    with gpu_context(s, options=options) as (mdx, ctx, t):
        assert mdx.get_info(ctx).n_list_entries == -1
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
        assert mdx.get_status(ctx) == 0
        info = mdx.get_info(ctx)
    ref = _oracle_pairs(s)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    # every pair is held from both ends (full list, the default) or once
    # (MDX_OPT_HALF_LIST); tiles come in groups of four
    assert info.n_list_entries == (1 if options & 1 else 2) * len(ref)
    assert info.n_builds == 1
    assert info.n_list_tiles % 4 == 0 and 16 * info.n_list_tiles >= info.n_list_entries


@pytest.mark.parametrize("m", [1, 2, 3])
def test_list_invariant_to_cell_width(m):
    s = synth.random_box(3000, [14.0, 15.0, 16.0], 2.5, 0.5, 77, n_excl_per_atom=2)
    announce(f"list cell_divisions={m}")
    with gpu_context(s, cell_divisions=m) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
    assert np.array_equal(got, _oracle_pairs(s))


@pytest.mark.parametrize("seed,n,box,rc,rg", [
    (101, 500, [6.0, 6.0, 6.0], 2.0, 0.5),     # 2-3 cells per dimension: stencil wraps onto itself
    (102, 1, [5.0, 5.0, 5.0], 1.0, 0.2),       # a single atom: empty list
    (103, 2000, [20.0, 9.0, 30.0], 3.0, 1.4),  # anisotropic box, ragged cells
    (104, 4097, [12.0, 12.0, 12.0], 2.2, 0.3), # ragged final wave
])
def test_list_edge_cases(seed, n, box, rc, rg):
    s = synth.random_box(n, box, rc, rg, seed, n_excl_per_atom=1)
    announce(f"list edge seed={seed} n={n}")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
    assert np.array_equal(got, _oracle_pairs(s))


def test_list_relabelling_and_capacity_growth():
    s = synth.random_box(1500, [10.0, 10.0, 10.0], 2.4, 0.4, 55, n_excl_per_atom=1)
    perm = np.random.default_rng(1).permutation(s.n_atoms)
    inv = np.argsort(perm)
    s2 = s.copy()
    s2.pos = np.ascontiguousarray(s.pos[:, perm])
    s2.atom_type = s.atom_type[perm]
    s2.charge = s.charge[perm]
    s2.mass = s.mass[perm]
    s2.vel = np.ascontiguousarray(s.vel[:, perm])
    s2.exclusions = inv[s.exclusions].astype(np.int32)
    announce("list relabelled, capacity 16 (forces regrowth)")
    with gpu_context(s2, nl_capacity=16) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
        assert mdx.get_info(ctx).nl_capacity > 16
        assert mdx.get_status(ctx) & mdx.MDX_FLAG_NL_OVERFLOW == 0
    mapped = np.sort(perm[got], axis=1)
    mapped = mapped[np.lexsort((mapped[:, 1], mapped[:, 0]))]
    assert np.array_equal(mapped, _oracle_pairs(s))


def test_list_crowded_column_grows_column_capacity():
    # 600 of 2000 atoms squeezed into one x-y column: far more than a column
    # holds by default, so the build latches the column overflow, grows the
    # column lists and builds again; the list is still the exact one
    s = synth.random_box(2000, [20.0, 20.0, 20.0], 2.0, 0.5, 31, n_excl_per_atom=1)
    rng = np.random.default_rng(5)
    s.pos[0, :600] = rng.uniform(0.0, 1.0, 600).astype(np.float32)
    s.pos[1, :600] = rng.uniform(0.0, 1.0, 600).astype(np.float32)
    announce("list with one crowded column")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
        assert mdx.get_status(ctx) == 0
    assert np.array_equal(got, _oracle_pairs(s))


def test_list_rebuilds_in_slot_order_stay_exact():
    # Later builds bin the atoms in the slot order of the build before, when
    # that build placed every atom, and in atom order otherwise (after a
    # column overflow). The list must be the exact one either way: a normal
    # build, a moved configuration (slot order), a crowded column (slot order,
    # overflow, regrown and rebuilt in atom order), and a normal one again.
    s = synth.random_box(2000, [20.0, 20.0, 20.0], 2.0, 0.5, 33, n_excl_per_atom=1)
    rng = np.random.default_rng(9)
    moved = s.copy()
    moved.pos = np.mod(s.pos + rng.uniform(-1.5, 1.5, s.pos.shape), 20.0).astype(np.float32)
    moved.pos[moved.pos >= 20.0] = 0.0   # float32 rounding onto the box edge
    crowded = s.copy()
    crowded.pos = s.pos.copy()
    crowded.pos[0, :600] = rng.uniform(0.0, 1.0, 600).astype(np.float32)
    crowded.pos[1, :600] = rng.uniform(0.0, 1.0, 600).astype(np.float32)
    import torch
    announce("list rebuilt in slot order (moved, crowded, normal)")
    with gpu_context(s) as (mdx, ctx, t):
        for k, cfg in enumerate([s, moved, crowded, s]):
            p = torch.from_numpy(np.ascontiguousarray(cfg.pos)).to(t["pos"].device)
            mdx.build_neighbors(ctx, p)
            got = mdx.get_neighbor_pairs(ctx)
            assert mdx.get_status(ctx) == 0, k
            assert np.array_equal(got, _oracle_pairs(cfg)), k


def test_list_water96k_whole_list_and_sampled_rows():
    # the whole sorted pair list against the oracle's (its count and sha256,
    # written by tests/golden/make_counts.py from the oracle), then 300 rows
    # against the brute-force rows of the oracle
    import hashlib
    import json
    import os
    s = synth.config_system("water96k")
    announce("list water96k")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
        assert mdx.get_status(ctx) == 0
    with open(os.path.join(os.path.dirname(__file__), "golden", "pair_counts.json")) as f:
        golden = json.load(f)["water96k"]
    assert len(got) == golden["listed_pairs"]
    rows = np.ascontiguousarray(got, dtype="<i4")
    assert hashlib.sha256(rows.tobytes()).hexdigest() == golden["list_sha256"]
    rng = np.random.default_rng(3)
    sample = rng.choice(s.n_atoms, 300, replace=False)
    first, second = got[:, 0], got[:, 1]
    order2 = np.argsort(second, kind="stable")
    s2 = second[order2]
    for i in sample:
        a = got[np.searchsorted(first, i):np.searchsorted(first, i, "right"), 1]
        b = got[order2[np.searchsorted(s2, i):np.searchsorted(s2, i, "right")], 0]
        row = np.sort(np.concatenate([a, b]))
        ref = neighbors.neighbors_of(s.pos, s.box, s.r_cut, s.r_ghost, int(i), s.exclusions)
        assert np.array_equal(row, ref), i
    # density check on the total: pairs within r_nl of a uniform liquid
    rnl = float(np.float32(s.r_cut + s.r_ghost))
    expect = 0.5 * s.n_atoms * (s.n_atoms / np.prod(s.box.astype(float))) * 4 / 3 * np.pi * rnl ** 3
    assert abs(len(got) / expect - 1.0) < 0.02


def test_list_with_nan_coordinates_flags_and_skips_them():
    # a diverged trajectory: atoms with a NaN coordinate are flagged out of
    # box, take part in no pair, and the rest of the list is unchanged
    s = synth.random_box(1500, [10.0, 10.0, 10.0], 2.4, 0.4, 56, n_excl_per_atom=1)
    bad = np.array([5, 17, 400, 1499])
    s2 = s.copy()
    s2.pos = s.pos.copy()
    s2.pos[2, bad[0]] = np.nan      # z only: the column sort key
    s2.pos[:, bad[1]] = np.nan      # every coordinate
    s2.pos[0, bad[2]] = np.nan      # x only: the binning
    s2.pos[2, bad[3]] = np.nan
    announce("list with NaN coordinates")
    with gpu_context(s2) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        got = mdx.get_neighbor_pairs(ctx)
        assert mdx.get_status(ctx) & mdx.MDX_FLAG_OUT_OF_BOX
    keep = np.setdiff1d(np.arange(s.n_atoms), bad)
    new = -np.ones(s.n_atoms, dtype=np.int64)
    new[keep] = np.arange(len(keep))
    ex = s.exclusions[np.all(new[s.exclusions] >= 0, axis=1)]
    ref = neighbors.tree_pairs(np.ascontiguousarray(s.pos[:, keep]), s.box, s.r_cut,
                               s.r_ghost, new[ex].astype(np.int32))
    assert np.array_equal(got, keep[ref])
