"""GPU parity: short-range forces/energies/virials and PME vs the FP64 oracle.

Bars: forces within 1e-5 relative RMS (||F_gpu - F_orc|| / ||F_orc|| over all 3N
components), energies within 1e-6 relative, virial entries within 1e-5 of the
largest diagonal entry.
"""
import numpy as np
import pytest

import synth
from oracle import forcefield
from helpers import announce, gpu_context, rel_rms

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6
W_TOL = 1e-5     # virial entries, relative to the largest diagonal entry


def _nonbonded_gpu(s, **kw):
    import torch
    with gpu_context(s, **kw) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
        torch.cuda.synchronize()
        flags = mdx.get_status(ctx)
        return t["force"].cpu().numpy(), t["e_nb"].cpu().numpy(), flags


HALF_LIST = 0x1   # MDX_OPT_HALF_LIST: each pair once, j forces summed in list order


@pytest.mark.parametrize("options", [0, HALF_LIST], ids=["full", "half"])
@pytest.mark.parametrize("name", ["lj1k", "water375", "water9k"])
def test_nonbonded_parity(name, options):
    s = synth.config_system(name)
    announce(f"nonbonded {name} options={options}")
    F, E, flags = _nonbonded_gpu(s, options=options)
    assert flags == 0
    ref = forcefield.nonbonded_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    Eref = ref["E"]
    scale = max(abs(Eref.sum()), 1e-30)
    for k in range(6):
        assert abs(E[k] - Eref[k]) <= E_TOL * max(abs(Eref[k]), scale), (k, E[k], Eref[k])
    assert abs(E.sum() - Eref.sum()) <= E_TOL * scale


def test_nonbonded_switched_random():
    s = synth.random_box(2500, [13.0, 13.0, 13.0], 3.0, 0.5, 211, min_dist=0.75)
    s.switch_r = np.float32(2.4)
    announce("nonbonded switched random")
    F, E, flags = _nonbonded_gpu(s)
    ref = forcefield.nonbonded_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    assert abs(E[:4].sum() - ref["E"][:4].sum()) <= E_TOL * abs(ref["E"][:4].sum())


def test_nonbonded_bitwise_deterministic():
    # the default full list uses no float atomics: forces and energies
    # repeat bit for bit
    import torch
    s = synth.config_system("water9k")
    announce("nonbonded determinism")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        outs = []
        for _ in range(2):
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
            mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
            torch.cuda.synchronize()
            outs.append((t["force"].cpu().numpy().copy(), t["e_nb"].cpu().numpy().copy(),
                         t["e_rec"].cpu().numpy().copy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_half_list_matches_full_list_and_repeats_bitwise():
    # the half list agrees with the full list to float32 rounding; it uses no
    # float atomics (the j forces are summed in list order), so its forces
    # and FP64 energies repeat bit for bit, in a fresh context and in the
    # same one after a rebuild
    import torch
    s = synth.config_system("water9k")
    announce("half vs full list")
    F_full, E_full, _ = _nonbonded_gpu(s)
    F1, E1, f1 = _nonbonded_gpu(s, options=HALF_LIST)
    F2, E2, f2 = _nonbonded_gpu(s, options=HALF_LIST)
    assert f1 == 0 and f2 == 0
    assert rel_rms(F1, F_full) < 1e-6
    assert np.array_equal(F1, F2)
    assert np.array_equal(E1, E2)
    assert np.allclose(E1, E_full, rtol=1e-12, atol=1e-9)
    with gpu_context(s, options=HALF_LIST) as (mdx, ctx, t):
        for _ in range(2):
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
        torch.cuda.synchronize()
        assert np.array_equal(t["force"].cpu().numpy(), F1)


@pytest.mark.parametrize("name", ["water375", "water9k"])
def test_pme_parity(name):
    import torch
    s = synth.config_system(name)
    announce(f"pme {name}")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        t["force"].zero_()
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
        torch.cuda.synchronize()
        F = t["force"].cpu().numpy()
        E = float(t["e_rec"].cpu().numpy()[0])
        assert mdx.get_status(ctx) == 0
    ref = forcefield.pme_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    assert abs(E - ref["E"]) <= E_TOL * abs(ref["E"])


def test_pme_mixed_radix_grid():
    import torch
    s = synth.water_box(300, 20.9, (27, 20, 25), 7.0, 1.5, 5e-4, 9, name="mixed")
    announce("pme grid 27x20x25")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        t["force"].zero_()
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
        torch.cuda.synchronize()
        F = t["force"].cpu().numpy()
        E = float(t["e_rec"].cpu().numpy()[0])
    ref = forcefield.pme_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    assert abs(E - ref["E"]) <= E_TOL * abs(ref["E"])


@pytest.mark.parametrize("grid", [(10, 10, 10), (12, 12, 12), (16, 10, 12)])
def test_pme_small_grids(grid):
    # grids of 11 or more points per axis spread by z-lines in registers,
    # smaller ones through the LDS atomic kernel; both against the oracle
    import torch
    s = synth.water_box(64, 12.4, grid, 5.0, 1.0, 5e-4, 4, name="small")
    announce(f"pme grid {grid}")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        t["force"].zero_()
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
        torch.cuda.synchronize()
        F = t["force"].cpu().numpy()
        E = float(t["e_rec"].cpu().numpy()[0])
        assert mdx.get_status(ctx) == 0
    ref = forcefield.pme_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    assert abs(E - ref["E"]) <= E_TOL * abs(ref["E"])


def test_total_force_water9k():
    import torch
    s = synth.config_system("water9k")
    announce("total force water9k")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
        torch.cuda.synchronize()
        F = t["force"].cpu().numpy()
        E = np.concatenate([t["e_nb"].cpu().numpy(), t["e_rec"].cpu().numpy()])
    nb = forcefield.nonbonded_terms(s)
    rec = forcefield.pme_terms(s)
    assert rel_rms(F, nb["F"] + rec["F"]) < F_TOL
    Et = nb["E"].sum() + rec["E"]
    assert abs(E.sum() - Et) <= E_TOL * abs(Et)


def test_water96k_full_size_sampled_forces_and_energies():
    # The benchmark's 96,000-atom box at full size, against FP64 oracle values
    # stored by tests/golden/make_w96k_forces.py: all energy components, and
    # the total force on 600 sampled atoms.
    import json
    import os
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "w96k_forces.json")))
    s = synth.config_system("water96k")
    announce("water96k full size")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"])
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        F = t["force"].cpu().numpy().astype(np.float64)
        E = np.concatenate([t["e_nb"].cpu().numpy(), t["e_rec"].cpu().numpy()])
        # 12 steps of the benchmark's path (in-step list rebuild, pruned
        # list, PME FFTs on the second stream, fused closing kernel): the
        # force it leaves behind equals a fresh full-list evaluation at the
        # new positions
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], 12, s.dt)
        torch.cuda.synchronize()
        F_step = t["force"].cpu().numpy().astype(np.float64)
        f2 = torch.zeros_like(t["force"])
        mdx.compute_nonbonded(ctx, t["pos"], f2)
        mdx.compute_pme(ctx, t["pos"], f2)
        torch.cuda.synchronize()
        F_fresh = f2.cpu().numpy().astype(np.float64)
        assert mdx.get_status(ctx) == 0
    sample = np.array(gold["sample"])
    Fref = np.array(gold["forces"]).T
    assert rel_rms(F[:, sample], Fref) < F_TOL
    Eref = np.array(gold["energies"])
    scale = abs(Eref.sum())
    for k in range(len(Eref)):
        assert abs(E[k] - Eref[k]) <= E_TOL * max(abs(Eref[k]), scale), (k, E[k], Eref[k])
    assert abs(E.sum() - Eref.sum()) <= E_TOL * scale, (E.sum(), Eref.sum())
    assert rel_rms(F_step, F_fresh) < 1e-6


def test_pruned_list_written_in_chunks_keeps_every_pair():
    # An LJ fluid with a long cutoff: about 450 tiles per cluster, so a walk
    # that writes the pruned list does so in several chunks of 256 tiles.
    # After steps that rebuild the list and write the pruned list again, the
    # force the step leaves equals a fresh full-list evaluation.
    import torch
    s = synth.lj_fluid(n_side=20, density=0.8, r_cut=6.0, r_ghost=1.0, temperature=1.0,
                       dt=0.002)
    announce(f"pruned list in chunks: LJ N={s.n_atoms} r_c=6")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        info = mdx.get_info(ctx)
        assert info.n_list_tiles > 256 * (s.n_atoms // 4)
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], 25, s.dt)
        torch.cuda.synchronize()
        F_step = t["force"].cpu().numpy().astype(np.float64)
        f2 = torch.zeros_like(t["force"])
        mdx.compute_nonbonded(ctx, t["pos"], f2)
        torch.cuda.synchronize()
        F_fresh = f2.cpu().numpy().astype(np.float64)
        assert mdx.get_status(ctx) == 0
        assert mdx.get_info(ctx).n_builds >= 3
    assert rel_rms(F_step, F_fresh) < 1e-6


def _off_equilibrium(s, seed=4):
    # water away from its rigid geometry, so bonds and angles carry force
    s = s.copy()
    p = s.pos.astype(np.float64) + np.random.default_rng(seed).normal(0.0, 0.02, s.pos.shape)
    s.pos = np.mod(p, s.box.astype(np.float64)[:, None]).astype(np.float32)
    return s


@pytest.mark.parametrize("options", [0, HALF_LIST], ids=["full", "half"])
@pytest.mark.parametrize("name", ["lj1k", "water375", "water9k"])
def test_nonbonded_virial_parity(name, options):
    import torch
    s = synth.config_system(name)
    if s.bonds.size:
        s = _off_equilibrium(s)
    announce(f"nonbonded virial {name} options={options}")
    with gpu_context(s, options=options) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        W = torch.zeros(9, dtype=torch.float64, device="cuda:0")
        # virial without energies, then with: the same numbers
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], None, W)
        torch.cuda.synchronize()
        W1 = W.cpu().numpy().reshape(3, 3).copy()
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"], W)
        torch.cuda.synchronize()
        W2 = W.cpu().numpy().reshape(3, 3)
        F = t["force"].cpu().numpy()
        assert mdx.get_status(ctx) == 0
    ref = forcefield.nonbonded_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    Wref = ref["W"]
    assert np.array_equal(W1, W2) and np.array_equal(W1, W1.T)
    scale = np.abs(np.diag(Wref)).max()
    assert np.abs(W1 - Wref).max() <= W_TOL * scale, (W1, Wref)
    if s.bonds.size:   # the bonded part is exercised
        assert np.abs(np.diag(ref["parts"]["bond"]["W"])).max() > 1e-3 * scale


@pytest.mark.parametrize("name", ["water375", "water9k"])
def test_pme_virial_parity(name):
    import torch
    s = synth.config_system(name)
    announce(f"pme virial {name}")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        t["force"].zero_()
        W = torch.zeros(9, dtype=torch.float64, device="cuda:0")
        mdx.compute_pme(ctx, t["pos"], t["force"], t["e_rec"], W)
        torch.cuda.synchronize()
        Wg = W.cpu().numpy().reshape(3, 3)
        E = float(t["e_rec"].cpu().numpy()[0])
        assert mdx.get_status(ctx) == 0
    ref = forcefield.pme_terms(s)
    assert abs(E - ref["E"]) <= E_TOL * abs(ref["E"])
    scale = np.abs(np.diag(ref["W"])).max()
    assert np.abs(Wg - ref["W"]).max() <= W_TOL * scale, (Wg, ref["W"])
    assert np.array_equal(Wg, Wg.T)


@pytest.mark.parametrize("n_mol", [12000, 14000], ids=["closing-kernel", "side-kernel"])
def test_pme_step_force_matches_fresh_evaluation(n_mol):
    # Water with PME on either side of the 40,000 atoms from which the PME
    # force gather and the bonded and exclusion terms run as a side kernel on
    # the second stream (below it the closing kernel evaluates them). After
    # steps that include a list rebuild, the force the step leaves equals a
    # fresh evaluation by the stand-alone kernels at the same positions.
    import torch
    L = (n_mol * 29.91) ** (1.0 / 3.0)
    s = synth.water_box(n_mol, L, (75, 75, 75) if n_mol > 12000 else (72, 72, 72), 9.0, None,
                        5e-4, 11, n_steps=100, name=f"water{3 * n_mol}")
    announce(f"PME step against a fresh evaluation: water N={s.n_atoms}")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.compute_pme(ctx, t["pos"], t["force"])
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], 12, float(s.dt))
        torch.cuda.synchronize()
        F_step = t["force"].cpu().numpy().astype(np.float64)
        f2 = torch.zeros_like(t["force"])
        mdx.compute_nonbonded(ctx, t["pos"], f2)
        mdx.compute_pme(ctx, t["pos"], f2)
        torch.cuda.synchronize()
        F_fresh = f2.cpu().numpy().astype(np.float64)
        assert mdx.get_status(ctx) == 0
        assert mdx.get_info(ctx).n_builds >= 2
    assert rel_rms(F_step, F_fresh) < 1e-6
