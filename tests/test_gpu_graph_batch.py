"""GPU: graph replay of mdx_integrate_step (mdx_set_graph), batched replicas in
one graph launch per chunk (mdx_batch_*), and the autotuner. Replays are
checked bit for bit against the launch-by-launch path, with the program's own
eager work and synchronisations between replays."""
import numpy as np
import pytest

import synth
from helpers import announce, gpu_context

pytestmark = pytest.mark.gpu


def _eager(s, steps, dt, **over):
    import torch
    with gpu_context(s, **over) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        if s.pme_grid[0]:
            mdx.compute_pme(ctx, t["pos"], t["force"])
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], steps, dt)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        return [t[k].cpu().numpy() for k in ("pos", "vel", "force")]


@pytest.mark.parametrize("name,rigid", [("water9k", False), ("lj1k", False), ("water375", True)])
def test_graph_replays_match_launch_by_launch(name, rigid):
    import math
    import torch
    s = synth.config_system(name)
    dt = float(s.dt)
    mols = None
    if rigid:
        from oracle import constraints
        w = synth.systems.WATER
        d_oh = w["bond_r0"]
        d_hh = 2.0 * d_oh * math.sin(math.radians(w["angle_theta0_deg"]) / 2.0)
        s.bond_k[:] = 0.0
        s.angle_k[:] = 0.0
        mols = np.arange(s.n_atoms, dtype=np.int32).reshape(-1, 3)
        s.vel = constraints.rattle_velocities(s.pos, s.vel, s.mass, s.box, mols).astype(np.float32)
        dt = 2.0
    announce(f"graph replay {name} rigid={rigid}")
    ref = {}
    for mode in ("eager", "graph"):
        with gpu_context(s) as (mdx, ctx, t):
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"])
            if s.pme_grid[0]:
                mdx.compute_pme(ctx, t["pos"], t["force"])
            if rigid:
                mdx.set_rigid_water(ctx, mols, d_oh, d_hh)
            args = (ctx, t["pos"], t["vel"], t["force"])
            snaps = []
            if mode == "graph":
                mdx.set_graph(ctx, 10)
            mdx.integrate_step(*args, 10, dt)                # graph: recorded, then launched
            torch.cuda.synchronize()
            snaps.append(t["pos"].cpu().numpy())
            assert mdx.get_status(ctx) == 0                   # eager work between replays
            mdx.integrate_step(*args, 20, dt)                # graph: two replays
            torch.cuda.synchronize()
            snaps.append(t["pos"].cpu().numpy())
            e = torch.zeros((5, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
            mdx.integrate_step(*args, 5, dt, e)              # launch by launch (energies)
            mdx.integrate_step(*args, 5, dt)                 # not a whole chunk: eager
            mdx.integrate_step(*args, 10, dt)                # the phase is back: replay
            torch.cuda.synchronize()
            assert mdx.get_status(ctx) == 0
            assert mdx.get_info(ctx).steps_taken == 50
            ref[mode] = snaps + [t[k].cpu().numpy() for k in ("pos", "vel", "force")]
    for a, b in zip(ref["eager"], ref["graph"]):
        assert np.array_equal(a, b)


def _small_batch():
    out = [synth.lj_fluid_n(n, 0.8, seed_stream=k) for k, n in enumerate((522, 1000, 2744))]
    for n_mol in (381, 700):
        L = (n_mol / synth.systems.WATER_MOLECULE_DENSITY) ** (1.0 / 3.0)
        K = synth.smooth_grid_size(int(np.ceil(L)))
        out.append(synth.water_box(n_mol, L, (K, K, K), 9.0, None, 5e-4, 3, o_jitter=0.05,
                                   name=f"w{n_mol}"))
    return out


def test_batch_matches_each_replica_alone():
    import torch
    import paper_2503_20541_amd as mdx
    systems = _small_batch()
    announce(f"batch of {len(systems)} replicas")
    ref = [_eager(s, 30, float(s.dt)) for s in systems]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    ctxs, keep, T = [], [], []
    try:
        for s in systems:
            desc, k = mdx.desc_from_system(s)
            keep.append(k)
            ctx = mdx.create(desc, stream)
            ctxs.append(ctx)
            t = dict(pos=torch.from_numpy(s.pos.copy()).to(dev),
                     vel=torch.from_numpy(s.vel.copy()).to(dev))
            t["force"] = torch.zeros_like(t["pos"])
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"])
            if s.pme_grid[0]:
                mdx.compute_pme(ctx, t["pos"], t["force"])
            T.append(t)
        b = mdx.batch_create(ctxs, 10)
        try:
            args = ([t["pos"] for t in T], [t["vel"] for t in T], [t["force"] for t in T])
            dts = [float(s.dt) for s in systems]
            mdx.batch_integrate(b, *args, 10, dts, stream)      # recorded, then launched
            torch.cuda.synchronize()
            for ctx in ctxs:
                assert mdx.get_status(ctx) == 0
            mdx.batch_integrate(b, *args, 20, dts, stream)      # two replays
            torch.cuda.synchronize()
        finally:
            mdx.batch_destroy(b)
        for ctx, t, r in zip(ctxs, T, ref):
            assert mdx.get_status(ctx) == 0
            for k, a in zip(("pos", "vel", "force"), r):
                assert np.array_equal(t[k].cpu().numpy(), a), k
    finally:
        torch.cuda.synchronize()
        for ctx in ctxs:
            mdx.destroy(ctx)


def test_autotune_picks_a_measured_configuration():
    import torch
    import paper_2503_20541_amd as mdx
    s = synth.config_system("water9k")
    desc, keep = mdx.desc_from_system(s)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(s.vel.copy()).to(dev)
    announce("autotune water9k")
    m, opt, ms = mdx.autotune(desc, pos, vel, float(s.dt), 10,
                              torch.cuda.current_stream(dev).cuda_stream)
    assert 1 <= m <= 4 and all(np.isfinite(ms)) and min(ms) > 0
    k = (4 if opt & mdx.MDX_OPT_COOPERATIVE_BUILD else 0) + m - 1
    assert ms[k] == min(ms)
    print("autotune water9k ms/step:", [round(v, 4) for v in ms], "->", m, opt, flush=True)
    # the inputs are untouched
    assert np.array_equal(pos.cpu().numpy(), s.pos)
